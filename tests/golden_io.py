"""Reader for the hand-worked fixtures under tests/golden/.

Each line is ``key value value ...``; values are numbers, fractions or
closed-form expressions built from + - * / ( ) and sqrt(). They are evaluated
with a tiny AST walker (no eval) in float64 (fractions exactly first).
"""
import ast
import math
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _ev(node):
    if isinstance(node, ast.Expression):
        return _ev(node.body)
    if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
        return Fraction(node.value)
    if isinstance(node, ast.UnaryOp) and isinstance(node.op, (ast.USub, ast.UAdd)):
        v = _ev(node.operand)
        return -v if isinstance(node.op, ast.USub) else v
    if isinstance(node, ast.BinOp):
        a, b = _ev(node.left), _ev(node.right)
        ops = {ast.Add: lambda: a + b, ast.Sub: lambda: a - b,
               ast.Mult: lambda: a * b, ast.Div: lambda: a / b}
        for k, f in ops.items():
            if isinstance(node.op, k):
                return f()
    if (isinstance(node, ast.Call) and isinstance(node.func, ast.Name)
            and node.func.id == "sqrt" and len(node.args) == 1):
        return math.sqrt(float(_ev(node.args[0])))
    raise ValueError("unsupported expression in golden file")


def value(text):
    return float(_ev(ast.parse(text, mode="eval")))


def load(name):
    """Return a dict: key -> list of rows (each a list of floats)."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out.setdefault(key, []).append([value(v) for v in vals])
    return out


def arr(d, key):
    return np.array(d[key], dtype=np.float64)
