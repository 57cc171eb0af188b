"""ctypes loader for the plain-C FP64 oracle (test infrastructure only).

``build()`` compiles ``oracle_cpu.c`` with gcc into ``liboracle_cpu.so`` next
to it; ``accel_pot`` and ``kdk`` call into it. The build uses IEEE double
arithmetic: no fast-math, no FMA contraction, generic x86-64 code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_cpu.c")
_LIB = os.path.join(_HERE, "liboracle_cpu.so")
_lib = None

CFLAGS = ["-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the C oracle; returns the path of the shared library."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_accel_pot.argtypes = [dp, dp, ctypes.c_int64, ip, ctypes.c_int64,
                                         ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_int]
        lib.oracle_accel_pot.restype = None
        lib.oracle_kdk.argtypes = [dp, dp, dp, dp, dp, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int]
        lib.oracle_kdk.restype = None
        lib.oracle_accel_jerk.argtypes = [dp, dp, dp, ctypes.c_int64, ip, ctypes.c_int64,
                                          ctypes.c_double, ctypes.c_double, dp, dp, dp, ctypes.c_int]
        lib.oracle_accel_jerk.restype = None
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def accel_pot(pos, mass, eps=0.0, G=1.0, targets=None, nthreads=0):
    """Same contract as ``oracle.oracle.accel_pot``, summed sequentially in C."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    if targets is None:
        tgt = None
        nt = n
    else:
        tgt = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tgt.shape[0]
        if nt and (tgt.min() < 0 or tgt.max() >= n):
            raise IndexError("target index out of range")
    acc = np.zeros((nt, 3))
    pot = np.zeros(nt)
    if nt == 0:
        return acc, pot
    lib.oracle_accel_pot(_dptr(pos), _dptr(mass), n,
                         None if tgt is None else tgt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         nt, float(eps), float(G), _dptr(acc), _dptr(pot), int(nthreads))
    return acc, pot


def kdk(pos, vel, mass, eps, G, dt, n_steps, acc=None, nthreads=0):
    """``n_steps`` KDK steps in C; returns ``(pos, vel, acc, pot)``."""
    lib = _load()
    pos = np.array(pos, dtype=np.float64, order="C")
    vel = np.array(vel, dtype=np.float64, order="C")
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    if acc is None:
        acc, pot = accel_pot(pos, mass, eps, G, nthreads=nthreads)
    else:
        acc = np.array(acc, dtype=np.float64, order="C")
        pot = np.zeros(n)
    lib.oracle_kdk(_dptr(pos), _dptr(vel), _dptr(acc), _dptr(pot), _dptr(mass), n,
                   float(eps), float(G), float(dt), int(n_steps), int(nthreads))
    return pos, vel, acc, pot


def accel_jerk(pos, vel, mass, eps=0.0, G=1.0, targets=None, nthreads=0):
    """Same contract as ``oracle.oracle.accel_jerk``, summed sequentially in C."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    if targets is None:
        tgt, nt = None, n
    else:
        tgt = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tgt.shape[0]
        if nt and (tgt.min() < 0 or tgt.max() >= n):
            raise IndexError("target index out of range")
    acc = np.zeros((nt, 3))
    jerk = np.zeros((nt, 3))
    pot = np.zeros(nt)
    if nt == 0:
        return acc, jerk, pot
    lib.oracle_accel_jerk(_dptr(pos), _dptr(vel), _dptr(mass), n,
                          None if tgt is None else tgt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                          nt, float(eps), float(G), _dptr(acc), _dptr(jerk), _dptr(pot), int(nthreads))
    return acc, jerk, pot
