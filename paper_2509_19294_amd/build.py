"""Build libnbody.so in-tree with hipcc for gfx950.

    python -m paper_2509_19294_amd.build

compiles ``csrc/kernels*.hip``, ``csrc/noalloc.hip`` and ``csrc/abi.cpp``
to objects (in parallel, under ``_build/``) and links them into
``paper_2509_19294_amd/libnbody.so``. Packed FP32 instructions are disabled
for device code (``-packed-fp32-ops``); the FP32 pair loop therefore issues
one FP32 operation per lane per instruction.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libnbody.so")
OBJ_DIR = os.path.join(ROOT, "_build")
ARCH = os.environ.get("NBODY_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return [os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "kernels_jerk.hip"),
            os.path.join(CSRC, "kernels_order.hip"), os.path.join(CSRC, "kernels_nf.hip"),
            os.path.join(CSRC, "kernels_nf_jerk.hip"), os.path.join(CSRC, "noalloc.hip"),
            os.path.join(CSRC, "abi.cpp")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed ({res.returncode}): {cmd[-1]}")


def compile_objects(srcs, obj_dir=OBJ_DIR, extra=(), verbose=False, jobs=None):
    """Compile ``srcs`` to ``obj_dir/<name>.o`` in parallel; returns the
    object paths in the order of ``srcs``."""
    os.makedirs(obj_dir, exist_ok=True)
    objs = [os.path.join(obj_dir, os.path.basename(src) + ".o") for src in srcs]
    cmds = [[hipcc(), *HIPCC_FLAGS, *extra, f"-I{INCLUDE}", f"-I{CSRC}", "-c", src, "-o", obj]
            for src, obj in zip(srcs, objs)]
    jobs = jobs or min(len(cmds), max(1, min(os.cpu_count() or 1, 16)))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        list(pool.map(lambda c: _run(c, verbose), cmds))
    return objs


def link(objs, out, extra=(), verbose=False):
    tmp = out + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, *objs, "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, extra=()) -> str:
    """Compile the library (always; callers decide when). Returns its path."""
    objs = compile_objects(sources(), extra=extra, verbose=verbose)
    return link(objs, LIB, verbose=verbose)


if __name__ == "__main__":
    print(build(verbose=True))
