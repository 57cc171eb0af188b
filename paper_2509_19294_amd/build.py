"""Build libnbody.so in-tree with hipcc for gfx950.

    python -m paper_2509_19294_amd.build

compiles ``csrc/kernels*.hip`` and ``csrc/abi.cpp`` into
``paper_2509_19294_amd/libnbody.so``. Packed FP32 instructions are disabled
for device code (``-packed-fp32-ops``); the FP32 pair loop therefore issues
one FP32 operation per lane per instruction.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libnbody.so")
ARCH = os.environ.get("NBODY_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
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


def build(verbose: bool = False, extra=()) -> str:
    """Compile the library (always; callers decide when). Returns its path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, f"-I{INCLUDE}", f"-I{CSRC}", *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed ({res.returncode})")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
