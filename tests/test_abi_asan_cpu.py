"""The host-side contract tests (tests/test_abi_cpu.py) rerun against a build
of the library whose host code is instrumented by AddressSanitizer: every
validation path of the C ABI runs under it and must report no invalid
access. Device code is built as usual (the sanitizer applies to host code
only); the kernels' objects are shared with the normal build."""
import glob
import os
import subprocess
import sys

import pytest

from paper_2509_19294_amd import build as nbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.slow
def test_abi_contract_under_host_asan(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime under /opt/rocm/llvm")
    host_srcs = [s for s in nbuild.sources() if os.path.basename(s) in ("abi.cpp", "noalloc.hip")]
    kernel_srcs = [s for s in nbuild.sources() if s not in host_srcs]
    kernel_objs = [os.path.join(nbuild.OBJ_DIR, os.path.basename(s) + ".o") for s in kernel_srcs]
    if not all(os.path.exists(o) for o in kernel_objs):
        kernel_objs = nbuild.compile_objects(kernel_srcs)
    asan_objs = nbuild.compile_objects(host_srcs, obj_dir=str(tmp_path / "obj"), extra=HOST_ASAN)
    lib = nbuild.link(kernel_objs + asan_objs, str(tmp_path / "libnbody_asan.so"),
                      extra=["-Xarch_host", "-fsanitize=address", "-shared-libasan"])
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_report_load" in syms, "the host code is not instrumented"
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               NBODY_LIB_UNDER_TEST=lib, PYTHONPATH=ROOT)
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
    assert "passed" in out
