"""Host-side contract of libnbody.so, checked without a GPU.

The library must load, export every function include/nbody.h declares, and
reject every invalid argument with its status code before any launch (these
paths touch no device, so fake non-NULL pointers are safe: validation never
dereferences them).
"""
import ctypes
import math
import os
import re

import pytest

from paper_2509_19294_amd import nbody

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")
FAKE = ctypes.c_void_p(0x100000)        # never dereferenced by validation
FAKE2 = ctypes.c_void_p(0x900000)
FAKE3 = ctypes.c_void_p(0x1100000)


@pytest.fixture(scope="module")
def lib():
    # NBODY_LIB_UNDER_TEST: another build of the same library (the
    # sanitizer-instrumented one of tests/test_abi_asan_cpu.py)
    return nbody.load(os.environ.get("NBODY_LIB_UNDER_TEST", nbody.LIB_PATH))


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
    assert lib.nbody_version().decode().startswith("nbody")


def test_workspace_bytes(lib):
    assert lib.nbody_workspace_bytes(-1, 1, 0) == 0
    assert lib.nbody_workspace_bytes(10, 0, 0) == 0
    assert lib.nbody_workspace_bytes(10, 1, 5) == 0
    a = lib.nbody_workspace_bytes(1000, 1, 0)
    b = lib.nbody_workspace_bytes(1000, 1, 1)
    c = lib.nbody_workspace_bytes(2000, 1, 0)
    assert 0 < a < b and a < c
    assert a % 256 == 0 and b % 256 == 0
    # packed float4 + 8 split partials + pot + diag partials + counters
    assert a >= 1000 * 16 + 8 * 1000 * 16 + 1000 * 8 + 512 * 16 * 8
    assert lib.nbody_workspace_bytes(0, 1, 0) > 0


def _accel(lib, pos=FAKE, mass=FAKE2, n=100, eps=0.01, G=1.0, variant=0, acc=FAKE3, pot=None,
           ws=None, ws_bytes=None):
    if ws is None:
        ws = ctypes.c_void_p(0x7000000)
    if ws_bytes is None:
        ws_bytes = lib.nbody_workspace_bytes(max(n, 0), 1, variant if variant in (0, 1) else 0)
    return lib.nbody_accel(pos, mass, n, eps, G, variant, acc, pot, ws, ws_bytes, None)


@pytest.mark.parametrize("kw,code", [
    (dict(n=-1), nbody.EINVAL),
    (dict(variant=7), nbody.ENOTSUP),
    (dict(eps=-1e-3), nbody.EINVAL),
    (dict(eps=math.nan), nbody.EINVAL),
    (dict(eps=math.inf), nbody.EINVAL),
    (dict(G=math.inf), nbody.EINVAL),
    (dict(G=math.nan), nbody.EINVAL),
    (dict(pos=None), nbody.EINVAL),
    (dict(mass=None), nbody.EINVAL),
    (dict(acc=None), nbody.EINVAL),
    (dict(acc=FAKE), nbody.EINVAL),                     # output overlaps pos
    (dict(pot=ctypes.c_void_p(0x100000 + 8)), nbody.EINVAL),
    (dict(ws=ctypes.c_void_p(0)), nbody.EWORKSPACE),
    (dict(ws_bytes=100), nbody.EWORKSPACE),
])
def test_accel_rejects(lib, kw, code):
    assert _accel(lib, **kw) == code
    assert lib.nbody_last_error().decode() != ""


def test_accel_n0_is_noop(lib):
    assert _accel(lib, n=0, pos=None, mass=None, acc=None) == nbody.OK
    assert lib.nbody_last_error().decode() == ""


def _step(lib, n=64, n_steps=3, dt=0.01, eps=0.01, G=1.0, variant=0, plan=None, ws_bytes=None,
          pos=FAKE, vel=ctypes.c_void_p(0x200000), acc=ctypes.c_void_p(0x300000),
          mass=ctypes.c_void_p(0x400000), diag=None):
    if ws_bytes is None:
        ws_bytes = lib.nbody_workspace_bytes(n, 1, variant if variant in (0, 1) else 0)
    return lib.nbody_step(pos, vel, acc, None, mass, n, eps, G, dt, n_steps, variant, plan, diag,
                          ctypes.c_void_p(0x7000000), ws_bytes, None)


@pytest.mark.parametrize("kw,code", [
    (dict(n=-5), nbody.EINVAL),
    (dict(n_steps=-1), nbody.EINVAL),
    (dict(dt=math.nan), nbody.EINVAL),
    (dict(eps=-1.0), nbody.EINVAL),
    (dict(G=math.inf), nbody.EINVAL),
    (dict(variant=3), nbody.ENOTSUP),
    (dict(vel=None), nbody.EINVAL),
    (dict(vel=FAKE), nbody.EINVAL),           # vel overlaps pos
    (dict(diag=ctypes.c_void_p(0x200010)), nbody.EINVAL),  # diag overlaps vel
    (dict(ws_bytes=10), nbody.EWORKSPACE),
])
def test_step_rejects(lib, kw, code):
    assert _step(lib, **kw) == code


def test_step_zero_steps_is_noop(lib):
    assert _step(lib, n_steps=0) == nbody.OK


def _plan(lib, offsets, variant=1, tune_path=None):
    import numpy as np
    off = np.asarray(offsets, dtype=np.int64)
    return lib.nbody_plan_create(off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(off) - 1,
                                 variant, tune_path)


@pytest.mark.parametrize("offsets,variant", [
    ([1, 5], 1),            # offsets[0] != 0
    ([0, 5, 3], 1),         # decreasing
    ([0, 5], 9),            # unknown variant
    ([0, 2 ** 31], 1),      # too large for a batched plan
    ([0, 2 ** 31 - 20], 0),  # too large once every cluster is padded to 16 slots
])
def test_plan_create_rejects(lib, offsets, variant):
    assert not _plan(lib, offsets, variant)
    assert lib.nbody_last_error().decode() != ""


def test_plan_create_rejects_k0_and_null(lib):
    import numpy as np
    off = np.zeros(1, dtype=np.int64)
    assert not lib.nbody_plan_create(off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 0, 1, None)
    assert not lib.nbody_plan_create(None, 3, 1, None)
    assert "offsets" in lib.nbody_last_error().decode()


def test_plan_create_rejects_a_bad_tuning_file(lib, tmp_path):
    bad = tmp_path / "bad.txt"
    bad.write_text("batched 1 12 99\n")
    assert not _plan(lib, [0, 5, 9], 1, str(bad).encode())
    assert "bad batched entry" in lib.nbody_last_error().decode()
    assert not _plan(lib, [0, 5, 9], 1, str(tmp_path / "missing.txt").encode())


def test_plan_tuning_file_leaves_the_process_table_alone(lib, tmp_path):
    """A plan's tuning file must not retune later single-system calls: its
    single and jerk lines are checked but only its batched lines apply, and
    only to that plan. (Plan creation itself needs a GPU for its device
    arrays, so on the CPU the call fails after the file is read.)"""
    before = (nbody.tune_get("plain", 1 << 20), nbody.tune_get("comp", 5000),
              nbody.tune_jerk_get("comp", 1 << 16))
    f = tmp_path / "plan.txt"
    f.write_text("single 0 20 2 4\nsingle 1 12 3 2\njerk 1 16 4 2\nbatched 1 11 1\n")
    h = _plan(lib, [0, 5, 9], 1, str(f).encode())
    if h:
        lib.nbody_plan_destroy(h)
    after = (nbody.tune_get("plain", 1 << 20), nbody.tune_get("comp", 5000),
             nbody.tune_jerk_get("comp", 1 << 16))
    assert after == before


def test_batched_calls_reject_null_plan(lib):
    eps = ctypes.c_void_p(0x5000000)
    st = lib.nbody_accel_batched(FAKE, FAKE2, None, eps, 1.0, 1, FAKE3, None, FAKE, 1 << 20, None)
    assert st == nbody.EINVAL and "plan" in lib.nbody_last_error().decode()
    st = lib.nbody_step_batched(FAKE, ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000), None,
                                ctypes.c_void_p(0x400000), 64, None, eps, 1.0, 0.01, 3, 1, None,
                                ctypes.c_void_p(0x7000000), 1 << 20, None)
    assert st == nbody.EINVAL and "plan" in lib.nbody_last_error().decode()


def test_step_rejects_a_plan(lib):
    """nbody_step steps one system; a plan (whose clusters need per-cluster
    softenings) is refused before it is touched."""
    assert _step(lib, plan=ctypes.c_void_p(0x123400)) == nbody.EINVAL
    assert "nbody_step_batched" in lib.nbody_last_error().decode()


def test_tuning_table(lib, tmp_path):
    cfgs = nbody.tune_configs("plain")
    assert len(cfgs) == lib.nbody_tune_count(0) >= 5
    for block, k, ls, sw, tile, ib in cfgs:
        assert block % 64 == 0 and tile % block == 0 and tile % (ls * sw) == 0
        assert ib == (block // 64 // sw) * (64 // ls) * k
    modes = nbody.batched_modes()
    assert len(modes) >= 2
    # the near/far configurations exist for the compensated form only; the
    # half-group one covers 128 targets per block, the others whole groups
    comp = nbody.tune_configs("comp")
    assert len(comp) == len(cfgs) + 7
    for c in range(len(cfgs), len(comp)):
        assert comp[c][5] % 256 == 0 or c == len(comp) - 1
        with pytest.raises(nbody.NbodyError):
            nbody.tune_set("plain", 18, c, 1)
    assert comp[-1] == (256, 2, 1, 4, 256, 128)
    buf = (ctypes.c_int32 * 6)()
    assert lib.nbody_tune_describe(0, 999, buf) == nbody.EINVAL
    assert lib.nbody_tune_describe(5, 0, buf) == nbody.ENOTSUP
    # forcing and restoring a configuration
    before = nbody.tune_get("comp", 5000)
    nbody.tune_set("comp", 12, 3, 2)
    assert nbody.tune_get("comp", 5000) == (3, 2)
    nbody.tune_set("comp", 12, -1)
    assert nbody.tune_get("comp", 5000) == before
    assert lib.nbody_tune_set(0, 99, 0) == nbody.EINVAL
    assert lib.nbody_tune_set(0, 3, 55) == nbody.EINVAL
    # tuning files
    good = tmp_path / "t.txt"
    good.write_text("# kind variant class cfg split\nsingle 0 20 2 4\nbatched 1 11 1\n")
    nbody.tune_load(str(good))
    assert nbody.tune_get("plain", 1 << 20) == (2, 4)
    bad = tmp_path / "b.txt"
    bad.write_text("single 0 20 999 1\n")
    with pytest.raises(nbody.NbodyError):
        nbody.tune_load(str(bad))
    with pytest.raises(nbody.NbodyError):
        nbody.tune_load(str(tmp_path / "missing.txt"))
    nbody.tune_reset()
    assert nbody.tune_get("plain", 1 << 20) == nbody.tune_get("plain", (1 << 20) + 5)
    assert nbody.tune_get("comp", 5000) == before


def test_jerk_entry_points_validate(lib):
    n = 100
    wsb = lib.nbody_workspace_bytes_jerk(n, 1)
    assert wsb > lib.nbody_workspace_bytes_jerk(n, 0) > 0
    assert lib.nbody_workspace_bytes_jerk(-1, 0) == 0 and lib.nbody_workspace_bytes_jerk(5, 3) == 0
    pos, vel, mass = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    acc, jerk = ctypes.c_void_p(0x400000), ctypes.c_void_p(0x500000)
    ws = ctypes.c_void_p(0x7000000)
    ok = dict(pos=pos, vel=vel, mass=mass, n=n, eps=0.01, G=1.0, variant=1, acc=acc, jerk=jerk)

    def call(**kw):
        a = dict(ok, **kw)
        return lib.nbody_accel_jerk(a["pos"], a["vel"], a["mass"], a["n"], a["eps"], a["G"], a["variant"],
                                    a["acc"], a["jerk"], None, kw.get("ws", ws), kw.get("wsb", wsb), None)
    assert call(n=-1) == nbody.EINVAL
    assert call(variant=4) == nbody.ENOTSUP
    assert call(eps=-1.0) == nbody.EINVAL
    assert call(vel=None) == nbody.EINVAL
    assert call(jerk=acc) == nbody.EINVAL          # outputs overlap
    assert call(acc=vel) == nbody.EINVAL           # output overlaps an input
    assert call(wsb=16) == nbody.EWORKSPACE
    assert call(ws=ctypes.c_void_p(0x7000010)) == nbody.EWORKSPACE   # misaligned
    assert call(n=0, pos=None) == nbody.OK

    def step(**kw):
        a = {**ok, "dt": 0.01, "steps": 3, **kw}
        return lib.nbody_step_hermite(a["pos"], a["vel"], a["acc"], a["jerk"], None, a["mass"], a["n"], a["eps"],
                                      a["G"], a["dt"], a["steps"], a["variant"], kw.get("diag"), ws, wsb, None)
    assert step(steps=-1) == nbody.EINVAL
    assert step(dt=math.nan) == nbody.EINVAL
    assert step(jerk=vel) == nbody.EINVAL
    assert step(diag=ctypes.c_void_p(0x100008)) == nbody.EINVAL
    assert step(steps=0) == nbody.OK


def test_jerk_shapes_and_forcing(lib, tmp_path):
    shapes = nbody.jerk_shapes()
    assert len(shapes) == lib.nbody_tune_jerk_count(0) >= 4
    assert lib.nbody_tune_jerk_count(1) == len(shapes) + 3 and lib.nbody_tune_jerk_count(9) == 0
    assert lib.nbody_tune_jerk_set(0, 10) == nbody.EINVAL   # near/far shapes: compensated only
    assert lib.nbody_tune_jerk_set(1, 10) == nbody.OK
    assert lib.nbody_tune_jerk_set(1, -1) == nbody.OK
    for k, sw, ib in shapes:
        assert k in (1, 2, 4) and sw in (1, 2, 4) and ib == (4 // sw) * 64 * k
    buf = (ctypes.c_int32 * 3)()
    assert lib.nbody_tune_jerk_describe(lib.nbody_tune_jerk_count(1), buf) == nbody.EINVAL
    assert lib.nbody_tune_jerk_describe(0, None) == nbody.EINVAL
    assert lib.nbody_tune_jerk_set(0, len(shapes)) == nbody.EINVAL
    assert lib.nbody_tune_jerk_set(0, 33 * 1000) == nbody.EINVAL
    assert lib.nbody_tune_jerk_set(7, 0) == nbody.ENOTSUP
    assert lib.nbody_tune_jerk_get(0, -1) == -1
    n = 65536
    before = nbody.tune_jerk_get("plain", n)
    assert before[1] >= 1
    # a forced split resizes the workspace the next call needs
    nbody.tune_jerk_set("plain", 0, 1)
    assert nbody.tune_jerk_get("plain", n) == (0, 1)
    small = lib.nbody_workspace_bytes_jerk(n, 0)
    nbody.tune_jerk_set("plain", 0, 16)
    assert nbody.tune_jerk_get("plain", n) == (0, 16)
    assert lib.nbody_workspace_bytes_jerk(n, 0) == small + 16 * n * 2 * 16
    # split 0 = the built-in rule; the partial buffer bound caps any split
    nbody.tune_jerk_set("plain", 3, 0)
    assert nbody.tune_jerk_get("plain", n)[0] == 3 and nbody.tune_jerk_get("plain", n)[1] >= 1
    nbody.tune_jerk_set("plain", 0, 32)
    assert nbody.tune_jerk_get("plain", 1 << 20) == (0, 8)
    nbody.tune_jerk_set("plain", -1)
    assert nbody.tune_jerk_get("plain", n) == before
    # tuning files carry jerk lines; reset restores the table
    f = tmp_path / "j.txt"
    f.write_text("jerk 1 16 4 2\n")
    nbody.tune_load(str(f))
    assert nbody.tune_jerk_get("comp", n) == (4, 2)
    bad = tmp_path / "jb.txt"
    bad.write_text("jerk 1 16 99 2\n")
    with pytest.raises(nbody.NbodyError):
        nbody.tune_load(str(bad))
    nbody.tune_jerk_set("comp", 2, 4)
    nbody.tune_reset()
    assert nbody.tune_jerk_get("comp", n) != (2, 4) and nbody.tune_jerk_get("comp", n) != (4, 2)


def test_noalloc_validates_before_touching_a_device(lib):
    """nbody_accel_noalloc checks its arguments and its size limit on the
    host, before it looks up its scratch on a device."""
    def call(n=100, eps=0.01, variant=0, pos=FAKE, acc=FAKE3):
        return lib.nbody_accel_noalloc(pos, FAKE2, n, eps, 1.0, variant, acc, None, None)
    assert call(n=-1) == nbody.EINVAL
    assert call(variant=3) == nbody.ENOTSUP
    assert call(eps=math.nan) == nbody.EINVAL
    assert call(pos=None) == nbody.EINVAL
    assert call(acc=FAKE) == nbody.EINVAL
    assert call(n=0, pos=None, acc=None) == nbody.OK
    # the static scratch holds at most 1,676,064 (plain) / 536,480 (compensated)
    # particles: one more is refused on the host; the limit itself passes the
    # host checks and only then looks for a device (none here: EHIP)
    far = [ctypes.c_void_p(k << 36) for k in (1, 2, 3)]
    for n, variant in ((1676064, 0), (536480, 1)):
        assert call(n=n + 1, variant=variant, pos=far[0], acc=far[2]) == nbody.EINVAL
        assert "scratch" in lib.nbody_last_error().decode()
        st = lib.nbody_accel_noalloc(far[0], far[1], n, 0.01, 1.0, variant, far[2], None, None)
        assert st in (nbody.OK, nbody.EHIP) and "workspace" not in lib.nbody_last_error().decode()


def test_tuning_file_from_the_environment(tmp_path):
    """NBODY_TUNE names a tuning file read when the table is first used (and
    again by nbody_tune_reset); a file that does not parse leaves the built-in
    table. Run in fresh processes, since the table is process-wide."""
    import subprocess
    import sys

    good = tmp_path / "t.txt"
    good.write_text("single 0 20 2 4\njerk 1 18 3 2\n")
    bad = tmp_path / "b.txt"
    bad.write_text("single 0 20 999 1\n")
    code = ("import sys; sys.path.insert(0, %r); from paper_2509_19294_amd import nbody; "
            "print(nbody.tune_get('plain', 1 << 20), nbody.tune_jerk_get('comp', 1 << 18)); "
            "nbody.tune_reset(); print(nbody.tune_get('plain', 1 << 20))" % ROOT)

    def run(path):
        env = dict(os.environ)
        env.pop("NBODY_TUNE", None)
        if path is not None:
            env["NBODY_TUNE"] = str(path)
        if "NBODY_LIB_UNDER_TEST" in env:
            env.pop("NBODY_LIB_UNDER_TEST")
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                             timeout=120, cwd=ROOT)
        assert out.returncode == 0, out.stderr[-2000:]
        return out.stdout.split("\n")

    default = run(None)
    lines = run(good)
    assert lines[0] == "(2, 4) (3, 2)" and lines[1] == "(2, 4)"
    assert run(bad) == default and default[0] != lines[0]
