"""GPU parity of the acceleration + jerk kernel and the Hermite integrator
against the FP64 oracle (through the C ABI).

Tolerances: accelerations, jerks and potentials within rel-RMS 1e-5 and
accelerations within 1e-4 per particle, against the oracle evaluated on the
inputs each form actually represents: the compensated form carries
separations and relative velocities to ~2^-24 of their own size, so its
reference is the oracle on the FP64 inputs; the plain form rounds absolute
positions, masses and the velocities relative to particle 0's to FP32
first, so its reference is the oracle on those rounded inputs (the rounding
alone moves an unsoftened close pair by ~2^-24 |x| / r, which can exceed
1e-5 on its own). Against the
oracle on the exact inputs both forms must meet the paper's criterion
(Section 3): every jerk component within 0.2 % of a typical jerk magnitude,
read as the RMS of |jerk|.
"""
import math

import numpy as np
import pytest
import torch

from oracle import cpu as ocpu
from oracle import oracle as orc
from paper_2509_19294_amd import ics, nbody
from tests import golden_io

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _setup():
    ocpu.build(force=False)
    nbody.load()
    nbody.tune_reset()
    yield
    nbody.tune_reset()


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def gpu_accel_jerk(pos, vel, mass, eps, variant, G=1.0):
    a, j, p = nbody.accel_jerk(T(pos), T(vel), T(mass), eps, G, variant)
    torch.cuda.synchronize()
    return a.cpu().numpy(), j.cpu().numpy(), p.cpu().numpy()


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def references(pos, vel, mass, eps, variant, accel_jerk=orc.accel_jerk):
    """(exact, form) oracle results: on the FP64 inputs, and on the inputs
    the form represents (FP32-rounded for the plain form)."""
    exact = accel_jerk(pos, vel, mass, eps)
    if variant == "comp":
        return exact, exact
    v0 = np.asarray(vel, dtype=np.float64)[0]
    return exact, accel_jerk(f32(pos), v0 + f32(vel - v0), f32(mass), eps)


def check(got, refs, what=""):
    a, j, p = got
    (ea, ej, ep), (ra, rj, rp) = refs
    e = (orc.rel_rms(a, ra), orc.rel_rms(j, rj), orc.paper_metric(j, ej))
    print(what, "acc rel-rms", e[0], "jerk rel-rms", e[1], "jerk paper metric (exact inputs)", e[2],
          "| against the exact inputs: acc rel-rms", orc.rel_rms(a, ea), "jerk rel-rms", orc.rel_rms(j, ej),
          "acc paper metric", orc.paper_metric(a, ea))
    assert orc.rel_rms(a, ra) <= 1e-5, (what, "acc", orc.rel_rms(a, ra))
    assert orc.max_rel(a, ra) <= 1e-4, (what, "acc max", orc.max_rel(a, ra))
    assert orc.rel_rms(p, rp) <= 1e-5, (what, "pot", orc.rel_rms(p, rp))
    assert orc.rel_rms(j, rj) <= 1e-5, (what, "jerk", orc.rel_rms(j, rj))
    assert orc.paper_metric(j, ej) <= 2e-3, (what, "jerk paper metric", orc.paper_metric(j, ej))
    assert orc.paper_metric(a, ea) <= 5e-4, (what, "acc paper metric", orc.paper_metric(a, ea))
    return e


@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_three_body_hand_worked(variant):
    g = golden_io.load("three_body_eps0.txt")
    pos, vel, mass = golden_io.arr(g, "pos"), golden_io.arr(g, "vel"), golden_io.arr(g, "mass")[0]
    a, j, p = gpu_accel_jerk(pos, vel, mass, 0.0, variant)
    np.testing.assert_allclose(a, golden_io.arr(g, "acc"), rtol=2e-6, atol=2e-7)
    np.testing.assert_allclose(j, golden_io.arr(g, "jerk"), rtol=2e-6, atol=2e-7)
    np.testing.assert_allclose(p, golden_io.arr(g, "pot")[0], rtol=2e-6)


@pytest.mark.parametrize("variant", ["plain", "comp"])
@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 129, 257, 1000, 4099])
@pytest.mark.parametrize("eps", [0.01, 0.0])
def test_sizes(variant, n, eps):
    pos, vel, mass = ics.plummer(n, seed=200 + n)
    a, j, p = gpu_accel_jerk(pos, vel, mass, eps, variant)
    if n == 1:
        assert np.all(a == 0) and np.all(j == 0) and np.all(p == 0)
        return
    check((a, j, p), references(pos, vel, mass, eps, variant), (variant, n, eps))
    a2, j2, p2 = gpu_accel_jerk(pos, vel, mass, eps, variant)
    assert np.array_equal(a, a2) and np.array_equal(j, j2) and np.array_equal(p, p2)


@pytest.mark.parametrize("variant", ["plain", "comp"])
@pytest.mark.parametrize("eps", [0.01, 0.0])
def test_every_shape_and_split(variant, eps):
    """Every compiled kernel shape, with and without a grid j-split, on a
    ragged size; each result is bitwise reproducible."""
    n = 3001
    pos, vel, mass = ics.plummer(n, seed=77)
    refs = references(pos, vel, mass, eps, variant)
    try:
        for cfg in range(len(nbody.jerk_shapes(variant))):
            for split in (1, 3, 4):
                nbody.tune_jerk_set(variant, cfg, split)
                assert nbody.tune_jerk_get(variant, n) == (cfg, split)
                got = gpu_accel_jerk(pos, vel, mass, eps, variant)
                check(got, refs, (variant, eps, cfg, split))
                again = gpu_accel_jerk(pos, vel, mass, eps, variant)
                assert all(np.array_equal(x, y) for x, y in zip(got, again)), (cfg, split)
    finally:
        nbody.tune_jerk_set(variant, -1)


@pytest.mark.parametrize("cfg", [10, 11, 12])
def test_near_far_shapes(cfg):
    """Near/far shapes (compensated form): tiny and ragged sizes, eps 0,
    a translated and boosted system, a permuted input, bitwise
    reproducibility and the full oracle at N = 65,536."""
    try:
        for n, eps in ((1, 0.01), (2, 0.0), (257, 0.01), (3001, 0.0), (3001, 0.01)):
            pos, vel, mass = ics.plummer(n, seed=500 + n)
            nbody.tune_jerk_set("comp", cfg, 2)
            got = gpu_accel_jerk(pos, vel, mass, eps, "comp")
            if n == 1:
                assert all(np.all(x == 0) for x in got)
                continue
            check(got, references(pos, vel, mass, eps, "comp"), (cfg, n, eps))
            again = gpu_accel_jerk(pos, vel, mass, eps, "comp")
            assert all(np.array_equal(x, y) for x, y in zip(got, again))
        pos, vel, mass = ics.plummer(4000, seed=61)
        refs = references(pos, vel, mass, 0.01, "comp")
        got = gpu_accel_jerk(pos + np.array([1e4, -2e3, 5e2]), vel + np.array([30.0, 0.0, -7.0]), mass, 0.01, "comp")
        check(got, refs, (cfg, "boosted"))
        perm = np.random.default_rng(3).permutation(4000)
        got = gpu_accel_jerk(pos[perm], vel[perm], mass[perm], 0.01, "comp")
        check(got, tuple(tuple(x[perm] for x in r) for r in refs), (cfg, "permuted"))
        pos, vel, mass, spec = ics.workload("plummer_64k")
        nbody.tune_jerk_set("comp", cfg, 16)
        got = gpu_accel_jerk(pos, vel, mass, spec["eps"], "comp")
        e = check(got, references(pos, vel, mass, spec["eps"], "comp", ocpu.accel_jerk), (cfg, "64k"))
        print(f"near/far jerk shape {cfg} N=65536: acc {e[0]:.3e} jerk {e[1]:.3e} paper {e[2]:.3e}")
    finally:
        nbody.tune_jerk_set("comp", -1)


def test_hermite_with_near_far_shape():
    pos, vel, mass, spec = ics.workload("plummer_1k")
    eps, dt, steps = spec["eps"], spec["dt"], spec["steps"]
    pr, vr, _, _, _, rows = orc.hermite(pos, vel, mass, eps, 1.0, dt, steps)
    nbody.tune_jerk_set("comp", 11, 2)
    try:
        tp, tv, tm = T(pos), T(vel), T(mass)
        acc, jerk, _ = nbody.accel_jerk(tp, tv, tm, eps, 1.0, "comp")
        diag = nbody.step_hermite(tp, tv, acc, jerk, tm, eps, 1.0, dt, steps, "comp")
        torch.cuda.synchronize()
    finally:
        nbody.tune_jerk_set("comp", -1)
    assert np.abs(tp.cpu().numpy() - pr).max() < 1e-7
    np.testing.assert_allclose(diag.cpu().numpy()[:, 2], rows[1:, 2], rtol=1e-5)


def test_jerk_boosted_frame_plain():
    """A Galilean boost of 30-60 velocity dispersions: the plain form takes
    velocities relative to particle 0's, so neither their rounding nor the
    split J1 sum (sum s v_j - v_i sum s) grows with the bulk velocity; the
    result equals the unboosted one's tolerance-wise."""
    pos, vel, mass = ics.plummer(3001, seed=19)
    boost = np.array([30.0, -15.0, 6.0])
    got = gpu_accel_jerk(pos, vel + boost, mass, 0.01, "plain")
    check(got, references(pos, vel + boost, mass, 0.01, "plain"), "boosted plain")
    ref = orc.accel_jerk(pos, vel, mass, 0.01)
    assert orc.rel_rms(got[1], ref[1]) <= 1e-5


def test_jerk_boosted_and_shifted_frame():
    """A Galilean boost and a shift: the compensated form (positions and
    velocities relative to particle 0) keeps the tolerance."""
    pos, vel, mass = ics.plummer(3000, seed=9)
    got = gpu_accel_jerk(pos + np.array([500.0, -300.0, 100.0]), vel + np.array([50.0, 0.0, -20.0]),
                         mass, 0.01, "comp")
    check(got, references(pos, vel, mass, 0.01, "comp"), "boosted")


@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_plummer_64k_full_oracle(variant):
    pos, vel, mass, spec = ics.workload("plummer_64k")
    got = gpu_accel_jerk(pos, vel, mass, spec["eps"], variant)
    e = check(got, references(pos, vel, mass, spec["eps"], variant, ocpu.accel_jerk), variant)
    print(f"plummer_64k jerk {variant}: acc rel-rms {e[0]:.3e} jerk rel-rms {e[1]:.3e} paper metric {e[2]:.3e}")


@pytest.mark.parametrize("workload,variant", [("plummer_256k", "plain"), ("plummer_256k", "comp"),
                                              ("kroupa_1m", "comp")])
def test_large_subsample(workload, variant):
    """N = 262,144 (eps = 0.002) and N = 1,048,576 with Kroupa masses
    (eps = 0.001), in the tuned launch (the compensated form's near/far
    shapes, the plain form's split J1 sum): 4096 strided targets against all
    sources in the C oracle."""
    pos, vel, mass, spec = ics.workload(workload)
    eps = spec["eps"]
    tgt = orc.subsample_targets(len(mass), 4096)
    got = tuple(x[tgt] for x in gpu_accel_jerk(pos, vel, mass, eps, variant))
    exact = ocpu.accel_jerk(pos, vel, mass, eps, targets=tgt)
    if variant == "comp":
        form = exact
    else:
        v0 = vel[0]
        form = ocpu.accel_jerk(f32(pos), v0 + f32(vel - v0), f32(mass), eps, targets=tgt)
    e = check(got, (exact, form), (workload, variant))
    print(f"{workload} {variant}: acc {e[0]:.3e} jerk {e[1]:.3e} jerk paper metric {e[2]:.3e}")


@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_hermite_plummer_1k(variant):
    pos, vel, mass, spec = ics.workload("plummer_1k")
    eps, dt, steps = spec["eps"], spec["dt"], spec["steps"]
    pr, vr, ar, jr, _, rows = orc.hermite(pos, vel, mass, eps, 1.0, dt, steps)
    tp, tv, tm = T(pos), T(vel), T(mass)
    acc, jerk, _ = nbody.accel_jerk(tp, tv, tm, eps, 1.0, variant)
    diag = nbody.step_hermite(tp, tv, acc, jerk, tm, eps, 1.0, dt, steps, variant)
    torch.cuda.synchronize()
    assert np.abs(tp.cpu().numpy() - pr).max() < 1e-7
    assert np.abs(tv.cpu().numpy() - vr).max() < 1e-6
    assert orc.rel_rms(acc.cpu().numpy(), ar) < 1e-5
    assert orc.rel_rms(jerk.cpu().numpy(), jr) < 1e-4
    d = diag.cpu().numpy()
    np.testing.assert_allclose(d[:, 0], rows[1:, 0], rtol=1e-8)
    np.testing.assert_allclose(d[:, 2], rows[1:, 2], rtol=1e-5)
    np.testing.assert_array_equal(d[:, 14], np.arange(1, steps + 1))


def test_hermite_kepler_eps0():
    m1, m2, e, s = 0.3, 0.7, 0.5, 1.0
    mu = m1 + m2
    rp = s * (1 - e)
    vp = math.sqrt(mu * (1 + e) / rp)
    pos = np.array([[-m2 / mu * rp, 0, 0], [m1 / mu * rp, 0, 0]])
    vel = np.array([[0, -m2 / mu * vp, 0], [0, m1 / mu * vp, 0]])
    mass = np.array([m1, m2])
    steps = 500
    dt = 2 * math.pi / steps
    pr, _, _, _, _, rows = orc.hermite(pos, vel, mass, 0.0, 1.0, dt, steps)
    tp, tv, tm = T(pos), T(vel), T(mass)
    acc, jerk, _ = nbody.accel_jerk(tp, tv, tm, 0.0, 1.0, "comp")
    diag = nbody.step_hermite(tp, tv, acc, jerk, tm, 0.0, 1.0, dt, steps, "comp")
    torch.cuda.synchronize()
    assert np.abs(tp.cpu().numpy() - pr).max() < 1e-5
    drift = np.abs(diag.cpu().numpy()[:, 2] - rows[0, 2]) / abs(rows[0, 2])
    assert drift.max() < 1e-4


def test_hermite_split_equals_straight_run():
    pos, vel, mass = ics.plummer(2000, seed=31)
    outs = []
    for split in ((4,), (1, 3)):
        tp, tv, tm = T(pos), T(vel), T(mass)
        acc, jerk, _ = nbody.accel_jerk(tp, tv, tm, 0.01, 1.0, "comp")
        for k in split:
            nbody.step_hermite(tp, tv, acc, jerk, tm, 0.01, 1.0, 1.0 / 128, k, "comp", diag=False)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in (tp, tv, acc, jerk)])
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)
