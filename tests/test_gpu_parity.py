"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: relative RMS error of the accelerations <= 1e-5 and largest
relative error of a single acceleration vector <= 1e-4 (the same bounds for
the potentials' RMS); the paper's own criterion (largest component error
below 5e-4 of a typical magnitude) is implied by these and checked too.
Index work (which particle lands where, which clusters interact) must be
exact; run-to-run results must be bitwise identical for a fixed tuning.
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

RMS_TOL = 1e-5
MAX_TOL = 1e-4
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


def gpu_accel(pos, mass, eps, variant, G=1.0):
    acc, pot = nbody.accel(T(pos), T(mass), eps, G, variant)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), pot.cpu().numpy()


def check(a, p, ref_a, ref_p, rms=RMS_TOL, mx=MAX_TOL, what=""):
    e1, e2, e3 = orc.rel_rms(a, ref_a), orc.max_rel(a, ref_a), orc.rel_rms(p, ref_p)
    assert e1 <= rms, (what, "acc rel-rms", e1)
    assert e2 <= mx, (what, "acc max-rel", e2)
    assert e3 <= rms, (what, "pot rel-rms", e3)
    assert orc.paper_metric(a, ref_a) <= 5e-4, (what, "paper metric")
    return e1, e2, e3


@pytest.mark.parametrize("variant", ["plain", "comp"])
@pytest.mark.parametrize("name", ["three_body_eps0.txt", "three_body_eps1.txt"])
def test_three_body_hand_worked(variant, name):
    g = golden_io.load(name)
    pos, mass, eps = golden_io.arr(g, "pos"), golden_io.arr(g, "mass")[0], g["eps"][0][0]
    a, p = gpu_accel(pos, mass, eps, variant)
    np.testing.assert_allclose(a, golden_io.arr(g, "acc"), rtol=2e-6, atol=2e-7)
    np.testing.assert_allclose(p, golden_io.arr(g, "pot")[0], rtol=2e-6)


@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_single_particle_and_empty(variant):
    a, p = gpu_accel(np.array([[0.3, -1.0, 2.0]]), np.array([0.7]), 0.1, variant)
    assert np.all(a == 0.0) and np.all(p == 0.0)
    a, p = gpu_accel(np.array([[0.3, -1.0, 2.0]]), np.array([0.7]), 0.0, variant)
    assert np.all(a == 0.0) and np.all(p == 0.0)
    acc, pot = nbody.accel(torch.zeros((0, 3), dtype=torch.float64, device=DEV),
                           torch.zeros(0, dtype=torch.float64, device=DEV), 0.1, 1.0, variant)
    assert acc.shape == (0, 3)


@pytest.mark.parametrize("variant", ["plain", "comp"])
@pytest.mark.parametrize("n", [2, 3, 31, 32, 33, 63, 64, 65, 255, 256, 257, 1000, 1024, 1025, 4099])
@pytest.mark.parametrize("eps", [0.01, 0.0])
def test_tile_boundaries(variant, n, eps):
    pos, _, mass = ics.plummer(n, seed=n)
    ref_a, ref_p = orc.accel_pot(pos, mass, eps)
    a, p = gpu_accel(pos, mass, eps, variant)
    check(a, p, ref_a, ref_p, what=(variant, n, eps))


@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_uneven_masses_and_G(variant):
    rng = np.random.default_rng(5)
    n = 777
    pos = rng.normal(size=(n, 3))
    mass = rng.uniform(0.0, 3.0, size=n)
    mass[::7] = 0.0
    ref_a, ref_p = orc.accel_pot(pos, mass, 0.05, 2.5)
    a, p = gpu_accel(pos, mass, 0.05, variant, G=2.5)
    check(a, p, ref_a, ref_p)


@pytest.mark.parametrize("variant", ["plain", "comp"])
@pytest.mark.parametrize("n", [1000, 3001])
def test_every_config_matches_oracle_and_is_deterministic(variant, n):
    pos, _, mass = ics.plummer(n, seed=77)
    ref_a, ref_p = orc.accel_pot(pos, mass, 0.01)
    cls = int(math.floor(math.log2(n)))
    results = []
    try:
        for cfg in range(len(nbody.tune_configs(variant))):
            for split in (1, 3, 8):
                nbody.tune_set(variant, cls, cfg, split)
                a1, p1 = gpu_accel(pos, mass, 0.01, variant)
                a2, p2 = gpu_accel(pos, mass, 0.01, variant)
                assert np.array_equal(a1, a2) and np.array_equal(p1, p2), (cfg, split)
                check(a1, p1, ref_a, ref_p, what=(variant, n, cfg, split))
                results.append(a1)
    finally:
        nbody.tune_set(variant, cls, -1)
    # Different tilings agree with each other far inside the tolerance.
    for r in results[1:]:
        assert orc.rel_rms(r, results[0]) < 2e-6


def test_every_config_compensated_survives_translation():
    """Every compiled configuration of the compensated form keeps the
    tolerance on a sphere shifted by 10^3 (each form's frame handling)."""
    n = 3001
    pos, _, mass = ics.plummer(n, seed=78)
    ref_a, ref_p = orc.accel_pot(pos, mass, 0.01)
    shifted = pos + np.array([-1000.0, 700.0, 1000.0])
    cls = int(math.floor(math.log2(n)))
    try:
        for cfg in range(len(nbody.tune_configs("comp"))):
            for split in (1, 4):
                nbody.tune_set("comp", cls, cfg, split)
                a, p = gpu_accel(shifted, mass, 0.01, "comp")
                check(a, p, ref_a, ref_p, what=("shifted", cfg, split))
    finally:
        nbody.tune_set("comp", cls, -1)


def test_permutation_moves_rows_exactly():
    n = 2048
    pos, _, mass = ics.plummer(n, seed=3)
    perm = np.random.default_rng(1).permutation(n)
    a0, p0 = gpu_accel(pos, mass, 0.01, "comp")
    a1, p1 = gpu_accel(pos[perm], mass[perm], 0.01, "comp")
    assert orc.rel_rms(a1, a0[perm]) < 2e-6
    ref_a, _ = orc.accel_pot(pos, mass, 0.01)
    assert orc.rel_rms(a1, ref_a[perm]) < RMS_TOL


def test_translation_purpose_of_compensated_form():
    """Shift a sphere by 10^3: the plain form loses ~3 decimal digits in
    the separations, the compensated form (coordinates relative to a block
    frame, double-single) keeps the tolerance."""
    n = 4096
    pos, _, mass = ics.plummer(n, seed=8)
    shifted = pos + np.array([1000.0, -1000.0, 500.0])
    ref_a, ref_p = orc.accel_pot(pos, mass, 0.005)
    ac, pc = gpu_accel(shifted, mass, 0.005, "comp")
    ap, pp = gpu_accel(shifted, mass, 0.005, "plain")
    err_c = orc.rel_rms(ac, ref_a)
    err_p = orc.rel_rms(ap, ref_a)
    assert err_c <= RMS_TOL and orc.max_rel(ac, ref_a) <= MAX_TOL
    assert err_p > 30 * err_c


@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_plummer_64k_full_oracle(variant):
    """N = 65,536 equal-mass Plummer sphere (seed 1), eps = 0.005: every
    particle against the full N^2 FP64 oracle."""
    pos, _, mass, spec = ics.workload("plummer_64k")
    ref_a, ref_p = ocpu.accel_pot(pos, mass, spec["eps"])
    a, p = gpu_accel(pos, mass, spec["eps"], variant)
    e = check(a, p, ref_a, ref_p, what=variant)
    print(f"plummer_64k {variant}: acc rel-rms {e[0]:.3e} max-rel {e[1]:.3e} pot rel-rms {e[2]:.3e}")


@pytest.mark.parametrize("variant", ["comp", "plain"])
def test_plummer_256k_subsample(variant):
    """N = 262,144 Plummer sphere, eps = 0.002: 4096 strided targets against
    all sources."""
    pos, _, mass, spec = ics.workload("plummer_256k")
    tgt = orc.subsample_targets(len(mass), 4096)
    ref_a, ref_p = ocpu.accel_pot(pos, mass, spec["eps"], targets=tgt)
    a, p = gpu_accel(pos, mass, spec["eps"], variant)
    e = check(a[tgt], p[tgt], ref_a, ref_p, what=variant)
    print(f"plummer_256k {variant}: acc rel-rms {e[0]:.3e} max-rel {e[1]:.3e} pot rel-rms {e[2]:.3e}")


def test_kroupa_1m_subsample():
    """N = 1,048,576 Plummer sphere with Kroupa masses, eps = 0.001,
    compensated form: 4096 strided targets against all sources."""
    pos, _, mass, spec = ics.workload("kroupa_1m")
    tgt = orc.subsample_targets(len(mass), 4096)
    ref_a, ref_p = ocpu.accel_pot(pos, mass, spec["eps"], targets=tgt)
    a, p = gpu_accel(pos, mass, spec["eps"], "comp")
    e = check(a[tgt], p[tgt], ref_a, ref_p)
    print(f"kroupa_1m comp: acc rel-rms {e[0]:.3e} max-rel {e[1]:.3e} pot rel-rms {e[2]:.3e}")


# ---- integrator -------------------------------------------------------------

@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_kdk_plummer_1k_ten_steps(variant):
    """N = 1,024 Plummer sphere (seed 0), eps = 0.01, 10 KDK steps at
    dt = 1/128: trajectories, final forces and every diagnostics row against
    the FP64 oracle run."""
    pos, vel, mass, spec = ics.workload("plummer_1k")
    eps, dt, steps = spec["eps"], spec["dt"], spec["steps"]
    p_ref, v_ref, a_ref, pot_ref, rows = orc.kdk(pos, vel, mass, eps, 1.0, dt, steps)
    tp, tv, tm = T(pos), T(vel), T(mass)
    acc, _ = nbody.accel(tp, tm, eps, 1.0, variant)
    pot = torch.empty_like(tm)
    diag = nbody.step(tp, tv, acc, tm, eps, 1.0, dt, steps, variant, pot=pot)
    torch.cuda.synchronize()
    assert np.abs(tp.cpu().numpy() - p_ref).max() < 1e-7
    assert np.abs(tv.cpu().numpy() - v_ref).max() < 1e-6
    a = acc.cpu().numpy()
    # forces at the GPU's own final positions
    ref_a, ref_p = orc.accel_pot(tp.cpu().numpy(), mass, eps)
    check(a, pot.cpu().numpy(), ref_a, ref_p)
    d = diag.cpu().numpy()
    assert d.shape == (steps, 16)
    np.testing.assert_array_equal(d[:, 14], np.arange(1, steps + 1))
    np.testing.assert_allclose(d[:, 0], rows[1:, 0], rtol=1e-9)          # K
    np.testing.assert_allclose(d[:, 1], rows[1:, 1], rtol=1e-6)          # W
    np.testing.assert_allclose(d[:, 2], rows[1:, 2], rtol=1e-5)          # E
    assert np.abs(d[:, 3:6]).max() < 1e-9                               # P
    np.testing.assert_allclose(d[:, 6:9], rows[1:, 6:9], atol=1e-9)     # L
    np.testing.assert_allclose(d[:, 12], 1.0, rtol=1e-14)
    assert np.all(d[:, 13] == 0)
    drift_gpu = abs(d[-1, 2] - rows[0, 2]) / abs(rows[0, 2])
    drift_ref = orc.energy_drift(rows)[-1]
    assert abs(drift_gpu - drift_ref) < 2e-6
    print(f"plummer_1k {variant}: energy drift gpu {drift_gpu:.3e} oracle {drift_ref:.3e}")


def test_kdk_split_equals_straight_run():
    pos, vel, mass = ics.plummer(3000, seed=12)
    runs = []
    for split in ((6,), (3, 3), (1, 2, 3)):
        tp, tv, tm = T(pos), T(vel), T(mass)
        acc, _ = nbody.accel(tp, tm, 0.01, 1.0, "comp")
        for k in split:
            nbody.step(tp, tv, acc, tm, 0.01, 1.0, 1.0 / 256, k, "comp", diag=False)
        torch.cuda.synchronize()
        runs.append((tp.cpu().numpy(), tv.cpu().numpy(), acc.cpu().numpy()))
    for r in runs[1:]:
        for x, y in zip(r, runs[0]):
            assert np.array_equal(x, y)


def test_kdk_time_reversibility():
    pos, vel, mass = ics.plummer(512, seed=21)
    eps, dt, n = 0.02, 1.0 / 128, 10
    tp, tv, tm = T(pos), T(vel), T(mass)
    acc, _ = nbody.accel(tp, tm, eps, 1.0, "comp")
    nbody.step(tp, tv, acc, tm, eps, 1.0, dt, n, "comp", diag=False)
    tv.neg_()
    nbody.step(tp, tv, acc, tm, eps, 1.0, dt, n, "comp", diag=False)
    tv.neg_()
    torch.cuda.synchronize()
    # FP32 forces are reproducible functions of the positions, so the run
    # retraces itself up to the rounding of the FP64 update.
    assert np.abs(tp.cpu().numpy() - pos).max() < 1e-8
    assert np.abs(tv.cpu().numpy() - vel).max() < 1e-7


def test_kepler_eps0_on_gpu():
    m1, m2, e, s = 0.3, 0.7, 0.5, 1.0
    mu = m1 + m2
    rp = s * (1 - e)
    vp = math.sqrt(mu * (1 + e) / rp)
    pos = np.array([[-m2 / mu * rp, 0, 0], [m1 / mu * rp, 0, 0]])
    vel = np.array([[0, -m2 / mu * vp, 0], [0, m1 / mu * vp, 0]])
    mass = np.array([m1, m2])
    period = 2 * math.pi
    steps = 2000
    dt = period / steps
    p_ref, v_ref, _, _, rows = orc.kdk(pos, vel, mass, 0.0, 1.0, dt, steps)
    tp, tv, tm = T(pos), T(vel), T(mass)
    acc, _ = nbody.accel(tp, tm, 0.0, 1.0, "comp")
    diag = nbody.step(tp, tv, acc, tm, 0.0, 1.0, dt, steps, "comp")
    torch.cuda.synchronize()
    assert np.abs(tp.cpu().numpy() - p_ref).max() < 1e-5
    # FP32 forces are central only to rounding, so L drifts at ~1e-7.
    lz = diag.cpu().numpy()[:, 8]
    assert np.abs(lz - rows[0, 8]).max() < 2e-6 * abs(rows[0, 8])


# ---- batched ----------------------------------------------------------------

def _small_ensemble(k=24, seed=6):
    return ics.ensemble(k, seed=seed, n_min=64, n_max=3000)


def _batched_ref(ens):
    acc = np.empty_like(ens.pos)
    pot = np.empty(len(ens.mass))
    for c in range(len(ens.sizes)):
        s, e = ens.offsets[c], ens.offsets[c + 1]
        acc[s:e], pot[s:e] = orc.accel_pot(ens.pos[s:e], ens.mass[s:e], ens.eps[c])
    return acc, pot


@pytest.mark.parametrize("variant", ["comp", "plain"])
def test_batched_matches_per_cluster_oracle(variant):
    ens = _small_ensemble()
    ref_a, ref_p = _batched_ref(ens)
    plan = nbody.Plan(ens.offsets, variant)
    assert plan.n_total == len(ens.mass)
    assert plan.pairs == float(np.sum(ens.sizes.astype(np.float64) ** 2))
    a1, p1 = plan.accel(T(ens.pos), T(ens.mass), T(ens.eps))
    a2, p2 = plan.accel(T(ens.pos), T(ens.mass), T(ens.eps))
    torch.cuda.synchronize()
    a1, p1, a2, p2 = (x.cpu().numpy() for x in (a1, p1, a2, p2))
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)
    for c in range(len(ens.sizes)):
        s, e = ens.offsets[c], ens.offsets[c + 1]
        check(a1[s:e], p1[s:e], ref_a[s:e], ref_p[s:e], what=(variant, c))
    plan.close()


@pytest.mark.parametrize("variant", ["comp", "plain"])
def test_batched_every_mode(variant, tmp_path):
    """Every compiled batched mode (LDS-tiled and scalar-stream shapes),
    forced for all cluster sizes, matches the per-cluster oracle and is
    bitwise reproducible."""
    ens = _small_ensemble(k=10, seed=17)
    ref_a, ref_p = _batched_ref(ens)
    v = nbody.VARIANTS[variant]
    try:
        for mode in range(len(nbody.batched_modes())):
            path = tmp_path / f"mode{mode}.txt"
            path.write_text("".join(f"batched {v} {c} {mode}\n" for c in range(48)))
            plan = nbody.Plan(ens.offsets, variant, tune_path=str(path))
            a1, p1 = plan.accel(T(ens.pos), T(ens.mass), T(ens.eps))
            a2, p2 = plan.accel(T(ens.pos), T(ens.mass), T(ens.eps))
            torch.cuda.synchronize()
            a1, p1, a2, p2 = (x.cpu().numpy() for x in (a1, p1, a2, p2))
            assert np.array_equal(a1, a2) and np.array_equal(p1, p2), mode
            for c in range(len(ens.sizes)):
                s, e = ens.offsets[c], ens.offsets[c + 1]
                check(a1[s:e], p1[s:e], ref_a[s:e], ref_p[s:e], what=(variant, mode, c))
            plan.close()
    finally:
        nbody.tune_reset()


def test_batched_leakage():
    """All clusters sit at the origin: if any pair crossed a cluster boundary
    the error would be of order one, not 1e-6."""
    ens = _small_ensemble(k=8, seed=9)
    ref_a, _ = _batched_ref(ens)
    whole_a, _ = orc.accel_pot(ens.pos, ens.mass, float(ens.eps.min()))
    assert orc.rel_rms(whole_a, ref_a) > 0.1
    plan = nbody.Plan(ens.offsets, "comp")
    a, _ = plan.accel(T(ens.pos), T(ens.mass), T(ens.eps))
    torch.cuda.synchronize()
    assert orc.rel_rms(a.cpu().numpy(), ref_a) < RMS_TOL


def test_batched_eps_k_per_call():
    """The softenings are an argument of every batched call: one plan, two
    eps_k arrays (the second scales cluster k's softening by a different
    factor per cluster, one cluster unsoftened), each result equal per
    cluster to the oracle with that cluster's own softening."""
    ens = _small_ensemble(k=9, seed=23)
    plan = nbody.Plan(ens.offsets, "comp")
    tp, tm = T(ens.pos), T(ens.mass)
    eps_b = ens.eps * np.linspace(0.5, 4.0, len(ens.eps))
    eps_b[3] = 0.0
    results = []
    for eps in (ens.eps, eps_b):
        a, p = plan.accel(tp, tm, T(eps))
        torch.cuda.synchronize()
        a, p = a.cpu().numpy(), p.cpu().numpy()
        for c in range(len(ens.sizes)):
            s, e = ens.offsets[c], ens.offsets[c + 1]
            ra, rp = orc.accel_pot(ens.pos[s:e], ens.mass[s:e], float(eps[c]))
            check(a[s:e], p[s:e], ra, rp, what=("eps_k", c, eps[c]))
        results.append(a)
    # the softening really changed every cluster's result
    for c in range(len(ens.sizes)):
        s, e = ens.offsets[c], ens.offsets[c + 1]
        assert orc.rel_rms(results[1][s:e], results[0][s:e]) > 1e-4, c
    plan.close()


def test_batched_call_validation_with_a_plan():
    """Host-side checks that need a real plan: the variant must be the
    plan's, eps_k must be present, aligned and apart from the outputs; a
    rejected call leaves its outputs untouched."""
    lib = nbody.load()
    ens = _small_ensemble(k=4, seed=31)
    plan = nbody.Plan(ens.offsets, "comp")
    tp, tm, te = T(ens.pos), T(ens.mass), T(ens.eps)
    acc = torch.full_like(tp, 7.0)
    ws = nbody.workspace(plan.n_total, plan.K, "comp", DEV)
    n = plan.n_total

    def call(eps_ptr, variant=1, acc_ptr=None):
        return lib.nbody_accel_batched(tp.data_ptr(), tm.data_ptr(), plan.handle, eps_ptr, 1.0, variant,
                                       acc.data_ptr() if acc_ptr is None else acc_ptr, None,
                                       ws.data_ptr(), ws.numel(), nbody._stream_handle(tp.device))
    assert call(te.data_ptr(), variant=0) == nbody.EINVAL
    assert "variant" in nbody.last_error()
    assert call(te.data_ptr(), variant=5) == nbody.ENOTSUP
    assert call(None) == nbody.EINVAL
    assert call(te.data_ptr() + 4) == nbody.EINVAL
    assert call(acc.data_ptr() + 8) == nbody.EINVAL          # eps_k inside acc
    torch.cuda.synchronize()
    assert torch.all(acc == 7.0)
    vel = torch.zeros_like(tp)
    st = lib.nbody_step_batched(tp.data_ptr(), vel.data_ptr(), acc.data_ptr(), None, tm.data_ptr(), n,
                                plan.handle, vel.data_ptr(), 1.0, 0.01, 1, 1, None, ws.data_ptr(),
                                ws.numel(), nbody._stream_handle(tp.device))
    assert st == nbody.EINVAL and "eps_k" in nbody.last_error()  # eps_k overlaps vel
    st = lib.nbody_step_batched(tp.data_ptr(), vel.data_ptr(), acc.data_ptr(), None, tm.data_ptr(), n + 1,
                                plan.handle, te.data_ptr(), 1.0, 0.01, 1, 1, None, ws.data_ptr(),
                                ws.numel(), nbody._stream_handle(tp.device))
    assert st == nbody.EINVAL and "plan covers" in nbody.last_error()
    st = lib.nbody_step(tp.data_ptr(), vel.data_ptr(), acc.data_ptr(), None, tm.data_ptr(), n, 0.01, 1.0,
                        0.01, 1, 1, plan.handle, None, ws.data_ptr(), ws.numel(), nbody._stream_handle(tp.device))
    assert st == nbody.EINVAL and "nbody_step_batched" in nbody.last_error()
    torch.cuda.synchronize()
    assert torch.all(acc == 7.0)
    plan.close()


def test_plan_tuning_file_is_plan_local(tmp_path):
    """A plan created with a tuning file takes its batched modes from it and
    leaves the process-wide tuning (single-system and jerk tables) alone."""
    before = (nbody.tune_get("plain", 1 << 20), nbody.tune_get("comp", 5000), nbody.tune_jerk_get("comp", 1 << 16))
    ens = _small_ensemble(k=6, seed=41)
    ref_a, ref_p = _batched_ref(ens)
    f = tmp_path / "plan.txt"
    f.write_text("single 0 20 2 4\nsingle 1 12 3 2\njerk 1 16 4 2\n"
                 + "".join(f"batched 1 {c} 0\n" for c in range(48)))
    plan = nbody.Plan(ens.offsets, "comp", tune_path=str(f))
    assert (nbody.tune_get("plain", 1 << 20), nbody.tune_get("comp", 5000),
            nbody.tune_jerk_get("comp", 1 << 16)) == before
    a, p = plan.accel(T(ens.pos), T(ens.mass), T(ens.eps))
    default = nbody.Plan(ens.offsets, "comp")
    a2, _ = default.accel(T(ens.pos), T(ens.mass), T(ens.eps))
    torch.cuda.synchronize()
    a, p, a2 = a.cpu().numpy(), p.cpu().numpy(), a2.cpu().numpy()
    for c in range(len(ens.sizes)):
        s, e = ens.offsets[c], ens.offsets[c + 1]
        check(a[s:e], p[s:e], ref_a[s:e], ref_p[s:e], what=("plan-local mode 0", c))
    # mode 0 (LDS tiles) and the default modes sum in different orders
    assert not np.array_equal(a, a2)
    plan.close()
    default.close()


def test_batched_empty_and_single_clusters():
    offsets = np.array([0, 0, 1, 1, 300, 300, 301], dtype=np.int64)
    eps = np.array([0.1, 0.1, 0.1, 0.02, 0.1, 0.0])
    rng = np.random.default_rng(4)
    pos = rng.normal(size=(301, 3))
    mass = rng.uniform(0.1, 1.0, size=301)
    plan = nbody.Plan(offsets, "comp")
    a, p = plan.accel(T(pos), T(mass), T(eps))
    torch.cuda.synchronize()
    a, p = a.cpu().numpy(), p.cpu().numpy()
    assert np.all(a[0] == 0) and np.all(a[300] == 0) and p[0] == 0 and p[300] == 0
    ra, rp = orc.accel_pot(pos[1:300], mass[1:300], 0.02)
    check(a[1:300], p[1:300], ra, rp)


@pytest.mark.parametrize("variant", ["comp", "plain"])
def test_batched_graph_steps(variant):
    """KDK steps replayed from the plan's HIP graph: equal to the FP64 oracle
    run per cluster (trajectories and diagnostics), bitwise equal across two
    runs, and a split run equals a straight one."""
    ens = _small_ensemble(k=12, seed=13)
    dt, steps = 1.0 / 256, 6
    plan = nbody.Plan(ens.offsets, variant)
    te = T(ens.eps)
    outs = []
    for split in ((steps,), (2, 4)):
        tp, tv, tm = T(ens.pos), T(ens.vel), T(ens.mass)
        acc, _ = plan.accel(tp, tm, te)
        diags = []
        for k in split:
            diags.append(nbody.step_batched(tp, tv, acc, tm, plan, te, 1.0, dt, k).cpu().numpy())
        torch.cuda.synchronize()
        outs.append((tp.cpu().numpy(), tv.cpu().numpy(), acc.cpu().numpy(), np.concatenate(diags)))
    for x, y in zip(outs[0][:3], outs[1][:3]):
        assert np.array_equal(x, y)
    p_gpu, v_gpu, a_gpu, d_gpu = outs[0]
    k_tot = 0.0
    for c in range(len(ens.sizes)):
        s, e = ens.offsets[c], ens.offsets[c + 1]
        pr, vr, ar, _, rows = orc.kdk(ens.pos[s:e], ens.vel[s:e], ens.mass[s:e], ens.eps[c], 1.0, dt, steps)
        assert np.abs(p_gpu[s:e] - pr).max() < 1e-7
        assert np.abs(v_gpu[s:e] - vr).max() < 1e-5
        k_tot += rows[-1, 0]
    np.testing.assert_allclose(d_gpu[-1, 0], k_tot, rtol=1e-8)
    np.testing.assert_allclose(d_gpu[-1, 12], len(ens.sizes), rtol=1e-13)
    plan.close()


@pytest.mark.parametrize("variant", ["comp", "plain"])
def test_batched_graph_replays_match_eager_steps(variant):
    """Each replay of the plan's captured step against the same step done
    eagerly (kick and drift as torch FP64 operations, forces from an eager
    batched launch), with other eager launches on the same workspace and
    host synchronisations between the replays: every replay rebuilds what
    the graph reads (packed slots, work counters), so none inherits a
    previous launch's state."""
    ens = _small_ensemble(k=10, seed=21)
    dt, h = 1.0 / 256, 0.5 / 256
    plan = nbody.Plan(ens.offsets, variant)
    te = T(ens.eps)
    tm = T(ens.mass)
    x, v = T(ens.pos), T(ens.vel)
    a, _ = plan.accel(x, tm, te)
    xr, vr, ar = x.clone(), v.clone(), a.clone()
    other = T(ens.pos[::-1].copy())
    diag = torch.empty((1, nbody.DIAG_LEN), dtype=torch.float64, device=DEV)
    for step in range(6):
        nbody.step_batched(x, v, a, tm, plan, te, 1.0, dt, 1, diag=diag)
        torch.cuda.synchronize()
        # the same step, eagerly
        vr = vr + h * ar
        xr = xr + dt * vr
        ar, pr = plan.accel(xr, tm, te)
        vr = vr + h * ar
        # unrelated eager work on the shared workspace between replays
        plan.accel(other, tm, te)
        torch.cuda.synchronize()
        for got, ref, name in ((x, xr, "pos"), (v, vr, "vel"), (a, ar, "acc")):
            g, r = got.cpu().numpy(), ref.cpu().numpy()
            scale = np.abs(r).max()
            assert np.abs(g - r).max() <= 1e-12 * scale, (variant, step, name, np.abs(g - r).max() / scale)
        kin = 0.5 * float((tm * (vr * vr).sum(1)).sum())
        np.testing.assert_allclose(diag[0, nbody.DIAG["K"]].item(), kin, rtol=1e-12)
        np.testing.assert_allclose(diag[0, nbody.DIAG["W"]].item(), 0.5 * float((tm * pr).sum()), rtol=1e-10)
    plan.close()
