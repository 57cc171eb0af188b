"""Full-size, full-length runs of every workload, checked against the FP64
oracle at the GPU's own state.

Each multi-step workload runs its whole step count through the C ABI; the
forces the GPU holds after the last step (the accelerations at the final
positions) are then compared with the oracle evaluated on those same final
positions (trajectories are chaotic, so force parity is taken on the GPU's
own state, at the first and at the last step). The 65,536-particle run is
also compared step for step with the oracle's own ten-step trajectory.
Tolerances are the metric's: acceleration rel-RMS <= 1e-5 and per-particle
max-rel <= 1e-4, potential rel-RMS <= 1e-5, and the paper's per-component
criterion (5e-4 of the RMS magnitude). Energy drift has no paper or
closed-form value (parity unpinned): it is printed, and only checked for
being finite and small.
"""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import cpu as ocpu
from oracle import oracle as orc
from paper_2509_19294_amd import ics, nbody

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _setup():
    ocpu.build(force=False)
    nbody.load()
    nbody.tune_reset()
    yield


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def check(a, p, ref_a, ref_p, what):
    e = (orc.rel_rms(a, ref_a), orc.max_rel(a, ref_a), orc.rel_rms(p, ref_p), orc.paper_metric(a, ref_a))
    assert e[0] <= 1e-5, (what, "acc rel-rms", e[0])
    assert e[1] <= 1e-4, (what, "acc max-rel", e[1])
    assert e[2] <= 1e-5, (what, "pot rel-rms", e[2])
    assert e[3] <= 5e-4, (what, "paper metric", e[3])
    print(f"{what}: acc rel-rms {e[0]:.3e} max-rel {e[1]:.3e} pot rel-rms {e[2]:.3e} paper {e[3]:.3e}",
          flush=True)
    return e


def run_single(name, variant, steps=None):
    """The workload's initial forces, a zero-length step (initial energy row)
    and its KDK steps. Returns the initial and final GPU state and the rows."""
    pos, vel, mass, spec = ics.workload(name)
    eps, dt = spec["eps"], spec["dt"]
    steps = spec["steps"] if steps is None else steps
    tp, tv, tm = T(pos), T(vel), T(mass)
    pot = torch.empty_like(tm)
    acc, _ = nbody.accel(tp, tm, eps, 1.0, variant, pot=pot)
    torch.cuda.synchronize()
    a0, p0 = acc.cpu().numpy(), pot.cpu().numpy()
    d0 = nbody.step(tp, tv, acc, tm, eps, 1.0, 0.0, 1, variant, pot=pot)
    rows = nbody.step(tp, tv, acc, tm, eps, 1.0, dt, steps, variant, pot=pot)
    torch.cuda.synchronize()
    out = dict(pos0=pos, vel0=vel, mass=mass, eps=eps, dt=dt, steps=steps, a0=a0, p0=p0,
               pos=tp.cpu().numpy(), vel=tv.cpu().numpy(), acc=acc.cpu().numpy(), pot=pot.cpu().numpy(),
               e0=float(d0.cpu().numpy()[0, 2]), rows=rows.cpu().numpy())
    return out


def report_drift(name, variant, r):
    rows = r["rows"]
    de = np.abs(rows[:, 2] - r["e0"]) / abs(r["e0"])
    assert np.all(rows[:, 13] == 0), "non-finite positions or velocities"
    assert np.all(np.isfinite(de)) and de.max() < 1e-4, de.max()
    np.testing.assert_array_equal(rows[:, 14], np.arange(1, r["steps"] + 1))
    print(f"{name} {variant}: {r['steps']} steps, energy drift final {de[-1]:.3e} max {de.max():.3e}, "
          f"max |P| {np.abs(rows[:, 3:6]).max():.3e}", flush=True)


@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_plummer_64k_ten_steps(variant):
    """N = 65,536 (seed 1, eps 0.005): ten KDK steps at dt = 1/256; the full
    N^2 oracle at step 0 and at the final positions, and the trajectory
    against the oracle's own ten steps."""
    r = run_single("plummer_64k", variant)
    ref_a, ref_p = ocpu.accel_pot(r["pos0"], r["mass"], r["eps"])
    check(r["a0"], r["p0"], ref_a, ref_p, ("plummer_64k", variant, "step 0"))
    ref_a, ref_p = ocpu.accel_pot(r["pos"], r["mass"], r["eps"])
    check(r["acc"], r["pot"], ref_a, ref_p, ("plummer_64k", variant, "step 10"))
    p_ref, v_ref, _, _ = ocpu.kdk(r["pos0"], r["vel0"], r["mass"], r["eps"], 1.0, r["dt"], r["steps"])
    # FP32 force errors (per particle up to ~2e-5 relative) move a particle
    # by ~1e-8 over ten steps of 1/256
    assert np.abs(r["pos"] - p_ref).max() < 1e-7
    assert np.abs(r["vel"] - v_ref).max() < 1e-5
    report_drift("plummer_64k", variant, r)


def test_plummer_256k_thousand_steps():
    """N = 262,144 (seed 4, eps 0.002), compensated form: all 1,000 KDK steps
    at dt = 1/512; 4,096 strided targets against all sources at step 0 and
    at the final positions; energy drift reported."""
    r = run_single("plummer_256k", "comp")
    tgt = orc.subsample_targets(len(r["mass"]), 4096)
    ref_a, ref_p = ocpu.accel_pot(r["pos0"], r["mass"], r["eps"], targets=tgt)
    check(r["a0"][tgt], r["p0"][tgt], ref_a, ref_p, ("plummer_256k", "comp", "step 0"))
    ref_a, ref_p = ocpu.accel_pot(r["pos"], r["mass"], r["eps"], targets=tgt)
    check(r["acc"][tgt], r["pot"][tgt], ref_a, ref_p, ("plummer_256k", "comp", "step 1000"))
    report_drift("plummer_256k", "comp", r)


def test_kroupa_1m_ten_steps():
    """N = 1,048,576 with Kroupa masses (seed 3, eps 0.001), compensated form:
    ten KDK steps at dt = 1/1024; 4,096 strided targets against all sources
    at step 0 and at the final positions."""
    r = run_single("kroupa_1m", "comp")
    tgt = orc.subsample_targets(len(r["mass"]), 4096)
    ref_a, ref_p = ocpu.accel_pot(r["pos0"], r["mass"], r["eps"], targets=tgt)
    check(r["a0"][tgt], r["p0"][tgt], ref_a, ref_p, ("kroupa_1m", "comp", "step 0"))
    ref_a, ref_p = ocpu.accel_pot(r["pos"], r["mass"], r["eps"], targets=tgt)
    check(r["acc"][tgt], r["pot"][tgt], ref_a, ref_p, ("kroupa_1m", "comp", "step 10"))
    report_drift("kroupa_1m", "comp", r)


def _per_cluster(ens, pos, acc, pot, what, variant):
    """Every cluster against its own oracle. The compensated form meets the
    metric's tolerances and the paper's per-component criterion against the
    exact FP64 inputs. The plain form takes its inputs in FP32, and rounding
    the absolute coordinates alone (the oracle evaluated exactly on the
    rounded inputs) misses both on a few of this ensemble's clusters: rel-RMS
    up to 5.7e-5 (12 of 512 clusters above 1e-5) and the paper's metric up to
    2.5e-3 (10 above 5e-4), on clusters of 4,000-8,000 particles softened by
    4/N_k. So the plain kernel is held to the metric's tolerances against the
    oracle on the rounded inputs, and against the exact ones to that
    rounding's own error plus the tolerance."""
    worst = np.zeros(4)
    for c in range(len(ens.sizes)):
        s, e = int(ens.offsets[c]), int(ens.offsets[c + 1])
        x, m = pos[s:e], ens.mass[s:e]
        ra, rp = ocpu.accel_pot(x, m, float(ens.eps[c]))
        a, p = acc[s:e], pot[s:e]
        exact = orc.rel_rms(a, ra)
        if variant == "plain":
            x32 = x.astype(np.float32).astype(np.float64)
            m32 = m.astype(np.float32).astype(np.float64)
            rra, rrp = ocpu.accel_pot(x32, m32, float(ens.eps[c]))
            assert exact <= orc.rel_rms(rra, ra) + 1e-5, (what, c, exact, orc.rel_rms(rra, ra))
            ra, rp = rra, rrp
        else:
            assert orc.paper_metric(a, ra) <= 5e-4, (what, c)
        e1, e2, e3 = orc.rel_rms(a, ra), orc.max_rel(a, ra), orc.rel_rms(p, rp)
        assert e1 <= 1e-5 and e2 <= 1e-4 and e3 <= 1e-5, (what, c, e - s, e1, e2, e3)
        worst = np.maximum(worst, (e1, e2, e3, exact))
    print(f"ensemble_512 {what}: worst cluster acc rel-rms {worst[0]:.3e} max-rel {worst[1]:.3e} "
          f"pot rel-rms {worst[2]:.3e}; against exact inputs acc rel-rms {worst[3]:.3e}", flush=True)


@pytest.mark.parametrize("variant", ["comp", "plain"])
def test_ensemble_512_hundred_graph_steps(variant):
    """The 512-cluster ensemble (seed 2, N_k log-uniform in [256, 8192],
    eps_k = 4/N_k, 1,166,512 particles): every particle of every cluster
    against that cluster's own oracle at step 0 and after all 100 KDK steps
    replayed from the plan's HIP graph (dt = 1/256)."""
    ens, spec = ics.workload("ensemble_512")
    assert len(ens.sizes) == 512 and len(ens.mass) == 1166512
    plan = nbody.Plan(ens.offsets, variant)
    tp, tv, tm, te = T(ens.pos), T(ens.vel), T(ens.mass), T(ens.eps)
    pot = torch.empty_like(tm)
    acc, _ = plan.accel(tp, tm, te, pot=pot)
    torch.cuda.synchronize()
    _per_cluster(ens, ens.pos, acc.cpu().numpy(), pot.cpu().numpy(), f"{variant} step 0", variant)
    d0 = nbody.step_batched(tp, tv, acc, tm, plan, te, 1.0, 0.0, 1, pot=pot)
    rows = nbody.step_batched(tp, tv, acc, tm, plan, te, 1.0, spec["dt"], spec["steps"], pot=pot)
    torch.cuda.synchronize()
    _per_cluster(ens, tp.cpu().numpy(), acc.cpu().numpy(), pot.cpu().numpy(), f"{variant} step 100",
                 variant)
    r = dict(rows=rows.cpu().numpy(), e0=float(d0.cpu().numpy()[0, 2]), steps=spec["steps"])
    report_drift("ensemble_512", variant, r)
    plan.close()


@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_paper_shaped_run_ten_steps(variant):
    """The paper-shaped run (Section 4): N = 102,400, fourth-order Hermite
    with accelerations and jerks on the GPU, ten steps, time- and
    energy-to-solution. The final state's accelerations and jerks meet the
    paper's own criterion against the FP64 oracle on 4,096 targets (every
    component within 5e-4, jerks within 2e-3, of the RMS magnitude); the
    energy record carries the GPU energy counter's integral, or says why not."""
    sys.path.insert(0, ROOT)
    import bench

    (res,) = bench.paper_run(variant, cpu_seconds=0, readings=("steps",), min_seconds=3.0)
    assert res["n"] == 102400 and res["steps"] == 10 and res["nonfinite"] == 0
    fc = res["final_check"]
    assert fc["targets"] == 4096
    assert fc["acc_paper_metric"] <= 5e-4 and fc["jerk_paper_metric"] <= 2e-3, fc
    assert fc["acc_rel_rms"] <= 1e-5, fc
    assert res["time_to_solution_s"] > 0 and res["runs"] >= 3
    en = res["energy_to_solution"]
    for key in ("wall_s", "gpu_energy_j", "gpu_power_samples", "gpu_energy_from_power_samples_j",
                "host_energy_j", "notes", "runs_measured"):
        assert key in en, key
    try:
        import amdsmi  # noqa: F401
        have_smi = True
    except Exception:
        have_smi = False
    if have_smi and en["gpu_energy_j"] is None:
        assert en["notes"], "no GPU energy and no note saying why"
    if en["gpu_energy_j"] is not None:
        assert en["gpu_energy_j"] > 0 and en["gpu_energy_j_per_run"] > 0
    if not have_smi:
        assert any("amdsmi" in n for n in en["notes"])
    print(f"paper run {variant}: {res['time_to_solution_s']} s per ten-step run, "
          f"GPU energy {en['gpu_energy_j']} J over {en['runs_measured']} runs, notes {en['notes']}", flush=True)
