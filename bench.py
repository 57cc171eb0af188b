"""Benchmark of the direct-summation N-body hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--variant plain|comp] [--hermite] [--full-run] [--paper-run]

The default workload is the largest single-GPU system: a Plummer sphere of
N = 1,048,576 particles with Kroupa masses (seed 3), eps = 0.001,
dt = 1/1024, in the compensated form (double-single coordinates on a spatial
order, far tiles on the hi words); the plain FP32 kernel is timed beside it
on the same inputs.

A step is one kick-drift-kick leapfrog step of the whole path: kick and drift
(FP64), the force evaluation (pack or double-single staging, the FP32 pair
kernel, the j-split combine, the FP64 epilogue) and the closing kick fused
with the FP64 energy/momentum diagnostics. Inputs are seeded synthetic
Plummer spheres (or the cluster ensemble) already resident in HBM. With
--hermite a step is one fourth-order Hermite step instead (FP64 predictor,
the acceleration + jerk pair kernel, FP64 corrector and diagnostics).

Prints one JSON line: throughput in G pair-interactions/s (N^2 pair
evaluations per step, self pairs included, over the measured step time), the
roofline of the force kernel (20 flops per interaction against the FP32
vector peak, duration measured with HIP events around every force launch in
the timed region), the accuracy gate against the FP64 oracle on a target
subsample, and the FP64 oracle's own rate on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_CLOCK_MHZ = 2400.0           # the clock that peak is quoted at
FLOPS_PER_INTERACTION = 20        # the conventional count for one softened pair
# Acceleration + jerk: the force's 20 plus the jerk's own FP32 work per pair
# (relative velocity 3, d.w 5, alpha 2, w - alpha d 6, accumulation 6; an FMA
# counts 2).
FLOPS_PER_JERK_INTERACTION = 42
DEFAULT_VARIANT = {"plummer_1k": "plain", "plummer_64k": "plain", "plummer_256k": "comp",
                   "kroupa_1m": "comp", "ensemble_512": "comp", "plummer_102k": "plain"}

# HBM bytes per force-kernel launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
# passes, scaled by a 1 GiB copy (fetch x2.000, write x1.000), for the tuned
# dispatch they were taken on: (workload, variant, cfg, split) -> bytes. A run
# whose dispatch differs reports null.
MEASURED_TRAFFIC = {
    ("plummer_64k", "plain", 15, 16): 32541696,
    # near/far compensated kernel on half box groups, configuration 25
    ("plummer_256k", "comp", 25, 32): 334614642,
    # near/far with the stored frame, configuration 24, per-XCD block order
    ("kroupa_1m", "comp", 24, 16): 1081401037,
    # the plain scalar-stream kernel on the same inputs
    ("kroupa_1m", "plain", 15, 2): 50237857997,
    # acceleration + jerk kernel (bench.py --hermite): shape 2, split 32
    ("plummer_64k", "plain", "jerk", 2, 32): 98617549,
    # near/far acceleration + jerk kernel on half box groups, shape 12
    ("plummer_256k", "comp", "jerk", 12, 32): 687650464,
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="kroupa_1m",
                    choices=sorted(DEFAULT_VARIANT))
    ap.add_argument("--variant", default=None, choices=["plain", "comp"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--hermite", action="store_true",
                    help="time fourth-order Hermite steps (acceleration + jerk kernel) "
                         "instead of kick-drift-kick steps")
    ap.add_argument("--paper-run", action="store_true",
                    help="the paper's representative run (N = 102,400, Hermite): time- and "
                         "energy-to-solution for ten steps and for ten N-body time units")
    ap.add_argument("--full-run", action="store_true",
                    help="run the workload's whole step count and report time-to-solution, "
                         "energy/momentum drift and the final-state force error")
    return ap.parse_args()


def full_run(name, variant, steps=None):
    """The workload's complete run: initial force, all KDK steps with a
    diagnostics row each, then the final-state accelerations against the FP64
    oracle on 4096 strided targets (per cluster for the ensemble)."""
    import torch

    from oracle import cpu as ocpu
    from oracle import oracle as orc
    from paper_2509_19294_amd import energy, ics, nbody

    nbody.load()
    dev = torch.device("cuda:0")
    plan = None
    te = None
    if name == "ensemble_512":
        ens, spec = ics.workload(name)
        pos, vel, mass, eps = ens.pos, ens.vel, ens.mass, 0.0
        plan = nbody.Plan(ens.offsets, variant)
        te = torch.from_numpy(ens.eps).to(dev)
        pairs = plan.pairs
    else:
        pos, vel, mass, spec = ics.workload(name)
        eps = spec["eps"]
        pairs = float(len(mass)) ** 2
    steps = spec["steps"] if steps is None else steps
    tp, tv, tm = (torch.from_numpy(x).to(dev) for x in (pos, vel, mass))
    pot = torch.empty_like(tm)
    diag = torch.empty((steps, nbody.DIAG_LEN), dtype=torch.float64, device=dev)
    d0 = torch.empty((1, nbody.DIAG_LEN), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # the initial forces, a zero-length step for the initial energy (same
    # kernels), then the run
    if plan is not None:
        acc, _ = plan.accel(tp, tm, te, 1.0, pot=pot)
        nbody.step_batched(tp, tv, acc, tm, plan, te, 1.0, 0.0, 1, diag=d0, pot=pot)
        nbody.step_batched(tp, tv, acc, tm, plan, te, 1.0, spec["dt"], steps, diag=diag, pot=pot)
    else:
        acc, _ = nbody.accel(tp, tm, eps, 1.0, variant, pot=pot)
        nbody.step(tp, tv, acc, tm, eps, 1.0, 0.0, 1, variant, diag=d0, pot=pot)
        nbody.step(tp, tv, acc, tm, eps, 1.0, spec["dt"], steps, variant, diag=diag, pot=pot)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    d = diag.cpu().numpy()
    e0 = float(d0.cpu().numpy()[0, 2])
    de = np.abs(d[:, 2] - e0) / abs(e0)
    pf, af = tp.cpu().numpy(), acc.cpu().numpy()
    if plan is not None:
        k = int(np.argsort(ens.sizes)[len(ens.sizes) // 2])
        s, e = int(ens.offsets[k]), int(ens.offsets[k + 1])
        ref_a, _ = ocpu.accel_pot(pf[s:e], mass[s:e], float(ens.eps[k]))
        a_s = af[s:e]
        where = f"cluster {k} ({e - s} particles), all targets"
    else:
        tgt = orc.subsample_targets(len(mass), 4096)
        ref_a, _ = ocpu.accel_pot(pf, mass, eps, targets=tgt)
        a_s = af[tgt]
        where = f"{len(tgt)} strided targets"
    out = {
        "full_run": name, "variant": variant, "steps": steps, "dt": spec["dt"],
        "force_evaluations": steps + 2, "time_to_solution_s": round(wall, 3),
        "G_pair_per_s": round(pairs * (steps + 2) / wall / 1e9, 1),
        "energy_drift_final": float(f"{de[-1]:.3e}"), "energy_drift_max": float(f"{de.max():.3e}"),
        "momentum_max": float(f"{np.abs(d[:, 3:6]).max():.3e}"),
        "angular_momentum_change_max": float(f"{np.abs(d[:, 6:9] - d[0, 6:9]).max():.3e}"),
        "nonfinite": int(d[:, 13].max()),
        "final_acc_rel_rms": float(f"{orc.rel_rms(a_s, ref_a):.3e}"),
        "final_acc_max_rel": float(f"{orc.max_rel(a_s, ref_a):.3e}"),
        "final_check": where,
    }
    print(json.dumps(out), flush=True)
    if plan is not None:
        plan.close()


PAPER_TIME_TO_SOLUTION_S = {"wormhole_n300_plus_host": 301.40, "cpu_2x_epyc_9124": 672.90}
PAPER_ENERGY_TO_SOLUTION_KJ = {"wormhole_n300_plus_host": 71.56, "cpu_2x_epyc_9124": 128.89}


def paper_run(variant, units=10.0, cpu_seconds=10.0, readings=("steps", "units"), min_seconds=3.0):
    """The paper's representative run (Section 4) on one GPU: N = 102,400
    Plummer sphere, fourth-order Hermite with acceleration + jerk on the GPU
    and the FP64 update on the GPU. The paper does not define its "time
    cycle"; two readings are run: ten steps, and ten N-body time units at the
    workload's step. Time-to-solution spans the host's initial conditions,
    the upload, every force evaluation and update, and the download of the
    final state; energy-to-solution covers the same span (GPU energy counter,
    host RAPL when readable). ``readings`` picks "steps" and/or "units";
    ``cpu_seconds`` = 0 skips the CPU oracle's timing. Prints one JSON line
    per reading and returns them."""
    import torch

    from oracle import cpu as ocpu
    from oracle import oracle as orc
    from paper_2509_19294_amd import ics, nbody
    from paper_2509_19294_amd.energy import EnergyMeter

    nbody.load()
    dev = torch.device("cuda:0")
    spec = dict(ics.WORKLOADS["plummer_102k"])
    n, eps, dt = spec["n"], spec["eps"], spec["dt"]
    # load the kernels' code objects once, outside the timed span
    w = torch.zeros((256, 3), dtype=torch.float64, device=dev)
    w[:, 0] = torch.arange(256, dtype=torch.float64, device=dev)
    wm = torch.full((256,), 1.0 / 256, dtype=torch.float64, device=dev)
    wa, wj, _ = nbody.accel_jerk(w, w.clone(), wm, eps, 1.0, variant)
    nbody.step_hermite(w, w.clone(), wa, wj, wm, eps, 1.0, dt, 1, variant)
    torch.cuda.synchronize()

    def run_once(steps):
        """One complete simulation; returns its wall time, the host
        initial-conditions time, the final state and the diagnostics."""
        t0 = time.perf_counter()
        pos, vel, mass = ics.plummer(n, seed=spec["seed"])
        t_ic = time.perf_counter() - t0
        tp, tv, tm = (torch.from_numpy(x).to(dev) for x in (pos, vel, mass))
        pot = torch.empty_like(tm)
        acc, jerk, _ = nbody.accel_jerk(tp, tv, tm, eps, 1.0, variant, pot=pot)
        d0 = nbody.step_hermite(tp, tv, acc, jerk, tm, eps, 1.0, 0.0, 1, variant, pot=pot)
        diag = nbody.step_hermite(tp, tv, acc, jerk, tm, eps, 1.0, dt, steps, variant, pot=pot)
        pf, vf = tp.cpu().numpy(), tv.cpu().numpy()
        d = diag.cpu().numpy()
        e0 = float(d0.cpu().numpy()[0, 2])
        wall = time.perf_counter() - t0
        return wall, t_ic, (pos, vel, mass, pf, vf), d, e0

    todo = []
    if "steps" in readings:
        todo.append(("ten steps", spec["steps"]))
    if "units" in readings:
        todo.append((f"{units:g} time units", int(round(units / dt))))
    results = []
    for reading, steps in todo:
        # A short run is repeated back to back (at least 3 times, about 3 s in
        # all) so that the GPU energy counter, which advances at its own
        # interval, spans it; time and energy are reported per run.
        walls, ics_s = [], []
        with EnergyMeter() as em:
            t_all = time.perf_counter()
            while True:
                wall, t_ic, state, d, e0 = run_once(steps)
                walls.append(wall)
                ics_s.append(t_ic)
                if len(walls) >= 3 and time.perf_counter() - t_all >= min_seconds:
                    break
                if steps > 100:
                    break
        energy = em.result()
        runs = len(walls)
        energy["runs_measured"] = runs
        for key in ("gpu_energy_j", "gpu_energy_from_power_samples_j", "host_energy_j"):
            if energy.get(key) is not None:
                energy[key.replace("_j", "_j_per_run")] = round(energy[key] / runs, 3)
        pos, vel, mass, pf, vf = state
        de = np.abs(d[:, 2] - e0) / abs(e0)
        wall = float(np.median(walls))
        out = {
            "paper_run": "plummer_102k", "reading": reading, "variant": variant, "n": n, "eps": eps,
            "dt": dt, "steps": steps, "force_jerk_evaluations": steps + 2,
            "time_to_solution_s": round(wall, 4), "runs": runs,
            "time_to_solution_s_min": round(float(np.min(walls)), 4),
            "host_initial_conditions_s": round(float(np.median(ics_s)), 4),
            "G_pair_per_s": round(float(n) * n * (steps + 2) / wall / 1e9, 1),
            "energy_drift_final": float(f"{de[-1]:.3e}"), "energy_drift_max": float(f"{de.max():.3e}"),
            "nonfinite": int(d[:, 13].max()),
            "energy_to_solution": energy,
            "paper_time_to_solution_s": PAPER_TIME_TO_SOLUTION_S,
            "paper_energy_to_solution_kJ": PAPER_ENERGY_TO_SOLUTION_KJ,
        }
        if reading == "ten steps":
            # the final state's accelerations and jerks against the FP64 oracle
            tp, tv, tm = (torch.from_numpy(x).to(dev) for x in (pf, vf, mass))
            ta, tj, _ = nbody.accel_jerk(tp, tv, tm, eps, 1.0, variant)
            tgt = orc.subsample_targets(n, 4096)
            ra, rj, _ = ocpu.accel_jerk(pf, vf, mass, eps, targets=tgt)
            ga, gj = ta.cpu().numpy()[tgt], tj.cpu().numpy()[tgt]
            out["final_check"] = {
                "targets": len(tgt), "acc_rel_rms": float(f"{orc.rel_rms(ga, ra):.3e}"),
                "acc_paper_metric": float(f"{orc.paper_metric(ga, ra):.3e}"),
                "jerk_rel_rms": float(f"{orc.rel_rms(gj, rj):.3e}"),
                "jerk_paper_metric": float(f"{orc.paper_metric(gj, rj):.3e}"),
            }
            if cpu_seconds > 0:
                cb, _, _ = cpu_baseline(pos, mass, eps, cpu_seconds, vel=vel)
                per_eval = float(n) * n / (cb["value"] * 1e9)
                cb["time_to_solution_s_extrapolated"] = round(per_eval * (steps + 2), 1)
                out["cpu_baseline"] = cb
        print(json.dumps(out), flush=True)
        results.append(out)
    return results


def cpu_baseline(pos, mass, eps, budget_s, vel=None):
    """Time the FP64 C oracle (OpenMP over all host threads) on a bounded
    sample of the workload: whole force evaluations repeated, or, when one
    evaluation exceeds the budget, a strided subset of targets against all
    sources. With ``vel`` the oracle evaluates accelerations and jerks.
    Returns the rate, the sample description, the gate targets (a strided
    subsample of at most 4096) and the oracle's values on them: (acc, pot)
    or (acc, pot, jerk)."""
    from oracle import cpu as ocpu
    from oracle import oracle as orc

    ocpu.build(force=False)
    n = len(mass)
    threads = ocpu.max_threads()

    def evaluate(targets=None):
        if vel is None:
            return ocpu.accel_pot(pos, mass, eps, targets=targets)
        a, j, p = ocpu.accel_jerk(pos, vel, mass, eps, targets=targets)
        return a, p, j

    # rate probe: strided targets against all sources, grown until it takes
    # a measurable time (thread start-up dominates tiny probes)
    nprobe = min(n, 64)
    while True:
        probe = orc.subsample_targets(n, nprobe)
        t0 = time.perf_counter()
        evaluate(probe)
        dt_probe = time.perf_counter() - t0
        if dt_probe >= 0.25 or nprobe >= n:
            break
        nprobe = min(n, nprobe * 4)
    rate = len(probe) * n / max(dt_probe, 1e-6)
    gate = orc.subsample_targets(n, 4096)
    full_s = float(n) * n / rate
    if full_s <= 0.5 * budget_s:
        # whole evaluations, repeated until the budget is spent
        reps = 0
        t0 = time.perf_counter()
        while True:
            full = evaluate()
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget_s or reps >= 1000:
                break
        pairs = reps * float(n) * n
        sample = f"{reps} full evaluations of {n} x {n} pairs"
        refs = tuple(x[gate] for x in full)
    else:
        nt = int(min(n, max(256, budget_s * rate / n)))
        tgt = orc.subsample_targets(n, nt)
        t0 = time.perf_counter()
        evaluate(tgt)
        el = time.perf_counter() - t0
        pairs = float(len(tgt)) * n
        sample = f"{len(tgt)} strided targets x {n} sources"
        refs = evaluate(gate)
    # one whole evaluation, extrapolated from a target subset's rate
    extrapolated = None if full_s <= 0.5 * budget_s else round(float(n) * n / (pairs / el), 2)
    what = "accelerations and potentials" if vel is None else "accelerations, jerks and potentials"
    return {
        "value": pairs / el / 1e9,
        "unit": "G pair-interactions/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{sample} ({pairs:.3e} FP64 pairs in {el:.1f} s; {what}; C + OpenMP, {threads} threads)",
        "cpu_model": _cpu_model(),
        "full_evaluation_s_extrapolated": extrapolated,
        "numpy_single_thread": _numpy_oracle_rate(pos, mass, eps, vel),
    }, gate, refs


def _cpu_model():
    """The host CPU's model name, from /proc/cpuinfo (None if unreadable)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _numpy_oracle_rate(pos, mass, eps, vel=None, min_s=0.2):
    """Rate of the numpy oracle (one thread) on strided targets against all
    sources, for information beside the C oracle's."""
    from oracle import oracle as orc

    n = len(mass)
    k = min(n, 4)
    while True:
        tgt = orc.subsample_targets(n, k)
        t0 = time.perf_counter()
        if vel is None:
            orc.accel_pot(pos, mass, eps, targets=tgt)
        else:
            orc.accel_jerk(pos, vel, mass, eps, targets=tgt)
        el = time.perf_counter() - t0
        if el >= min_s or k >= n:
            break
        k = min(n, k * 4)
    return {"value": round(len(tgt) * n / max(el, 1e-9) / 1e9, 4), "unit": "G pair-interactions/s",
            "sample": f"{len(tgt)} strided targets x {n} sources"}


def device_info():
    """Name, compute units and temperatures of cuda:0 at the end of a run
    (temperatures from the system-management library, None if unreadable)."""
    import torch

    from paper_2509_19294_amd import energy

    props = torch.cuda.get_device_properties(0)
    info = {"name": props.name, "arch": getattr(props, "gcnArchName", None),
            "compute_units": props.multi_processor_count}
    info.update(energy.temperatures(0))
    return info


def copy_calibration(mib: int = 1024, reps: int = 5):
    """A plain device-to-device copy of known size, for scaling the HBM
    traffic counters (FETCH_SIZE / WRITE_SIZE) of the force kernel."""
    import torch

    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": a.numel() * 4, "reps": reps}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                          "(the library has no multi-GPU path)"}))
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    if args.full_run:
        full_run(args.workload, args.variant or DEFAULT_VARIANT[args.workload])
        return
    if args.paper_run:
        paper_run(args.variant or "plain", cpu_seconds=args.cpu_seconds)
        return

    import torch

    from paper_2509_19294_amd import energy, ics, nbody

    nbody.load()
    dev = torch.device("cuda:0")
    name = args.workload
    variant = args.variant or DEFAULT_VARIANT[name]
    hermite = args.hermite
    if hermite and name == "ensemble_512":
        print(json.dumps({"error": "--hermite runs on a single system, not the cluster ensemble"}))
        sys.exit(2)
    plan = plain_plan = te = None
    if name == "ensemble_512":
        ens, spec = ics.workload(name)
        pos, vel, mass = ens.pos, ens.vel, ens.mass
        eps = 0.0
        plan = nbody.Plan(ens.offsets, variant)
        te = torch.from_numpy(ens.eps).to(dev)
        pairs_per_eval = plan.pairs
        n = len(mass)
    else:
        pos, vel, mass, spec = ics.workload(name)
        eps = spec["eps"]
        n = len(mass)
        pairs_per_eval = float(n) * float(n)
    dt = spec["dt"]

    tp = torch.from_numpy(pos).to(dev)
    tv = torch.from_numpy(vel).to(dev)
    tm = torch.from_numpy(mass).to(dev)
    pot = torch.empty_like(tm)
    acc = torch.empty_like(tp)
    jerk = torch.empty_like(tp) if hermite else None

    def force(form=variant, on_plan=None):
        """One force (or acceleration + jerk) evaluation on the current state."""
        if on_plan is not None:
            on_plan.accel(tp, tm, te, 1.0, acc=acc, pot=pot)
        elif hermite:
            nbody.accel_jerk(tp, tv, tm, eps, 1.0, form, acc=acc, jerk=jerk, pot=pot)
        else:
            nbody.accel(tp, tm, eps, 1.0, form, acc=acc, pot=pot)

    force(on_plan=plan)
    torch.cuda.synchronize()
    acc0 = acc.cpu().numpy()
    pot0 = pot.cpu().numpy()
    jerk0 = jerk.cpu().numpy() if hermite else None

    diag = torch.empty((1, nbody.DIAG_LEN), dtype=torch.float64, device=dev)

    def one_step():
        if hermite:
            nbody.step_hermite(tp, tv, acc, jerk, tm, eps, 1.0, dt, 1, variant, diag=diag, pot=pot)
        elif plan is not None:
            nbody.step_batched(tp, tv, acc, tm, plan, te, 1.0, dt, 1, diag=diag, pot=pot)
        else:
            nbody.step(tp, tv, acc, tm, eps, 1.0, dt, 1, variant, diag=diag, pot=pot)

    # Bring the GPU out of its idle clock state before the warm-up steps: force
    # evaluations on the same inputs (no state change) for about 0.3 s.
    t_ramp = time.perf_counter() + 0.3
    while time.perf_counter() < t_ramp:
        for _ in range(10 if pairs_per_eval < 1e11 else 1):
            force(on_plan=plan)
        torch.cuda.synchronize()

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    # the graphics clock, sampled over the timed steps and the repeated force
    # evaluations (the fraction of peak is also stated at that clock)
    clock = energy.ClockSampler(0)
    clock.__enter__()
    # one event between consecutive steps: the first and last bracket the
    # timed region, the others give per-step durations (median, min)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    nbody.timing_enable(plan is None)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    marks[0].record(stream)
    for s_ in range(args.steps):
        one_step()
        marks[s_ + 1].record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_total = marks[0].elapsed_time(marks[-1])
    step_ms = [marks[k].elapsed_time(marks[k + 1]) for k in range(args.steps)]
    launches, kernel_ms = nbody.timing_read()
    nbody.timing_enable(False)

    def evaluations(reps, form=variant, on_plan=None):
        """The force evaluation alone (ordering or pack, pair kernel, split
        combine, epilogue), repeated on the same inputs: per-evaluation times
        and the pair kernel's own (launches, total ms) from the library's
        event brackets."""
        times = []
        nbody.timing_enable(True)
        for _ in range(reps):
            a_ev = torch.cuda.Event(enable_timing=True)
            b_ev = torch.cuda.Event(enable_timing=True)
            a_ev.record(stream)
            force(form, on_plan)
            b_ev.record(stream)
            b_ev.synchronize()
            times.append(a_ev.elapsed_time(b_ev))
        kern = nbody.timing_read()
        nbody.timing_enable(False)
        return times, kern

    force_ms, kern_eval = evaluations(max(args.steps, 5), on_plan=plan)
    clock.__exit__(None, None, None)
    clk = clock.result()
    if plan is not None:
        # The batched force kernel runs inside the graph replay: its duration
        # comes from the same kernels launched eagerly on the same stream.
        launches, kernel_ms = kern_eval

    traffic = None
    if hermite:
        cfg, split = nbody.tune_jerk_get(variant, n)
        traffic = MEASURED_TRAFFIC.get((name, variant, "jerk", cfg, split))
    elif plan is None:
        cfg, split = nbody.tune_get(variant, n)
        traffic = MEASURED_TRAFFIC.get((name, variant, cfg, split))
    else:
        traffic = MEASURED_TRAFFIC.get((name, variant, "batched"))
    ms_per_step = ms_total / args.steps
    value = pairs_per_eval / (ms_per_step * 1e-3) / 1e9
    kernel_avg_ms = kernel_ms / max(launches, 1)
    flops = FLOPS_PER_JERK_INTERACTION if hermite else FLOPS_PER_INTERACTION
    achieved = flops * pairs_per_eval / (kernel_avg_ms * 1e-3) / 1e12

    # The plain FP32 kernel on the same inputs (the state the timed steps
    # left), the reference point the compensated form is reported against.
    plain = None
    if variant == "comp":
        plain_plan = nbody.Plan(ens.offsets, "plain") if plan is not None else None
        force("plain", plain_plan)   # first use: code objects, workspace
        torch.cuda.synchronize()
        p_ms, (p_l, p_k) = evaluations(max(3, min(args.steps, 10)), "plain", plain_plan)
        p_avg = p_k / max(p_l, 1)
        p_ach = flops * pairs_per_eval / (p_avg * 1e-3) / 1e12
        p_traffic = None
        if plain_plan is None:
            p_cfg, p_split = nbody.tune_get("plain", n)
            p_traffic = MEASURED_TRAFFIC.get((name, "plain", p_cfg, p_split))
        plain = {
            "what": "the plain FP32 kernel on the same inputs and GPU, repeated evaluations",
            "kernel_avg_ms": round(p_avg, 4), "kernel_launches": p_l, "traffic": p_traffic,
            "achieved_TFLOPs": round(p_ach, 2), "frac": round(p_ach / FP32_VECTOR_PEAK_TFLOPS, 4),
            "evaluation_ms_median": round(float(np.median(p_ms)), 4),
            "G_pair_per_s_median": round(pairs_per_eval / (float(np.median(p_ms)) * 1e-3) / 1e9, 1),
            "compensated_kernel_over_plain": round(p_avg / kernel_avg_ms, 4),
        }

    out = {
        "metric": ("G pair-interactions/s (acceleration + jerk) and % FP32 VALU peak at rel-RMS "
                   "accel err \u22641e-5 vs FP64" if hermite else
                   "G pair-interactions/s and % FP32 VALU peak at rel-RMS accel err \u22641e-5 vs FP64"),
        "value": round(value, 2),
        "unit": "G pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_median": round(float(np.median(step_ms)), 4),
        "ms_per_step_min": round(float(np.min(step_ms)), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{name}: " + (
                f"{plan.K} Plummer clusters, N_total={n}, eps_k=4/N_k" if plan is not None
                else f"Plummer sphere N={n}" + (" Kroupa masses" if name == "kroupa_1m" else "")
                + f", eps={eps}") + f", dt={dt}, one "
                + ("fourth-order Hermite" if hermite else "KDK") + " step with diagnostics",
            "variant": variant,
            "n": n,
            "pairs_per_step": pairs_per_eval,
        },
        "force_evaluation": {
            "what": "one " + ("acceleration + jerk" if hermite else "force") + " evaluation alone "
                    "(ordering or pack, pair kernel, split combine, FP64 epilogue), repeated",
            "ms_median": round(float(np.median(force_ms)), 4),
            "ms_min": round(float(np.min(force_ms)), 4),
            "G_pair_per_s_median": round(pairs_per_eval / (float(np.median(force_ms)) * 1e-3) / 1e9, 1),
        },
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 2),
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "kernel_avg_ms": round(kernel_avg_ms, 4),
            "kernel_launches": launches,
            "flops_per_interaction": flops,
            # the same fraction against the peak scaled to the sampled clock
            "frac_at_measured_clock": (round(achieved / (FP32_VECTOR_PEAK_TFLOPS * clk["gfx_mhz_median"]
                                                         / PEAK_CLOCK_MHZ), 4)
                                       if clk["gfx_mhz_median"] else None),
        },
        "clock": {"what": "graphics clock sampled every 50 ms over the timed steps and the repeated "
                          "force evaluations (mean over the XCDs)", **clk},
    }
    if plain is not None:
        out["plain_same_inputs"] = plain
    try:
        out["device"] = device_info()
    except Exception as e:  # informational only
        out["device"] = {"note": f"device information unavailable: {e}"}

    if not args.no_cpu_baseline:
        from oracle import oracle as orc

        if plan is not None:
            # one mid-sized cluster's targets against its own sources
            k = int(np.argsort(ens.sizes)[len(ens.sizes) // 2])
            s, e = int(ens.offsets[k]), int(ens.offsets[k + 1])
            cb, tgt, refs = cpu_baseline(pos[s:e], mass[s:e], float(ens.eps[k]), args.cpu_seconds)
            a_s, p_s = acc0[s:e][tgt], pot0[s:e][tgt]
        else:
            cb, tgt, refs = cpu_baseline(pos, mass, eps, args.cpu_seconds, vel=vel if hermite else None)
            a_s, p_s = acc0[tgt], pot0[tgt]
        ref_a, ref_p = refs[0], refs[1]
        out["cpu_baseline"] = cb
        acc_err = orc.rel_rms(a_s, ref_a)
        out["accuracy"] = {
            "acc_rel_rms": float(f"{acc_err:.3e}"),
            "acc_max_rel": float(f"{orc.max_rel(a_s, ref_a):.3e}"),
            "pot_rel_rms": float(f"{orc.rel_rms(p_s, ref_p):.3e}"),
            **({"jerk_rel_rms": float(f"{orc.rel_rms(jerk0[tgt], refs[2]):.3e}"),
                "jerk_paper_metric": float(f"{orc.paper_metric(jerk0[tgt], refs[2]):.3e}")} if hermite else {}),
            "targets": int(len(tgt)),
            "where": "the initial state, before the warm-up steps",
            "gate_rel_rms_1e-5": bool(acc_err <= 1e-5),
        }
        if plain is not None:
            # the plain kernel's error on the same targets of the initial state
            tp.copy_(torch.from_numpy(pos))
            force("plain", plain_plan)
            torch.cuda.synchronize()
            if plan is not None:
                pa = acc.cpu().numpy()[s:e][tgt]
            else:
                pa = acc.cpu().numpy()[tgt]
            plain["acc_rel_rms"] = float(f"{orc.rel_rms(pa, ref_a):.3e}")
            plain["acc_max_rel"] = float(f"{orc.max_rel(pa, ref_a):.3e}")
        if acc_err > 1e-5:
            out["value"] = None
            out["note"] = "accuracy gate failed: throughput not reported"
    print(json.dumps(out), flush=True)
    for p_ in (plan, plain_plan):
        if p_ is not None:
            p_.close()


if __name__ == "__main__":
    main()
