"""Autotuner for the pair kernels.

    python -m paper_2509_19294_amd.autotune [--out FILE] [--max-log2 20]

For every size class (n = 2^c) and both forms it times each compiled
configuration (block shape, i per thread, lane and wave j-splits, j-tile,
LDS or scalar source stream) with every grid j-split the workspace allows, on
a seeded Plummer sphere, and keeps the fastest. For the batched kernel it
times each mode on ensembles whose clusters all fall in one size class. The
result is a tuning file for ``nbody_tune_load`` / ``NBODY_TUNE`` (lines
``single <variant> <class> <cfg> <split>``, ``batched <variant> <class>
<mode>`` and ``jerk <variant> <class> <shape> <split>`` for the acceleration +
jerk kernel) and a JSON record of every measurement.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import tempfile

import numpy as np

from paper_2509_19294_amd import ics, nbody


def _time(fn, reps, warm=1):
    import torch

    for _ in range(warm):
        fn()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def tune_single(variant, log2n, reps=5, splits=(1, 2, 4, 8, 16, 32), configs=None, log=None,
                large_splits=(1, 2)):
    import torch

    n = 1 << log2n
    pos, _, mass = ics.plummer(n, seed=1000 + log2n)
    tp = torch.from_numpy(pos).cuda()
    tm = torch.from_numpy(mass).cuda()
    acc = torch.empty_like(tp)
    pot = torch.empty_like(tm)
    cfgs = nbody.tune_configs(variant)
    idx = range(len(cfgs)) if configs is None else configs
    best = None
    rows = []
    # large systems: fewer repetitions and no deep splits
    if n >= (1 << 19):
        reps = min(reps, 2)
        splits = tuple(s for s in splits if s in large_splits)
    try:
        for c in idx:
            for sp in splits:
                nb_blocks = math.ceil(n / cfgs[c][5]) * sp
                if sp > 1 and nb_blocks > 64 * 1024:
                    continue
                nbody.tune_set(variant, log2n, c, sp)
                ms = _time(lambda: nbody.accel(tp, tm, 0.01, 1.0, variant, acc=acc, pot=pot), reps)
                rate = float(n) * n / (ms * 1e-3) / 1e9
                rows.append({"variant": variant, "log2n": log2n, "cfg": c, "split": sp, "ms": round(ms, 4),
                             "G_int_per_s": round(rate, 1)})
                if log:
                    log(rows[-1])
                if best is None or ms < best[2]:
                    best = (c, sp, ms)
    finally:
        nbody.tune_set(variant, log2n, -1)
    return best, rows


def tune_jerk(variant, log2n, reps=5, splits=(1, 2, 4, 8, 16, 32), log=None, shape_list=None):
    """Time every acceleration + jerk kernel shape with every grid j-split on
    a Plummer sphere of 2^log2n particles; returns the fastest."""
    import torch

    n = 1 << log2n
    pos, vel, mass = ics.plummer(n, seed=2000 + log2n)
    tp, tv, tm = (torch.from_numpy(x).cuda() for x in (pos, vel, mass))
    acc, jerk, pot = torch.empty_like(tp), torch.empty_like(tp), torch.empty_like(tm)
    shapes = nbody.jerk_shapes(variant)
    if n >= (1 << 19):
        reps = min(reps, 2)
    best, rows = None, []
    try:
        for c, (k, sw, ib) in enumerate(shapes):
            if shape_list is not None and c not in shape_list:
                continue
            for sp in splits:
                if sp > 1 and (math.ceil(n / ib) * sp > 64 * 1024 or n // sp < 1024 or sp * n > (1 << 23)):
                    continue
                nbody.tune_jerk_set(variant, c, sp)
                ms = _time(lambda: nbody.accel_jerk(tp, tv, tm, 0.01, 1.0, variant, acc=acc, jerk=jerk,
                                                    pot=pot), reps)
                rate = float(n) * n / (ms * 1e-3) / 1e9
                rows.append({"kernel": "jerk", "variant": variant, "log2n": log2n, "cfg": c, "k": k, "sw": sw,
                             "split": sp, "ms": round(ms, 4), "G_int_per_s": round(rate, 1)})
                if log:
                    log(rows[-1])
                if best is None or ms < best[2]:
                    best = (c, sp, ms)
    finally:
        nbody.tune_jerk_set(variant, -1)
    return best, rows


def _class_ensemble(c, k, seed):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1 << c, (1 << (c + 1)) - 1, size=k, endpoint=True)
    offsets = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    pos = np.empty((offsets[-1], 3))
    mass = np.empty(offsets[-1])
    for i in range(k):
        p, _, m = ics.plummer(int(sizes[i]), rng=np.random.default_rng(seed + 1 + i))
        pos[offsets[i]:offsets[i + 1]] = p
        mass[offsets[i]:offsets[i + 1]] = m
    return pos, mass, offsets, 4.0 / sizes


def tune_batched(variant, c, reps=5, log=None):
    import torch

    k = max(8, min(512, (1 << 22) // (1 << (2 * c - 8))))
    pos, mass, offsets, eps = _class_ensemble(c, k, 77 + c)
    tp = torch.from_numpy(pos).cuda()
    tm = torch.from_numpy(mass).cuda()
    te = torch.from_numpy(eps).cuda()
    acc = torch.empty_like(tp)
    pot = torch.empty_like(tm)
    best = None
    rows = []
    for mode in range(len(nbody.batched_modes())):
        with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as f:
            f.write(f"batched {nbody.VARIANTS[variant]} {c} {mode}\n")
            path = f.name
        try:
            plan = nbody.Plan(offsets, variant, tune_path=path)
            ms = _time(lambda: plan.accel(tp, tm, te, 1.0, acc=acc, pot=pot), reps)
            rate = plan.pairs / (ms * 1e-3) / 1e9
            plan.close()
        finally:
            os.unlink(path)
        rows.append({"variant": variant, "class": c, "mode": mode, "clusters": k, "ms": round(ms, 4),
                     "G_int_per_s": round(rate, 1)})
        if log:
            log(rows[-1])
        if best is None or ms < best[1]:
            best = (mode, ms)
    return best, rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.txt"))
    ap.add_argument("--json", default=None)
    ap.add_argument("--min-log2", type=int, default=10)
    ap.add_argument("--max-log2", type=int, default=20)
    ap.add_argument("--variants", default="plain,comp")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--no-jerk", action="store_true")
    ap.add_argument("--configs", default=None,
                    help="comma-separated configurations (or jerk shapes) to time (default: all)")
    ap.add_argument("--large-splits", default="1,2",
                    help="grid splits timed for systems of 2^19 particles and more")
    ap.add_argument("--batched-classes", default="8,9,10,11,12,13",
                    help="cluster size classes (log2 N_k) timed for the batched kernel")
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions per candidate")
    args = ap.parse_args(argv)
    cfg_list = [int(c) for c in args.configs.split(",")] if args.configs else None
    large = tuple(int(c) for c in args.large_splits.split(","))
    nbody.load()
    nbody.tune_reset()
    lines = ["# kind variant class cfg [split] -- written by paper_2509_19294_amd.autotune"]
    record = []

    def log(r):
        print(json.dumps(r), flush=True)
        record.append(r)

    for variant in args.variants.split(","):
        v = nbody.VARIANTS[variant]
        for c in ([] if args.no_single else range(args.min_log2, args.max_log2 + 1)):
            (cfg, sp, ms), _ = tune_single(variant, c, reps=args.reps, log=log, configs=cfg_list,
                                           large_splits=large)
            lines.append(f"single {v} {c} {cfg} {sp}")
            print(f"# best {variant} 2^{c}: cfg {cfg} split {sp} {ms:.4f} ms", flush=True)
        for c in ([] if args.no_jerk else range(args.min_log2, args.max_log2 + 1)):
            (cfg, sp, ms), _ = tune_jerk(variant, c, reps=args.reps, log=log, shape_list=cfg_list)
            lines.append(f"jerk {v} {c} {cfg} {sp}")
            print(f"# best jerk {variant} 2^{c}: shape {cfg} split {sp} {ms:.4f} ms", flush=True)
        if not args.no_batched:
            for c in (int(x) for x in args.batched_classes.split(",") if x):
                (mode, ms), _ = tune_batched(variant, c, reps=args.reps, log=log)
                lines.append(f"batched {v} {c} {mode}")
                print(f"# best batched {variant} 2^{c}: mode {mode} {ms:.4f} ms", flush=True)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    if args.json:
        with open(args.json, "w") as f:
            json.dump(record, f)
    print(f"# wrote {args.out}")
    return args.out, record


if __name__ == "__main__":
    main()
