"""The autotuner run end to end on small size classes: it writes one line per
variant and class, each pick is the fastest candidate it timed, the file
loads into the library's tuning table, and the tuned dispatches meet the
metric's tolerances against the FP64 oracle (single systems, acceleration +
jerk, and a batched plan that reads the file's batched modes)."""
import collections

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2509_19294_amd import autotune, ics, nbody

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def test_autotuner_end_to_end(tmp_path):
    nbody.load()
    nbody.tune_reset()
    out, record = autotune.main(["--out", str(tmp_path / "tune.txt"), "--min-log2", "10", "--max-log2", "11",
                                 "--batched-classes", "8,9", "--reps", "1"])
    lines = [ln.split() for ln in open(out) if ln.strip() and not ln.startswith("#")]
    kinds = collections.Counter((ln[0], ln[1]) for ln in lines)
    assert kinds == {(k, v): 2 for k in ("single", "jerk", "batched") for v in ("0", "1")}, kinds
    names = {0: "plain", 1: "comp"}
    for ln in lines:
        kind, v, c = ln[0], names[int(ln[1])], int(ln[2])
        if kind == "batched":
            rows = [r for r in record if r.get("class") == c and r["variant"] == v and "mode" in r]
            pick = [r for r in rows if r["mode"] == int(ln[3])]
        else:
            want = "jerk" if kind == "jerk" else None
            rows = [r for r in record if r.get("log2n") == c and r["variant"] == v and r.get("kernel") == want]
            pick = [r for r in rows if r["cfg"] == int(ln[3]) and r["split"] == int(ln[4])]
        assert rows and len(pick) == 1, ln
        assert pick[0]["ms"] <= min(r["ms"] for r in rows) + 1e-4, (ln, pick[0], min(r["ms"] for r in rows))

    try:
        nbody.tune_load(out)
        for ln in lines:
            if ln[0] == "single":
                assert nbody.tune_get(names[int(ln[1])], 1 << int(ln[2])) == (int(ln[3]), max(int(ln[4]), 1))
        for n in (1024, 2047):
            pos, vel, mass = ics.plummer(n, seed=n)
            tp, tv, tm = T(pos), T(vel), T(mass)
            ra, rp = orc.accel_pot(pos, mass, 0.01)
            rja, rj, _ = orc.accel_jerk(pos, vel, mass, 0.01)
            for variant in ("plain", "comp"):
                a, p = nbody.accel(tp, tm, 0.01, 1.0, variant)
                ja, jj, _ = nbody.accel_jerk(tp, tv, tm, 0.01, 1.0, variant)
                torch.cuda.synchronize()
                a, p, ja, jj = (x.cpu().numpy() for x in (a, p, ja, jj))
                assert orc.rel_rms(a, ra) <= 1e-5 and orc.max_rel(a, ra) <= 1e-4, (n, variant)
                assert orc.rel_rms(p, rp) <= 1e-5, (n, variant)
                assert orc.rel_rms(ja, rja) <= 1e-5, (n, variant)
                assert orc.paper_metric(jj, rj) <= 2e-3, (n, variant)
        ens = ics.ensemble(12, seed=5, n_min=256, n_max=1023)
        te, tp, tm = T(ens.eps), T(ens.pos), T(ens.mass)
        for variant in ("plain", "comp"):
            plan = nbody.Plan(ens.offsets, variant, tune_path=out)
            a, p = plan.accel(tp, tm, te)
            torch.cuda.synchronize()
            a, p = a.cpu().numpy(), p.cpu().numpy()
            plan.close()
            for k in range(len(ens.sizes)):
                s, e = int(ens.offsets[k]), int(ens.offsets[k + 1])
                ra, rp = orc.accel_pot(ens.pos[s:e], ens.mass[s:e], float(ens.eps[k]))
                assert orc.rel_rms(a[s:e], ra) <= 1e-5 and orc.max_rel(a[s:e], ra) <= 1e-4, (variant, k)
                assert orc.rel_rms(p[s:e], rp) <= 1e-5, (variant, k)
    finally:
        nbody.tune_reset()
