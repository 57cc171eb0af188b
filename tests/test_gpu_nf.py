"""GPU parity of the near/far compensated kernel (configurations 19-25 of
the compensated form): spatial ordering, per-block frames, hi-only far
tiles. Same tolerances as the compensated form (rel-RMS <= 1e-5, worst
particle <= 1e-4); results must be bitwise reproducible, translation must not
degrade them, and the ordering must stay invisible (outputs at the caller's
indices)."""
import math

import numpy as np
import pytest
import torch

from oracle import cpu as ocpu
from oracle import oracle as orc
from paper_2509_19294_amd import ics, nbody

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NF_CFGS = (19, 20, 21, 22, 23, 24, 25)


@pytest.fixture(scope="module", autouse=True)
def _setup():
    ocpu.build(force=False)
    nbody.load()
    nbody.tune_reset()
    yield
    nbody.tune_reset()


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def nf_accel(pos, mass, eps, cfg, split=1):
    n = len(mass)
    c = max(int(math.floor(math.log2(n))), 0)
    nbody.tune_set("comp", c, cfg, split)
    try:
        a, p = nbody.accel(T(pos), T(mass), eps, 1.0, "comp")
        torch.cuda.synchronize()
        return a.cpu().numpy(), p.cpu().numpy()
    finally:
        nbody.tune_set("comp", c, -1)


def check(a, p, ra, rp, what):
    assert orc.rel_rms(a, ra) <= 1e-5, (what, orc.rel_rms(a, ra))
    assert orc.max_rel(a, ra) <= 1e-4, (what, orc.max_rel(a, ra))
    assert orc.rel_rms(p, rp) <= 1e-5, (what, orc.rel_rms(p, rp))


def test_configurations_exist_for_compensated_only():
    assert len(nbody.tune_configs("comp")) == len(nbody.tune_configs("plain")) + len(NF_CFGS)
    with pytest.raises(nbody.NbodyError):
        nbody.tune_set("plain", 10, 19, 1)


@pytest.mark.parametrize("cfg", NF_CFGS)
@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 513, 1000, 4099])
@pytest.mark.parametrize("eps", [0.01, 0.0])
def test_sizes_and_splits(cfg, n, eps):
    pos, _, mass = ics.plummer(n, seed=300 + n)
    ra, rp = orc.accel_pot(pos, mass, eps)
    for split in (1, 3):
        a, p = nf_accel(pos, mass, eps, cfg, split)
        if n == 1:
            assert np.all(a == 0) and np.all(p == 0)
            continue
        check(a, p, ra, rp, (cfg, n, eps, split))
        a2, p2 = nf_accel(pos, mass, eps, cfg, split)
        assert np.array_equal(a, a2) and np.array_equal(p, p2)


@pytest.mark.parametrize("cfg", NF_CFGS)
def test_translation_and_permutation(cfg):
    pos, _, mass = ics.plummer(5000, seed=41)
    ra, rp = orc.accel_pot(pos, mass, 0.01)
    for shift in (1e3, 1e5):
        a, p = nf_accel(pos + np.array([shift, -shift, 0.5 * shift]), mass, 0.01, cfg, 2)
        check(a, p, ra, rp, (cfg, "shift", shift))
    perm = np.random.default_rng(5).permutation(5000)
    a, p = nf_accel(pos[perm], mass[perm], 0.01, cfg, 2)
    check(a, p, ra[perm], rp[perm], (cfg, "permuted"))


@pytest.mark.parametrize("cfg", NF_CFGS)
def test_distant_clusters_take_far_tiles(cfg):
    """Two clusters 100 apart: most tiles are far; the result still meets the
    tolerance (the far path's separations carry a few ulps)."""
    p1, _, m1 = ics.plummer(3000, seed=7)
    p2, _, m2 = ics.plummer(3000, seed=8)
    pos = np.concatenate([p1, p2 * 0.5 + np.array([100.0, 0, 0])])
    mass = np.concatenate([m1, m2]) * 0.5
    ra, rp = orc.accel_pot(pos, mass, 0.001)
    a, p = nf_accel(pos, mass, 0.001, cfg, 1)
    check(a, p, ra, rp, (cfg, "clusters"))
    # the far path's bound (separations within 6 u |d|, u = 2^-24) keeps the
    # result near FP32 rounding (measured 1.0e-7 to 2.8e-7): far tiles
    # staged relative to a frame in the other cluster, 100 away, would round
    # every intra-cluster separation to about u 100, 1e-5 of a typical one
    e = orc.rel_rms(a, ra)
    print(f"distant clusters cfg {cfg}: rel-rms {e:.3e} max-rel {orc.max_rel(a, ra):.3e}")
    assert e <= 1e-6, (cfg, e)


@pytest.mark.parametrize("cfg", NF_CFGS)
def test_plummer_64k_full_oracle(cfg):
    pos, _, mass, spec = ics.workload("plummer_64k")
    ra, rp = ocpu.accel_pot(pos, mass, spec["eps"])
    a, p = nf_accel(pos, mass, spec["eps"], cfg, 16)
    check(a, p, ra, rp, cfg)
    print(f"near/far cfg {cfg} N=65536: rel-rms {orc.rel_rms(a, ra):.3e} max-rel {orc.max_rel(a, ra):.3e}")


def test_kdk_steps_with_near_far():
    pos, vel, mass, spec = ics.workload("plummer_1k")
    eps, dt, steps = spec["eps"], spec["dt"], spec["steps"]
    p_ref, v_ref, _, _, rows = orc.kdk(pos, vel, mass, eps, 1.0, dt, steps)
    nbody.tune_set("comp", 10, 19, 2)
    try:
        tp, tv, tm = T(pos), T(vel), T(mass)
        acc, _ = nbody.accel(tp, tm, eps, 1.0, "comp")
        diag = nbody.step(tp, tv, acc, tm, eps, 1.0, dt, steps, "comp")
        torch.cuda.synchronize()
    finally:
        nbody.tune_set("comp", 10, -1)
    assert np.abs(tp.cpu().numpy() - p_ref).max() < 1e-7
    np.testing.assert_allclose(diag.cpu().numpy()[:, 2], rows[1:, 2], rtol=1e-5)


def _shapes(n, seed):
    rng = np.random.default_rng(seed)
    plane = np.column_stack([rng.normal(size=n), rng.normal(size=n), np.zeros(n)])
    line = np.column_stack([np.linspace(-3, 3, n) + rng.normal(scale=1e-3, size=n), np.zeros(n), np.zeros(n)])
    cube = rng.uniform(-1, 1, size=(n, 3))
    halo = rng.normal(size=(n, 3)) * np.exp(rng.uniform(-6, 9, size=(n, 1)))  # radii 1e-3 .. 1e4
    return {"plane": plane, "line": line, "cube": cube, "halo": halo}


@pytest.mark.parametrize("cfg", (19, 23, 24, 25))
@pytest.mark.parametrize("shape", ["plane", "line", "cube", "halo"])
def test_degenerate_and_extreme_layouts(cfg, shape):
    """Flat, one-dimensional, uniform and huge-dynamic-range layouts: the
    ordering's scale (zero variance on an axis) and the box tests must stay
    correct. The line has particles whose acceleration cancels 4,000-fold
    (the middle of the line), which no FP32 sum, double-single or not,
    reaches to 1e-4 per particle (measured: 1.4e-2 to 3.8e-2 for every
    compensated configuration): there the per-particle bound is replaced by
    the paper's criterion (largest component error within 5e-4 of the RMS
    magnitude) and the near/far result must stay within 3x the error of the
    double-single kernel."""
    n = 6000
    pos = _shapes(n, 11)[shape]
    mass = np.full(n, 1.0 / n)
    ra, rp = orc.accel_pot(pos, mass, 0.01)
    a, p = nf_accel(pos, mass, 0.01, cfg, 2)
    if shape != "line":
        check(a, p, ra, rp, (cfg, shape))
        return
    assert orc.rel_rms(a, ra) <= 1e-5 and orc.rel_rms(p, rp) <= 1e-5
    assert orc.paper_metric(a, ra) <= 5e-4
    ds, _ = nf_accel(pos, mass, 0.01, 9, 2)  # the double-single LDS kernel
    assert orc.rel_rms(a, ra) <= 3 * orc.rel_rms(ds, ra)


def test_stored_frame_matches_computed_frame():
    """Configuration 24 runs configuration 23's arithmetic with the block's
    centre and far threshold taken from the ordering pass instead of
    recomputed: same tiles on the same paths, so the same bits."""
    pos, _, mass = ics.plummer(20000, seed=77)
    for split in (1, 4):
        a23, p23 = nf_accel(pos, mass, 0.01, 23, split)
        a24, p24 = nf_accel(pos, mass, 0.01, 24, split)
        assert np.array_equal(a23, a24) and np.array_equal(p23, p24), split
