"""Checks of the seeded synthetic initial conditions (CPU only)."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2509_19294_amd import ics


def test_plummer_reproducible_and_normalised():
    a = ics.plummer(2048, seed=7)
    b = ics.plummer(2048, seed=7)
    c = ics.plummer(2048, seed=8)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    assert not np.array_equal(a[0], c[0])
    pos, vel, mass = a
    assert pos.shape == (2048, 3) and vel.shape == (2048, 3) and mass.shape == (2048,)
    assert pos.dtype == np.float64 and pos.flags.c_contiguous
    assert math.isclose(mass.sum(), 1.0, rel_tol=1e-14)
    assert np.abs((mass[:, None] * pos).sum(0)).max() < 1e-14
    assert np.abs((mass[:, None] * vel).sum(0)).max() < 1e-15


def test_plummer_radii_follow_mass_profile():
    pos, vel, _ = ics.plummer(20000, seed=1)
    r = np.linalg.norm(pos, axis=1)
    cdf = lambda x: x ** 3 / (1 + x * x) ** 1.5
    assert stats.kstest(r, cdf).pvalue > 1e-3
    # bound speeds: every particle is below the local escape speed
    vesc = math.sqrt(2.0) * (1 + r * r) ** -0.25
    assert np.all(np.linalg.norm(vel, axis=1) < vesc + 1e-3)


def test_plummer_velocity_dispersion():
    """Isotropic Plummer model: one-dimensional dispersion sigma^2(r) = 1 / (6 sqrt(1 + r^2))."""
    pos, vel, _ = ics.plummer(40000, seed=2)
    r = np.linalg.norm(pos, axis=1)
    v2 = np.sum(vel * vel, axis=1) / 3.0
    for lo, hi in [(0, 0.5), (0.5, 1), (1, 2), (2, 5)]:
        sel = (r >= lo) & (r < hi)
        expect = np.mean(1.0 / (6.0 * np.sqrt(1 + r[sel] ** 2)))
        se = v2[sel].std(ddof=1) / math.sqrt(sel.sum())
        assert abs(v2[sel].mean() - expect) < 5 * se


def test_directions_isotropic():
    pos, vel, _ = ics.plummer(20000, seed=3)
    for x in (pos, vel):
        u = x / np.linalg.norm(x, axis=1, keepdims=True)
        assert np.abs(u.mean(0)).max() < 5 / math.sqrt(20000)
        assert stats.kstest(u[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-3


def test_kroupa_masses():
    pos, vel, mass = ics.plummer_kroupa(100000, seed=3)
    assert math.isclose(mass.sum(), 1.0, rel_tol=1e-13)
    raw = mass / mass.min()
    assert raw.max() <= 100 / 0.08 + 1e-6
    rng = np.random.default_rng(0)
    m = ics.kroupa_masses(200000, rng)
    assert m.min() >= 0.08 and m.max() <= 100.0
    f_low = np.mean(m < 0.5)
    expect, _ = ics._kroupa_segment_weights()
    assert abs(expect - 0.7607) < 1e-3
    assert abs(f_low - expect) < 5 * math.sqrt(expect * (1 - expect) / m.size)
    # upper segment: dN/dm ~ m^-2.3 -> the fraction above 5 of those above 0.5
    hi = m[m >= 0.5]
    frac = np.mean(hi > 5.0)
    e = (5.0 ** -1.3 - 100.0 ** -1.3) / (0.5 ** -1.3 - 100.0 ** -1.3)
    assert abs(frac - e) < 5 * math.sqrt(e * (1 - e) / hi.size)
    assert np.abs((mass[:, None] * vel).sum(0)).max() < 1e-15
    assert np.abs((mass[:, None] * pos).sum(0)).max() < 1e-14


def test_ensemble_structure():
    ens = ics.ensemble(64, seed=2)
    assert ens.offsets[0] == 0 and np.all(np.diff(ens.offsets) == ens.sizes)
    assert ens.sizes.min() >= 256 and ens.sizes.max() <= 8192
    np.testing.assert_array_equal(ens.eps, 4.0 / ens.sizes)
    for k in range(64):
        s, e = ens.offsets[k], ens.offsets[k + 1]
        assert math.isclose(ens.mass[s:e].sum(), 1.0, rel_tol=1e-13)
        assert np.abs((ens.mass[s:e, None] * ens.pos[s:e]).sum(0)).max() < 1e-13


def test_ensemble_512_sizes_log_uniform():
    children = np.random.SeedSequence(2).spawn(513)
    r0 = np.random.default_rng(children[0])
    u = r0.uniform(math.log(256), math.log(8192), size=512)
    sizes = np.clip(np.rint(np.exp(u)), 256, 8192)
    assert stats.kstest(np.log(sizes), "uniform", args=(math.log(256), math.log(32))).pvalue > 1e-3
    assert 2.0e3 < sizes.mean() < 3.0e3


@pytest.mark.slow
def test_ensemble_512_full():
    ens = ics.ensemble(512, seed=2)
    assert len(ens.sizes) == 512 and ens.offsets[-1] == ens.sizes.sum()
    # expected sum of N_k^2 for log-uniform sizes on [256, 8192] ~ 4.95e9
    assert 3e9 < float(np.sum(ens.sizes.astype(np.float64) ** 2)) < 7e9


def test_workload_table():
    assert set(ics.WORKLOADS) == {"plummer_1k", "plummer_64k", "plummer_256k", "ensemble_512", "kroupa_1m",
                                  "plummer_102k"}
    pos, vel, mass, spec = ics.workload("plummer_1k")
    assert pos.shape == (1024, 3) and spec["eps"] == 0.01 and spec["dt"] == 1.0 / 128
    np.testing.assert_array_equal(pos, ics.plummer(1024, seed=0)[0])
