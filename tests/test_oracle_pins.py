"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle (numpy and C builds) against something the paper
or the mathematics fixes: hand-worked values of the force equation of
Section 3, closed forms (softened three-body, Kepler orbits, the exact
leapfrog map of a harmonic oscillator), invariants (Newton's third law,
translation, scaling, permutation, time reversibility, angular momentum) and
the statistical limits of a Plummer sphere.
"""
import math

import numpy as np
import pytest

from oracle import cpu as ocpu
from oracle import oracle as orc
from paper_2509_19294_amd import ics
from tests import golden_io


@pytest.fixture(scope="module", autouse=True)
def _build_c_oracle():
    ocpu.build(force=False)


def _three(name):
    g = golden_io.load(name)
    return g, golden_io.arr(g, "pos"), golden_io.arr(g, "mass")[0], float(g["eps"][0][0])


# ---- hand-worked three-body cases -------------------------------------------

@pytest.mark.parametrize("impl", ["numpy", "c", "brute"])
@pytest.mark.parametrize("name", ["three_body_eps0.txt", "three_body_eps1.txt"])
def test_three_body_hand_worked(impl, name):
    g, pos, mass, eps = _three(name)
    f = {"numpy": orc.accel_pot, "c": ocpu.accel_pot, "brute": orc.brute_force}[impl]
    acc, pot = f(pos, mass, eps, 1.0)
    np.testing.assert_allclose(acc, golden_io.arr(g, "acc"), rtol=0, atol=4e-16)
    np.testing.assert_allclose(pot, golden_io.arr(g, "pot")[0], rtol=0, atol=4e-16)
    w = 0.5 * np.sum(mass * pot)
    assert abs(w - g["W"][0][0]) <= 1e-15


def test_three_body_diagnostics():
    g, pos, mass, eps = _three("three_body_eps0.txt")
    vel = golden_io.arr(g, "vel")
    _, pot = orc.accel_pot(pos, mass, eps)
    row = orc.diagnostics(pos, vel, mass, pot)
    assert row[orc.D_K] == g["K"][0][0]
    assert abs(row[orc.D_W] - g["W"][0][0]) < 1e-15
    np.testing.assert_array_equal(row[orc.D_P], g["P"][0])
    np.testing.assert_array_equal(row[orc.D_L], g["L"][0])
    np.testing.assert_array_equal(row[orc.D_COM], g["COM"][0])
    assert row[orc.D_M] == 6.0


def test_three_body_G_and_self_term():
    # G multiplies everything; the self term never enters (eps = 1 would add
    # -m_i/eps to phi_i if it did).
    g, pos, mass, _ = _three("three_body_eps1.txt")
    a1, p1 = orc.accel_pot(pos, mass, 1.0, 1.0)
    a2, p2 = ocpu.accel_pot(pos, mass, 1.0, 2.5)
    np.testing.assert_allclose(a2, 2.5 * a1, rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(p2, 2.5 * p1, rtol=1e-15)


# ---- invariants ---------------------------------------------------------------

def _random_system(n, seed, spread=1.0):
    rng = np.random.default_rng(seed)
    pos = rng.normal(size=(n, 3)) * spread
    mass = rng.uniform(0.5, 2.0, size=n)
    return pos, mass / mass.sum()


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_newton_third_law(eps):
    pos, mass = _random_system(400, 7)
    for f in (orc.accel_pot, ocpu.accel_pot):
        acc, _ = f(pos, mass, eps)
        net = (mass[:, None] * acc).sum(axis=0)
        scale = (mass * np.linalg.norm(acc, axis=1)).sum()
        assert np.linalg.norm(net) <= 1e-14 * scale


def test_scaling_laws():
    pos, mass = _random_system(200, 11)
    eps = 0.03
    a0, p0 = orc.accel_pot(pos, mass, eps)
    a1, p1 = orc.accel_pot(pos, 3.0 * mass, eps)
    np.testing.assert_allclose(a1, 3.0 * a0, rtol=1e-13, atol=1e-14 * np.abs(a0).max())
    lam = 2.0  # a power of two keeps the scaling exact in binary
    a2, p2 = orc.accel_pot(lam * pos, mass, lam * eps)
    np.testing.assert_allclose(a2, a0 / lam ** 2, rtol=0, atol=0)
    np.testing.assert_allclose(p2, p0 / lam, rtol=0, atol=0)


def test_translation_invariance():
    pos, mass = _random_system(300, 13)
    a0, p0 = ocpu.accel_pot(pos, mass, 0.02)
    a1, p1 = ocpu.accel_pot(pos + np.array([1.5, -2.0, 0.75]), mass, 0.02)
    np.testing.assert_allclose(a1, a0, rtol=1e-12, atol=1e-12 * np.abs(a0).max())
    np.testing.assert_allclose(p1, p0, rtol=1e-12)


def test_permutation_equivariance():
    pos, mass = _random_system(257, 17)
    perm = np.random.default_rng(3).permutation(257)
    a0, p0 = orc.accel_pot(pos, mass, 0.01)
    a1, p1 = orc.accel_pot(pos[perm], mass[perm], 0.01)
    np.testing.assert_allclose(a1, a0[perm], rtol=1e-12, atol=1e-13 * np.abs(a0).max())
    np.testing.assert_allclose(p1, p0[perm], rtol=1e-12)


def test_brute_force_numpy_and_c_agree():
    pos, mass = _random_system(23, 19)
    for eps in (0.0, 0.1):
        ab, pb = orc.brute_force(pos.tolist(), mass.tolist(), eps, 1.7)
        an, pn = orc.accel_pot(pos, mass, eps, 1.7)
        ac, pc = ocpu.accel_pot(pos, mass, eps, 1.7)
        for a, p in ((an, pn), (ac, pc)):
            np.testing.assert_allclose(a, ab, rtol=1e-13, atol=1e-14 * np.abs(ab).max())
            np.testing.assert_allclose(p, pb, rtol=1e-13)


def test_c_oracle_targets_and_numpy_agree():
    pos, _, mass = ics.plummer(3000, seed=5)
    tgt = orc.subsample_targets(3000, 500)
    an, pn = orc.accel_pot(pos, mass, 0.01, targets=tgt)
    ac, pc = ocpu.accel_pot(pos, mass, 0.01, targets=tgt)
    assert orc.rel_rms(ac, an) < 1e-13
    assert orc.max_rel(ac, an) < 1e-12
    assert orc.rel_rms(pc, pn) < 1e-14


def test_single_particle_and_empty():
    acc, pot = orc.accel_pot(np.zeros((1, 3)), np.ones(1), 0.0)
    assert np.all(acc == 0) and np.all(pot == 0)
    acc, pot = ocpu.accel_pot(np.zeros((1, 3)), np.ones(1), 0.1)
    assert np.all(acc == 0) and np.all(pot == 0)
    acc, pot = orc.accel_pot(np.zeros((0, 3)), np.zeros(0), 0.1)
    assert acc.shape == (0, 3) and pot.shape == (0,)


# ---- integrator ---------------------------------------------------------------

def test_kdk_harmonic_oscillator_exact_map():
    """Kick-drift-kick on a = -w^2 x is the linear map
    x' = (1 - h^2 w^2 / 2) x + h v,  v' = -w^2 h (1 - h^2 w^2 / 4) x + (1 - h^2 w^2 / 2) v,
    and conserves the shadow energy v^2/2 + w^2 x^2 (1 - (w h / 2)^2) / 2 exactly."""
    w, h, n = 1.3, 0.05, 200
    x0 = np.array([[0.7, -0.2, 0.1]])
    v0 = np.array([[0.0, 0.4, -0.3]])

    def accel(x):
        return -w * w * x, np.zeros(len(x))

    x, v, _, _, _ = orc.kdk(x0, v0, np.ones(1), 0.0, 1.0, h, n, accel=accel, diag=False)
    c = 1.0 - 0.5 * (h * w) ** 2
    m = np.array([[c, h], [-w * w * h * (1.0 - 0.25 * (h * w) ** 2), c]])
    mn = np.linalg.matrix_power(m, n)
    xe = mn[0, 0] * x0 + mn[0, 1] * v0
    ve = mn[1, 0] * x0 + mn[1, 1] * v0
    np.testing.assert_allclose(x, xe, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(v, ve, rtol=1e-12, atol=1e-13)
    shadow = lambda x, v: 0.5 * np.sum(v * v) + 0.5 * w * w * np.sum(x * x) * (1 - (w * h / 2) ** 2)
    assert abs(shadow(x, v) - shadow(x0, v0)) < 1e-14


def _kepler_state(e, s=1.0, m1=0.3, m2=0.7):
    """Two bodies at pericentre of a relative orbit with semi-major axis s,
    eccentricity e, G = 1; centre of mass at rest at the origin."""
    mu = m1 + m2
    rp = s * (1 - e)
    vp = math.sqrt(mu * (1 + e) / rp)
    r = np.array([rp, 0.0, 0.0])
    v = np.array([0.0, vp, 0.0])
    pos = np.stack([-m2 / mu * r, m1 / mu * r])
    vel = np.stack([-m2 / mu * v, m1 / mu * v])
    return pos, vel, np.array([m1, m2]), mu


def _kepler_relative(t, e, s, mu):
    """Closed-form relative position at time t after pericentre (Kepler's equation)."""
    nmean = math.sqrt(mu / s ** 3)
    mm = nmean * t
    ecc = mm if e < 0.8 else math.pi
    for _ in range(100):
        ecc -= (ecc - e * math.sin(ecc) - mm) / (1 - e * math.cos(ecc))
    return np.array([s * (math.cos(ecc) - e), s * math.sqrt(1 - e * e) * math.sin(ecc), 0.0])


@pytest.mark.parametrize("e", [0.0, 0.5])
def test_kepler_two_body(e):
    s = 1.0
    pos, vel, mass, mu = _kepler_state(e, s)
    period = 2 * math.pi * math.sqrt(s ** 3 / mu)
    errs = []
    for nsteps in (2000, 4000):
        dt = 0.37 * period / nsteps
        p, v, _, _, rows = orc.kdk(pos, vel, mass, 0.0, 1.0, dt, nsteps)
        rel = p[1] - p[0]
        ref = _kepler_relative(nsteps * dt, e, s, mu)
        errs.append(np.linalg.norm(rel - ref))
        # Angular momentum is conserved exactly by KDK for a central pair force.
        lz = rows[:, 8]
        assert np.max(np.abs(lz - lz[0])) <= 1e-13 * abs(lz[0])
        # Energy error stays bounded (no secular trend at this step).
        assert np.max(orc.energy_drift(rows)) < 20 * (2 * math.pi * dt / period) ** 2 / (1 - e) ** 3
    # Second order: halving dt cuts the phase error by four.
    assert errs[0] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_c_kdk_matches_numpy_kdk():
    pos, vel, mass = ics.plummer(200, seed=9)
    p1, v1, a1, _, _ = orc.kdk(pos, vel, mass, 0.02, 1.0, 1.0 / 128, 5, diag=False)
    p2, v2, a2, _ = ocpu.kdk(pos, vel, mass, 0.02, 1.0, 1.0 / 128, 5)
    np.testing.assert_allclose(p2, p1, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(v2, v1, rtol=1e-12, atol=1e-14)
    assert orc.rel_rms(a2, a1) < 1e-12


def test_time_reversibility():
    pos, vel, mass = ics.plummer(64, seed=21)
    eps, dt, n = 0.05, 1.0 / 64, 10
    p, v, a, _, _ = orc.kdk(pos, vel, mass, eps, 1.0, dt, n, diag=False)
    p, v, _, _, _ = orc.kdk(p, -v, mass, eps, 1.0, dt, n, acc=a, diag=False)
    np.testing.assert_allclose(p, pos, rtol=0, atol=1e-12 * np.abs(pos).max())
    np.testing.assert_allclose(-v, vel, rtol=0, atol=1e-12 * np.abs(vel).max())


def test_momentum_conserved_under_kdk():
    pos, vel, mass = ics.plummer(300, seed=23)
    _, _, _, _, rows = orc.kdk(pos, vel, mass, 0.01, 1.0, 1.0 / 128, 10)
    p = rows[:, 3:6]
    l = rows[:, 6:9]
    assert np.abs(p).max() < 1e-14
    assert np.abs(l - l[0]).max() < 1e-13 * np.linalg.norm(l[0]) + 1e-15


# ---- Plummer sphere limits ----------------------------------------------------

def test_plummer_potential_energy_limit():
    """E[W_N] = -(3 pi / 32)(1 - 1/N) G M^2 / a for N equal masses. The
    sampling scatter of W is about 0.78/sqrt(N) relative; 16 independent
    spheres are averaged and checked at four standard errors plus the
    softening bias (about 2.3e-4 at eps = 0.01)."""
    n = 1024
    ws = []
    for seed in range(16):
        pos, _, mass = ics.plummer(n, seed=100 + seed)
        _, pot = ocpu.accel_pot(pos, mass, 0.01)
        ws.append(0.5 * np.sum(mass * pot))
    expect = -(3 * math.pi / 32) * (1 - 1 / n)
    tol = 4 * 0.78 / math.sqrt(n) / 4 + 2.3e-4
    assert abs(np.mean(ws) / expect - 1) < tol


def test_plummer_virial_and_gauss_law():
    """Virial ratio 2K/|W| ~ 1 for a sampled Plummer sphere, and Gauss's law:
    averaged over a sphere of radius r the radial field is -G M(<r) / r^2,
    with M(<r) the sampled mass inside r. Particles in a shell sample that
    sphere at random directions, so their mean radial acceleration matches
    -M(<r_i)/r_i^2 within a few standard errors (softening at eps = 1e-3
    changes the field by ~ eps^2/r^2, far below that)."""
    n = 8192
    pos, vel, mass = ics.plummer(n, seed=31)
    acc, pot = ocpu.accel_pot(pos, mass, 0.001)
    k = 0.5 * np.sum(mass * np.sum(vel * vel, axis=1))
    w = 0.5 * np.sum(mass * pot)
    assert abs(2 * k / abs(w) - 1) < 4 * 1.0 / math.sqrt(n) + 0.01
    r = np.linalg.norm(pos, axis=1)
    order = np.argsort(r)
    menc = np.empty(n)
    menc[order] = np.cumsum(mass[order]) - mass[order]
    ar = np.sum(acc * pos, axis=1) / r
    edges = np.array([0.2, 0.4, 0.6, 0.9, 1.3, 2.0, 3.5])
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (r >= lo) & (r < hi)
        gauss = -menc[sel] / r[sel] ** 2
        dev = ar[sel] - gauss
        se = dev.std(ddof=1) / math.sqrt(sel.sum())
        assert abs(dev.mean()) < 4 * se, (lo, hi)
        # and the field is attractive and of the right size
        assert 0.9 < ar[sel].mean() / gauss.mean() < 1.1


# ---- error metrics ------------------------------------------------------------

def test_error_metrics():
    ref = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    x = ref + np.array([[0.0, 1e-3, 0.0], [0.0, 0.0, 0.0]])
    assert math.isclose(orc.rel_rms(x, ref), 1e-3 / math.sqrt(5), rel_tol=1e-12)
    assert math.isclose(orc.max_rel(x, ref), 1e-3, rel_tol=1e-12)
    typ = math.sqrt((1 + 4) / 2)
    assert math.isclose(orc.paper_metric(x, ref), 1e-3 / typ, rel_tol=1e-12)
    np.testing.assert_array_equal(orc.subsample_targets(10, 4), [0, 2, 5, 7])
    np.testing.assert_array_equal(orc.subsample_targets(3, 4), [0, 1, 2])
