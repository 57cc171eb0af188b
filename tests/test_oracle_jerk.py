"""Pins of the oracle's jerk and Hermite integrator.

The jerk is pinned by the hand-worked three-body values (rational numbers),
by its definition as the time derivative of the acceleration (a centred
finite difference along straight-line motion converges to it at second
order), and by Newton's third law; the Hermite scheme by its fourth-order
convergence on a Kepler orbit against Kepler's equation.
"""
import math

import numpy as np
import pytest

from oracle import cpu as ocpu
from oracle import oracle as orc
from paper_2509_19294_amd import ics
from tests import golden_io
from tests.test_oracle_pins import _kepler_relative, _kepler_state


@pytest.fixture(scope="module", autouse=True)
def _build_c_oracle():
    ocpu.build(force=False)


@pytest.mark.parametrize("impl", ["numpy", "c", "brute"])
def test_three_body_jerk_hand_worked(impl):
    g = golden_io.load("three_body_eps0.txt")
    pos, vel, mass = golden_io.arr(g, "pos"), golden_io.arr(g, "vel"), golden_io.arr(g, "mass")[0]
    if impl == "brute":
        jerk = orc.brute_force_jerk(pos.tolist(), vel.tolist(), mass.tolist())
    else:
        f = orc.accel_jerk if impl == "numpy" else ocpu.accel_jerk
        acc, jerk, pot = f(pos, vel, mass, 0.0, 1.0)
        np.testing.assert_allclose(acc, golden_io.arr(g, "acc"), rtol=0, atol=4e-16)
        np.testing.assert_allclose(pot, golden_io.arr(g, "pot")[0], rtol=0, atol=4e-16)
    np.testing.assert_allclose(jerk, golden_io.arr(g, "jerk"), rtol=0, atol=4e-16)


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_jerk_is_the_time_derivative_of_acceleration(eps):
    """Along x(t) = x + v t, (a(x + v h) - a(x - v h)) / 2h -> jerk as O(h^2)."""
    pos, vel, mass = ics.plummer(64, seed=44)
    _, jerk, _ = orc.accel_jerk(pos, vel, mass, eps)
    errs = []
    for h in (1e-3, 5e-4):
        ap, _ = orc.accel_pot(pos + h * vel, mass, eps)
        am, _ = orc.accel_pot(pos - h * vel, mass, eps)
        fd = (ap - am) / (2 * h)
        errs.append(np.linalg.norm(fd - jerk) / np.linalg.norm(jerk))
    assert errs[1] < 1e-4
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_jerk_newton_third_law_and_c_agreement():
    pos, vel, mass = ics.plummer(300, seed=45)
    mass = mass * np.random.default_rng(1).uniform(0.5, 2.0, size=300)
    a, j, p = orc.accel_jerk(pos, vel, mass, 0.01)
    net = (mass[:, None] * j).sum(axis=0)
    assert np.linalg.norm(net) <= 1e-13 * (mass * np.linalg.norm(j, axis=1)).sum()
    a2, j2, p2 = ocpu.accel_jerk(pos, vel, mass, 0.01)
    assert orc.rel_rms(a2, a) < 1e-13 and orc.rel_rms(j2, j) < 1e-13 and orc.rel_rms(p2, p) < 1e-14
    tgt = orc.subsample_targets(300, 37)
    a3, j3, _ = ocpu.accel_jerk(pos, vel, mass, 0.01, targets=tgt)
    assert orc.rel_rms(j3, j[tgt]) < 1e-13
    # the acceleration part matches the plain force oracle
    a4, p4 = orc.accel_pot(pos, mass, 0.01)
    assert orc.rel_rms(a, a4) < 1e-14 and orc.rel_rms(p, p4) < 1e-15


def test_hermite_kepler_fourth_order():
    e, s = 0.5, 1.0
    pos, vel, mass, mu = _kepler_state(e, s)
    period = 2 * math.pi * math.sqrt(s ** 3 / mu)
    errs = []
    for nsteps in (400, 800):
        dt = 0.37 * period / nsteps
        p, v, _, _, _, rows = orc.hermite(pos, vel, mass, 0.0, 1.0, dt, nsteps)
        ref = _kepler_relative(nsteps * dt, e, s, mu)
        errs.append(np.linalg.norm((p[1] - p[0]) - ref))
    assert errs[0] < 1e-5
    assert 12.0 < errs[0] / errs[1] < 20.0


def test_hermite_beats_leapfrog_at_equal_cost():
    pos, vel, mass = ics.plummer(64, seed=46)
    eps, dt, n = 0.05, 1.0 / 64, 32
    _, _, _, _, _, rows_h = orc.hermite(pos, vel, mass, eps, 1.0, dt, n)
    _, _, _, _, rows_k = orc.kdk(pos, vel, mass, eps, 1.0, dt, n)
    assert orc.energy_drift(rows_h).max() < orc.energy_drift(rows_k).max()
