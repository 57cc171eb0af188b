"""Seeded synthetic initial conditions for the direct-summation N-body path.

This module only draws inputs. It holds none of the force, integrator or
diagnostic arithmetic, so both the GPU path and the FP64 oracle can take their
inputs from here without sharing any of the method.

The paper never states its initial conditions (Section 4 only gives the
particle count), so the standard stellar-dynamics workloads below stand in:

* ``plummer``: equal-mass Plummer sphere in units G = M = a = 1, sampled with
  the Aarseth, Henon and Wielen (1974) method: radius from the inverted
  cumulative mass profile, speed by rejection sampling of the isotropic
  distribution function, isotropic directions, then the centre of mass moved
  to the origin.
* ``kroupa_masses``: the two-segment Kroupa (2001) mass function on
  [0.08, 100], slopes 1.3 below 0.5 and 2.3 above, normalised to total mass 1.
* ``ensemble``: many independent Plummer clusters of log-uniform size, all
  centred on the origin (the clusters do not interact, so any leakage between
  them shows up as a large error).

All arrays are float64 and C-contiguous. The draw order is fixed, so a seed
gives the same system on every machine that runs numpy's PCG64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "plummer",
    "kroupa_masses",
    "plummer_kroupa",
    "ensemble",
    "Ensemble",
    "WORKLOADS",
    "workload",
]

# Rejection envelope for g(q) = q^2 (1 - q^2)^(7/2); its maximum is
# g(1/3) = (1/9)(8/9)^(7/2) ~= 0.0921.
_Q_ENVELOPE = 0.1


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere: cos(theta) ~ U(-1, 1), phi ~ U(0, 2 pi)."""
    cth = 2.0 * rng.random(n) - 1.0
    phi = 2.0 * math.pi * rng.random(n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], axis=1)


def _plummer_q(rng: np.random.Generator, n: int) -> np.ndarray:
    """Draw q = v / v_esc from g(q) = q^2 (1 - q^2)^(7/2) by rejection.

    Rounds are vectorised: each round draws a (q, y) pair for every particle
    still waiting, and a particle keeps the first pair it accepts.
    """
    q = np.empty(n)
    pending = np.arange(n)
    while pending.size:
        qq = rng.random(pending.size)
        yy = _Q_ENVELOPE * rng.random(pending.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[pending[ok]] = qq[ok]
        pending = pending[~ok]
    return q


def _sample_plummer_phase(rng: np.random.Generator, n: int):
    x = rng.random(n)
    # x = M(<r) = r^3 / (1 + r^2)^(3/2) inverted; x == 0 gives r == 0.
    with np.errstate(divide="ignore"):
        r = 1.0 / np.sqrt(x ** (-2.0 / 3.0) - 1.0)
    pos = r[:, None] * _isotropic(rng, n)
    q = _plummer_q(rng, n)
    speed = q * math.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    vel = speed[:, None] * _isotropic(rng, n)
    return pos, vel


def _to_com_frame(pos, mass, vel):
    mt = mass.sum()
    pos -= (mass[:, None] * pos).sum(axis=0) / mt
    vel -= (mass[:, None] * vel).sum(axis=0) / mt


def plummer(n: int, seed=0, rng: np.random.Generator | None = None):
    """Equal-mass Plummer sphere (G = M = a = 1).

    Returns ``(pos, vel, mass)`` with shapes (n, 3), (n, 3), (n,), float64.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    if rng is None:
        rng = np.random.default_rng(seed)
    pos, vel = _sample_plummer_phase(rng, n)
    mass = np.full(n, 1.0 / n)
    _to_com_frame(pos, mass, vel)
    return np.ascontiguousarray(pos), np.ascontiguousarray(vel), mass


# Kroupa (2001): dN/dm proportional to m^-1.3 on [0.08, 0.5) and m^-2.3 on
# [0.5, 100], continuous at 0.5.
KROUPA_BREAKS = (0.08, 0.5, 100.0)
KROUPA_SLOPES = (1.3, 2.3)


def _kroupa_segment_weights():
    (m0, m1, m2), (a1, a2) = KROUPA_BREAKS, KROUPA_SLOPES
    k2 = m1 ** (a2 - a1)  # continuity at m1 with k1 = 1
    w1 = (m0 ** (1 - a1) - m1 ** (1 - a1)) / (a1 - 1)
    w2 = k2 * (m1 ** (1 - a2) - m2 ** (1 - a2)) / (a2 - 1)
    return w1 / (w1 + w2), w2 / (w1 + w2)


def _powerlaw_inverse(u, lo, hi, alpha):
    e = 1.0 - alpha
    return (lo ** e + u * (hi ** e - lo ** e)) ** (1.0 / e)


def kroupa_masses(n: int, rng: np.random.Generator) -> np.ndarray:
    """Raw Kroupa masses in solar units: a segment by its number fraction,
    then inversion of that segment's cumulative distribution."""
    f_low, _ = _kroupa_segment_weights()
    useg = rng.random(n)
    uinv = rng.random(n)
    (m0, m1, m2), (a1, a2) = KROUPA_BREAKS, KROUPA_SLOPES
    low = useg < f_low
    m = np.where(low, _powerlaw_inverse(uinv, m0, m1, a1), _powerlaw_inverse(uinv, m1, m2, a2))
    return m


def plummer_kroupa(n: int, seed=3):
    """Plummer positions and velocities (equal-mass sampler) with Kroupa
    masses drawn afterwards, normalised to total mass 1, then moved to the
    mass-weighted centre-of-mass frame."""
    rng = np.random.default_rng(seed)
    pos, vel = _sample_plummer_phase(rng, n)
    mass = kroupa_masses(n, rng)
    mass = mass / mass.sum()
    _to_com_frame(pos, mass, vel)
    return np.ascontiguousarray(pos), np.ascontiguousarray(vel), mass


@dataclass
class Ensemble:
    pos: np.ndarray        # (n_total, 3)
    vel: np.ndarray        # (n_total, 3)
    mass: np.ndarray       # (n_total,)
    offsets: np.ndarray    # int64 (K + 1,), cluster k owns [offsets[k], offsets[k+1])
    eps: np.ndarray        # float64 (K,)
    sizes: np.ndarray      # int64 (K,)


def ensemble(k: int = 512, seed: int = 2, n_min: int = 256, n_max: int = 8192,
             eps_scale: float = 4.0) -> Ensemble:
    """K independent Plummer clusters (each M = 1, a = 1, at the origin).

    ``SeedSequence(seed).spawn(k + 1)``: child 0 draws the sizes
    N_k = clip(round(exp(U(ln n_min, ln n_max))), n_min, n_max); child k + 1
    samples cluster k. Softening eps_k = eps_scale / N_k.
    """
    children = np.random.SeedSequence(seed).spawn(k + 1)
    r0 = np.random.default_rng(children[0])
    u = r0.uniform(math.log(n_min), math.log(n_max), size=k)
    sizes = np.clip(np.rint(np.exp(u)), n_min, n_max).astype(np.int64)
    offsets = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    pos = np.empty((offsets[-1], 3))
    vel = np.empty((offsets[-1], 3))
    mass = np.empty(offsets[-1])
    for c in range(k):
        p, v, m = plummer(int(sizes[c]), rng=np.random.default_rng(children[c + 1]))
        s, e = offsets[c], offsets[c + 1]
        pos[s:e], vel[s:e], mass[s:e] = p, v, m
    eps = eps_scale / sizes.astype(np.float64)
    return Ensemble(pos, vel, mass, offsets, eps, sizes)


# The five synthetic workloads: size, seed, softening, step and step count.
WORKLOADS = {
    "plummer_1k": dict(n=1024, seed=0, eps=0.01, dt=1.0 / 128, steps=10, masses="equal"),
    "plummer_64k": dict(n=65536, seed=1, eps=0.005, dt=1.0 / 256, steps=10, masses="equal"),
    "plummer_256k": dict(n=262144, seed=4, eps=0.002, dt=1.0 / 512, steps=1000, masses="equal"),
    "ensemble_512": dict(k=512, seed=2, dt=1.0 / 256, steps=100),
    "kroupa_1m": dict(n=1048576, seed=3, eps=0.001, dt=1.0 / 1024, steps=10, masses="kroupa"),
    # The paper's representative run (Section 4): 102,400 particles, ten steps.
    "plummer_102k": dict(n=102400, seed=5, eps=0.005, dt=1.0 / 256, steps=10, masses="equal"),
}


def workload(name: str):
    """Return ``(pos, vel, mass, spec)`` for a named single-system workload,
    or ``(Ensemble, spec)`` for the ensemble."""
    spec = dict(WORKLOADS[name])
    if name == "ensemble_512":
        return ensemble(spec["k"], spec["seed"]), spec
    if spec["masses"] == "kroupa":
        p, v, m = plummer_kroupa(spec["n"], spec["seed"])
    else:
        p, v, m = plummer(spec["n"], spec["seed"])
    return p, v, m, spec
