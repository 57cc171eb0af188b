"""Randomised tiny systems on the GPU against the FP64 oracle.

Hypothesis draws the shape of each case: particle count (tile boundaries
and arbitrary sizes), length scale, translation, softening (zero
included), G, mass spread (zero masses included), the arithmetic form and
the configuration and grid j-split the dispatch is forced to. The draws are
derandomised, so every run checks the same cases.

Random configurations can be ill-conditioned (a near-zero net force from
large opposing pair forces, an unsoftened close pair), where no relative
bound on the result holds. Each particle is therefore checked against a
bound on its own arithmetic instead: the error of a_i stays below
C u sum_j |f_ij| (u = 2^-24, f_ij the pair terms), the potential's within C u times the sum
of its terms (they share one sign; the softened self term, which the
kernels sum and then subtract, included), and the jerk's within C u times the sum of its
terms' magnitudes, widened by the velocity spread its velocity frames
round against. C = 256: the largest error seen over these cases is about
23 u times its sum (the potential's; 15 u for the acceleration, 2.5 u for
the jerk), and a worst case for FP32 sums over the longest (1024-source)
tile would be about 1024 u. A wrong index, a dropped or doubled term, or a
wrong sign moves a result by a whole pair term, which these bounds resolve
down to about 1/65000 of the sum. The plain form rounds its inputs to FP32 (as
packed), so its reference is the oracle on the rounded coordinates and
masses; the compensated form is checked against the exact inputs.
"""
import math

import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, assume, given, settings
from hypothesis import strategies as st

from oracle import oracle as orc
from paper_2509_19294_amd import nbody

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
C = 256.0
DEV = "cuda:0"
SETTINGS = dict(deadline=None, derandomize=True, database=None,
                suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
SIZES = st.one_of(st.sampled_from([1, 2, 3, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257]),
                  st.integers(1, 300))


WORST = {}  # largest error / (C u sum) seen per quantity, printed at the end


@pytest.fixture(scope="module", autouse=True)
def _setup():
    nbody.load()
    nbody.tune_reset()
    yield
    nbody.tune_reset()
    print("largest error over its bound:", {k: float(f"{v:.3g}") for k, v in WORST.items()}, flush=True)


def _note(key, err, scale):
    r = float(np.max(err / np.maximum(C * U * scale, 1e-300))) if len(err) else 0.0
    WORST[key] = max(WORST.get(key, 0.0), r)


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def system(seed, n, scale, shift, mass_sigma, zero_frac):
    """Seeded positions (uniform in a cube of side `scale`, or two clumps),
    masses (log-normal, some zero), all moved by `shift` along (1, -2, 3)."""
    rng = np.random.default_rng(seed)
    if seed % 2 == 0 or n < 4:
        pos = rng.uniform(-0.5, 0.5, (n, 3)) * scale
    else:
        half = n // 2
        pos = np.concatenate([rng.normal(0.0, 0.05, (half, 3)),
                              rng.normal(0.0, 0.2, (n - half, 3)) + 0.7]) * scale
    pos = pos + shift * np.array([1.0, -2.0, 3.0])
    mass = rng.lognormal(0.0, mass_sigma, n) / n
    mass[rng.uniform(size=n) < zero_frac] = 0.0
    return pos, mass


def rounded(pos, mass):
    """The inputs as the plain form packs them (FP32), back in float64."""
    return pos.astype(np.float32).astype(np.float64), mass.astype(np.float32).astype(np.float64)


def pair_sums(pos, mass, eps, G, vel=None, vspread=0.0):
    """Per particle: sum_j |f_ij| of the acceleration terms, |phi_i|'s terms'
    sum, and (with velocities) the jerk terms' magnitudes plus the rounding
    spread of the velocity frames."""
    d = pos[None, :, :] - pos[:, None, :]
    q = np.einsum("ijk,ijk->ij", d, d) + eps * eps
    np.fill_diagonal(q, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / np.sqrt(q)
    sa = G * (mass[None, :] * np.sqrt(np.einsum("ijk,ijk->ij", d, d)) * inv ** 3).sum(1)
    # the softened self pair's m_i / eps enters the FP32 potential sums
    # before the epilogue takes it out again, so its rounding counts too
    sp = G * ((mass[None, :] * inv).sum(1) + (mass / eps if eps > 0 else 0.0))
    if vel is None:
        return sa, sp
    w = np.linalg.norm(vel[None, :, :] - vel[:, None, :], axis=2)
    sj = G * (mass[None, :] * 4.0 * (w + vspread) * inv ** 3).sum(1)
    return sa, sp, sj


def check_bounds(a, p, ref_a, ref_p, sa, sp, what):
    ea = np.linalg.norm(a - ref_a, axis=1)
    ep = np.abs(p - ref_p)
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(p)), what
    _note("acc", ea, sa)
    _note("pot", ep, sp)
    assert np.all(ea <= C * U * sa + 1e-300), (what, "acc", float(np.max(ea / np.maximum(sa, 1e-300))))
    assert np.all(ep <= C * U * sp + 1e-300), (what, "pot", float(np.max(ep / np.maximum(sp, 1e-300))))


def no_coincident(pos):
    """Every pair apart (the unsoftened self-pair guard keys on r = 0)."""
    if len(pos) < 2:
        return True
    d = np.linalg.norm(pos[None, :, :] - pos[:, None, :], axis=2)
    np.fill_diagonal(d, np.inf)
    return bool(d.min() > 0)


@settings(max_examples=300, **SETTINGS)
@given(seed=st.integers(0, 2 ** 31 - 1), n=SIZES, scale=st.sampled_from([1e-3, 1.0, 1e3]),
       shift=st.sampled_from([0.0, 1.0, 1e3]), eps_rel=st.sampled_from([0.0, 1e-3, 0.05, 1.0]),
       G=st.floats(0.5, 2.0), mass_sigma=st.sampled_from([0.0, 1.0, 3.0]),
       zero_frac=st.sampled_from([0.0, 0.1]), variant=st.sampled_from(["plain", "comp"]),
       cfg_pick=st.integers(0, 10 ** 6), split=st.sampled_from([1, 2, 3, 8]))
def test_random_systems_any_configuration(seed, n, scale, shift, eps_rel, G, mass_sigma, zero_frac,
                                          variant, cfg_pick, split):
    pos, mass = system(seed, n, scale, shift * scale, mass_sigma, zero_frac)
    eps = eps_rel * scale
    ref_pos, ref_mass = (rounded(pos, mass) if variant == "plain" else (pos, mass))
    assume(eps > 0 or no_coincident(ref_pos))
    cfg = cfg_pick % len(nbody.tune_configs(variant))
    cls = int(math.floor(math.log2(n)))
    nbody.tune_set(variant, cls, cfg, split)
    try:
        acc, pot = nbody.accel(T(pos), T(mass), eps, G, variant)
        torch.cuda.synchronize()
    finally:
        nbody.tune_set(variant, cls, -1)
    ref_a, ref_p = orc.accel_pot(ref_pos, ref_mass, eps, G)
    sa, sp = pair_sums(ref_pos, ref_mass, eps, G)
    check_bounds(acc.cpu().numpy(), pot.cpu().numpy(), ref_a, ref_p, sa, sp,
                 (variant, n, cfg, split, seed, scale, shift, eps_rel))


@settings(max_examples=60, **SETTINGS)
@given(seed=st.integers(0, 2 ** 31 - 1),
       sizes=st.lists(st.one_of(st.sampled_from([0, 1, 2, 63, 64, 65]), st.integers(0, 400)),
                      min_size=1, max_size=10),
       eps_rel=st.lists(st.sampled_from([0.0, 1e-3, 0.02, 0.5]), min_size=10, max_size=10),
       G=st.floats(0.5, 2.0), variant=st.sampled_from(["plain", "comp"]))
def test_random_batched_plans(seed, sizes, eps_rel, G, variant):
    """Clusters of random sizes (empty ones included) at random places, each
    checked against its own oracle; a source from another cluster would
    move a result by far more than the bound."""
    rng = np.random.default_rng(seed)
    parts, masses = [], []
    for k, nk in enumerate(sizes):
        p, m = system(seed + k, nk, 1.0, 0.0, 1.0, 0.0) if nk > 0 else (np.zeros((0, 3)), np.zeros(0))
        parts.append(p + rng.uniform(-50.0, 50.0, 3))
        masses.append(m)
    pos, mass = np.concatenate(parts), np.concatenate(masses)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eps_k = np.array(eps_rel[:len(sizes)], dtype=np.float64)
    ref_pos, ref_mass = (rounded(pos, mass) if variant == "plain" else (pos, mass))
    for k in range(len(sizes)):
        s, e = int(offs[k]), int(offs[k + 1])
        assume(eps_k[k] > 0 or no_coincident(ref_pos[s:e]))
    plan = nbody.Plan(offs, variant)
    try:
        if len(mass) == 0:
            return
        acc, pot = plan.accel(T(pos), T(mass), T(eps_k), G)
        torch.cuda.synchronize()
    finally:
        plan.close()
    a, p = acc.cpu().numpy(), pot.cpu().numpy()
    for k in range(len(sizes)):
        s, e = int(offs[k]), int(offs[k + 1])
        if e == s:
            continue
        ref_a, ref_p = orc.accel_pot(ref_pos[s:e], ref_mass[s:e], eps_k[k], G)
        sa, sp = pair_sums(ref_pos[s:e], ref_mass[s:e], eps_k[k], G)
        check_bounds(a[s:e], p[s:e], ref_a, ref_p, sa, sp, (variant, k, sizes, seed))


@settings(max_examples=150, **SETTINGS)
@given(seed=st.integers(0, 2 ** 31 - 1), n=SIZES, shift=st.sampled_from([0.0, 1.0, 1e3]),
       bulk=st.sampled_from([0.0, 1.0, 30.0]), eps_rel=st.sampled_from([0.0, 1e-3, 0.05]),
       G=st.floats(0.5, 2.0), variant=st.sampled_from(["plain", "comp"]),
       shape_pick=st.integers(0, 10 ** 6), split=st.sampled_from([0, 1, 2, 8]))
def test_random_systems_acceleration_and_jerk(seed, n, shift, bulk, eps_rel, G, variant, shape_pick, split):
    pos, mass = system(seed, n, 1.0, shift, 1.0, 0.1)
    rng = np.random.default_rng(seed + 1)
    vel = rng.normal(0.0, 1.0, (n, 3)) + bulk * np.array([1.0, 0.5, -0.25])
    eps = eps_rel
    ref_pos, ref_mass = (rounded(pos, mass) if variant == "plain" else (pos, mass))
    assume(eps > 0 or no_coincident(ref_pos))
    shape = shape_pick % len(nbody.jerk_shapes(variant))
    nbody.tune_jerk_set(variant, shape, split)
    try:
        acc, jerk, pot = nbody.accel_jerk(T(pos), T(vel), T(mass), eps, G, variant)
        torch.cuda.synchronize()
    finally:
        nbody.tune_jerk_set(variant, -1)
    ref_a, ref_j, ref_p = orc.accel_jerk(ref_pos, vel, ref_mass, eps, G)
    # velocity frames (a particle's velocity) round relative velocities
    # against at most twice the largest distance from the mean velocity
    spread = 2.0 * float(np.max(np.linalg.norm(vel - vel.mean(0), axis=1))) if n > 1 else 0.0
    sa, sp, sj = pair_sums(ref_pos, ref_mass, eps, G, vel=vel, vspread=spread)
    what = (variant, n, shape, split, seed, shift, bulk, eps_rel)
    check_bounds(acc.cpu().numpy(), pot.cpu().numpy(), ref_a, ref_p, sa, sp, what)
    j = jerk.cpu().numpy()
    ej = np.linalg.norm(j - ref_j, axis=1)
    assert np.all(np.isfinite(j)), what
    _note("jerk", ej, sj)
    assert np.all(ej <= C * U * sj + 1e-300), (what, "jerk", float(np.max(ej / np.maximum(sj, 1e-300))))


def _vec_err(x, ref):
    return np.linalg.norm(x - ref, axis=1)


@settings(max_examples=40, **SETTINGS)
@given(seed=st.integers(0, 2 ** 31 - 1), n=st.integers(2, 200), eps_rel=st.sampled_from([1e-3, 0.05, 0.5]),
       G=st.floats(0.5, 2.0), dt=st.sampled_from([1.0 / 64, 1.0 / 256, 1.0 / 1024]),
       variant=st.sampled_from(["plain", "comp"]), cfg_pick=st.integers(0, 10 ** 6),
       split=st.sampled_from([1, 3, 8]))
def test_random_kdk_steps_from_the_gpu_state(seed, n, eps_rel, G, dt, variant, cfg_pick, split):
    """Three KDK steps, one call each, under a forced random configuration.
    Each step is checked from the state the GPU itself held before it: the
    drift is the FP64 update of that state, the new accelerations meet the
    force bound, and the closing kick differs from the oracle's only by
    dt/2 times that force error."""
    pos, mass = system(seed, n, 1.0, 0.0, 1.0, 0.1)
    rng = np.random.default_rng(seed + 7)
    vel = rng.normal(0.0, 0.3, (n, 3))
    eps = eps_rel
    cls = int(math.floor(math.log2(n)))
    tp, tv, tm = T(pos), T(vel), T(mass)
    nbody.tune_set(variant, cls, cfg_pick % len(nbody.tune_configs(variant)), split)
    try:
        acc, _ = nbody.accel(tp, tm, eps, G, variant)
        for step in range(3):
            x0, v0, a0 = tp.cpu().numpy(), tv.cpu().numpy(), acc.cpu().numpy()
            diag = nbody.step(tp, tv, acc, tm, eps, G, dt, 1, variant)
            torch.cuda.synchronize()
            x1, v1, a1 = tp.cpu().numpy(), tv.cpu().numpy(), acc.cpu().numpy()
            vh = v0 + 0.5 * dt * a0
            xr = x0 + dt * vh
            scale_x = np.abs(xr).max() + 1e-300
            assert np.abs(x1 - xr).max() <= 1e-14 * scale_x, (step, "drift")
            rp, rm = (rounded(x1, mass) if variant == "plain" else (x1, mass))
            ra, rpot = orc.accel_pot(rp, rm, eps, G)
            sa, sp = pair_sums(rp, rm, eps, G)
            ea = _vec_err(a1, ra)
            _note("kdk acc", ea, sa)
            assert np.all(ea <= C * U * sa + 1e-300), (step, variant, "acc")
            ev = _vec_err(v1, vh + 0.5 * dt * ra)
            assert np.all(ev <= 0.5 * dt * C * U * sa + 1e-14 * (np.abs(vh).max() + 1e-300)), (step, "kick")
            k = 0.5 * float(np.sum(mass * np.einsum("ik,ik->i", v1, v1)))
            np.testing.assert_allclose(diag[0, nbody.DIAG["K"]].item(), k, rtol=1e-12)
    finally:
        nbody.tune_set(variant, cls, -1)


@settings(max_examples=30, **SETTINGS)
@given(seed=st.integers(0, 2 ** 31 - 1), n=st.integers(2, 200), eps_rel=st.sampled_from([1e-3, 0.05, 0.5]),
       G=st.floats(0.5, 2.0), dt=st.sampled_from([1.0 / 64, 1.0 / 256, 1.0 / 1024]),
       variant=st.sampled_from(["plain", "comp"]), shape_pick=st.integers(0, 10 ** 6),
       split=st.sampled_from([0, 1, 8]))
def test_random_hermite_steps_from_the_gpu_state(seed, n, eps_rel, G, dt, variant, shape_pick, split):
    """Two Hermite steps, one call each, under a forced random acceleration
    + jerk shape. From the GPU's own state before each step: the predicted
    state is the FP64 predictor; the corrector's result differs from the one
    built on the oracle's acceleration and jerk at that predicted state by at
    most what the force and jerk bounds carry through the corrector."""
    pos, mass = system(seed, n, 1.0, 0.0, 1.0, 0.1)
    rng = np.random.default_rng(seed + 11)
    vel = rng.normal(0.0, 0.3, (n, 3))
    eps = eps_rel
    tp, tv, tm = T(pos), T(vel), T(mass)
    nbody.tune_jerk_set(variant, shape_pick % len(nbody.jerk_shapes(variant)), split)
    try:
        acc, jerk, _ = nbody.accel_jerk(tp, tv, tm, eps, G, variant)
        for step in range(2):
            x0, v0 = tp.cpu().numpy(), tv.cpu().numpy()
            a0, j0 = acc.cpu().numpy(), jerk.cpu().numpy()
            nbody.step_hermite(tp, tv, acc, jerk, tm, eps, G, dt, 1, variant)
            torch.cuda.synchronize()
            x1, v1 = tp.cpu().numpy(), tv.cpu().numpy()
            a1, j1 = acc.cpu().numpy(), jerk.cpu().numpy()
            xp = x0 + dt * v0 + (dt * dt / 2.0) * a0 + (dt ** 3 / 6.0) * j0
            vp = v0 + dt * a0 + (dt * dt / 2.0) * j0
            rp, rm = (rounded(xp, mass) if variant == "plain" else (xp, mass))
            ra, rj, _ = orc.accel_jerk(rp, vp, rm, eps, G)
            spread = 2.0 * float(np.max(np.linalg.norm(vp - vp.mean(0), axis=1)))
            sa, sp, sj = pair_sums(rp, rm, eps, G, vel=vp, vspread=spread)
            # position rounding of the plain form moves the predicted state by
            # u |x| per coordinate, which the oracle on rounded inputs absorbs
            da, dj = C * U * sa, C * U * sj
            ea, ej = _vec_err(a1, ra), _vec_err(j1, rj)
            _note("hermite acc", ea, sa)
            _note("hermite jerk", ej, sj)
            assert np.all(ea <= da + 1e-300), (step, variant, "acc")
            assert np.all(ej <= dj + 1e-300), (step, variant, "jerk")
            vr = v0 + (dt / 2.0) * (a0 + ra) + (dt * dt / 12.0) * (j0 - rj)
            xr = x0 + (dt / 2.0) * (v0 + vr) + (dt * dt / 12.0) * (a0 - ra)
            dv = (dt / 2.0) * da + (dt * dt / 12.0) * dj
            dx = (dt / 2.0) * dv + (dt * dt / 12.0) * da
            fv = 1e-14 * (np.abs(vr).max() + 1e-300)
            fx = 1e-14 * (np.abs(xr).max() + 1e-300)
            assert np.all(_vec_err(v1, vr) <= dv + fv), (step, "corrector v")
            assert np.all(_vec_err(x1, xr) <= dx + fx), (step, "corrector x")
    finally:
        nbody.tune_jerk_set(variant, -1)
