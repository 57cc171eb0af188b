"""FP64 CPU oracle for the direct-summation N-body hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this module;
only the tests, the smoke check and the benchmark's CPU-baseline leg do. It
shares no code with the GPU path.

What it computes, and where that comes from:

* Pair sum (Section 3, the force equation): the force on particle i is the
  sum over every other particle j != i of G m_i m_j (r_j - r_i) / r_ij^3.
  Dividing by m_i gives the acceleration. With Plummer softening eps the
  distance cubed becomes (r_ij^2 + eps^2)^(3/2); eps = 0 is the paper's
  unsoftened sum exactly. The potential is phi_i = -G sum_{j != i} m_j /
  (r_ij^2 + eps^2)^(1/2). The self term is excluded by index, in both sums.
* The paper's validation reference (Section 3, correctness paragraph) is a
  naive double-precision brute force over all pairs; this is that, in FP64.
* Kick-drift-kick leapfrog (the integrator the GPU path drives; the paper
  does not name its own): with a = A(x) known at the start of a step,
  v += dt/2 a; x += dt v; a = A(x); v += dt/2 a.
* Diagnostics: K = 1/2 sum m |v|^2, W = 1/2 sum m phi, E = K + W, total
  momentum P = sum m v, angular momentum L = sum m x cross v, centre of mass.
* Jerk (Section 3 names it beside the acceleration as the other quantity
  the device computes; the paper does not print its formula). It is the time
  derivative of the softened acceleration: with d = x_j - x_i,
  w = v_j - v_i and q = r^2 + eps^2,
  jerk_i = G sum_{j != i} m_j [w / q^{3/2} - 3 (d.w) d / q^{5/2}].
* Fourth-order Hermite predictor-corrector with a shared step (the scheme
  jerk is used for; the paper does not name its integrator): predict
  x_p = x + v dt + a dt^2/2 + j dt^3/6, v_p = v + a dt + j dt^2/2; evaluate
  a_1, j_1 at (x_p, v_p); correct v_1 = v + (a_0 + a_1) dt/2 + (j_0 - j_1) dt^2/12,
  x_1 = x + (v + v_1) dt/2 + (a_0 - a_1) dt^2/12.
* Error metrics used to compare the GPU results with this oracle.

Everything is float64. Sums over j use numpy reductions of whole rows (a
different association order than a sequential loop, which is immaterial at
FP64 against FP32 results; the C oracle next to this file sums sequentially).
"""
from __future__ import annotations

import numpy as np

# Layout of one diagnostics row (shared convention with the C ABI header,
# restated here rather than imported).
DIAG_LEN = 16
D_K, D_W, D_E = 0, 1, 2
D_P = slice(3, 6)
D_L = slice(6, 9)
D_COM = slice(9, 12)
D_M = 12
D_NONFINITE = 13
D_STEP = 14


def brute_force(pos, mass, eps=0.0, G=1.0):
    """Pure-Python double loop, for tiny N only: the force equation of
    Section 3 summed term by term over j != i, softened by eps."""
    n = len(mass)
    acc = [[0.0, 0.0, 0.0] for _ in range(n)]
    pot = [0.0] * n
    for i in range(n):
        for j in range(n):
            if j == i:
                continue
            d = [pos[j][c] - pos[i][c] for c in range(3)]
            r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps
            r = r2 ** 0.5
            for c in range(3):
                acc[i][c] += G * mass[j] * d[c] / (r2 * r)
            pot[i] -= G * mass[j] / r
    return np.array(acc, dtype=np.float64), np.array(pot, dtype=np.float64)


def accel_pot(pos, mass, eps=0.0, G=1.0, targets=None, chunk=None):
    """Softened accelerations and potentials on ``targets`` (all particles if
    None) from all N sources, self term excluded by index.

    Returns ``(acc, pot)`` with shapes (T, 3) and (T,), float64.
    """
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    t_idx = np.arange(n) if targets is None else np.asarray(targets, dtype=np.int64)
    nt = t_idx.shape[0]
    acc = np.zeros((nt, 3))
    pot = np.zeros(nt)
    if n == 0 or nt == 0:
        return acc, pot
    if chunk is None:
        chunk = max(1, min(nt, (1 << 23) // max(n, 1)))
    eps2 = float(eps) * float(eps)
    for s in range(0, nt, chunk):
        ti = t_idx[s:s + chunk]
        d = pos[None, :, :] - pos[ti, None, :]            # (c, N, 3): r_j - r_i
        r2 = np.einsum("cjk,cjk->cj", d, d) + eps2
        self_mask = np.arange(n)[None, :] == ti[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / np.sqrt(r2)
        inv = np.where(self_mask, 0.0, inv)
        w = mass[None, :] * inv                           # m_j / r
        w3 = w * inv * inv                                # m_j / r^3
        acc[s:s + chunk] = G * np.einsum("cj,cjk->ck", w3, d)
        pot[s:s + chunk] = -G * w.sum(axis=1)
    return acc, pot


def brute_force_jerk(pos, vel, mass, eps=0.0, G=1.0):
    """Pure-Python double loop for the jerk, for tiny N only."""
    n = len(mass)
    jerk = [[0.0, 0.0, 0.0] for _ in range(n)]
    for i in range(n):
        for j in range(n):
            if j == i:
                continue
            d = [pos[j][c] - pos[i][c] for c in range(3)]
            w = [vel[j][c] - vel[i][c] for c in range(3)]
            q = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps
            dw = d[0] * w[0] + d[1] * w[1] + d[2] * w[2]
            for c in range(3):
                jerk[i][c] += G * mass[j] * (w[c] / q ** 1.5 - 3.0 * dw * d[c] / q ** 2.5)
    return np.array(jerk, dtype=np.float64)


def accel_jerk(pos, vel, mass, eps=0.0, G=1.0, targets=None, chunk=None):
    """Accelerations, jerks and potentials on ``targets`` (all if None),
    self term excluded by index. Returns ``(acc, jerk, pot)``."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[0]
    t_idx = np.arange(n) if targets is None else np.asarray(targets, dtype=np.int64)
    nt = t_idx.shape[0]
    acc = np.zeros((nt, 3))
    jerk = np.zeros((nt, 3))
    pot = np.zeros(nt)
    if n == 0 or nt == 0:
        return acc, jerk, pot
    if chunk is None:
        chunk = max(1, min(nt, (1 << 22) // max(n, 1)))
    eps2 = float(eps) * float(eps)
    for s in range(0, nt, chunk):
        ti = t_idx[s:s + chunk]
        d = pos[None, :, :] - pos[ti, None, :]
        w = vel[None, :, :] - vel[ti, None, :]
        q = np.einsum("cjk,cjk->cj", d, d) + eps2
        self_mask = np.arange(n)[None, :] == ti[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / np.sqrt(q)
        inv = np.where(self_mask, 0.0, inv)
        m1 = mass[None, :] * inv                 # m / q^{1/2}
        m3 = m1 * inv * inv                      # m / q^{3/2}
        m5 = m3 * inv * inv                      # m / q^{5/2}
        dw = np.einsum("cjk,cjk->cj", d, w)
        acc[s:s + chunk] = G * np.einsum("cj,cjk->ck", m3, d)
        jerk[s:s + chunk] = G * (np.einsum("cj,cjk->ck", m3, w) - 3.0 * np.einsum("cj,cjk->ck", m5 * dw, d))
        pot[s:s + chunk] = -G * m1.sum(axis=1)
    return acc, jerk, pot


def hermite(pos, vel, mass, eps, G, dt, n_steps, acc=None, jerk=None, force=None, diag=True):
    """Fourth-order Hermite predictor-corrector, shared step, FP64.

    ``force(x, v) -> (acc, jerk, pot)`` defaults to the softened direct sum.
    Returns ``(pos, vel, acc, jerk, pot, rows)``; the potential of a row is the
    one evaluated at that step's predicted positions."""
    if force is None:
        def force(x, v):
            return accel_jerk(x, v, mass, eps, G)
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    if acc is None or jerk is None:
        acc, jerk, pot = force(pos, vel)
    else:
        acc = np.array(acc, dtype=np.float64)
        jerk = np.array(jerk, dtype=np.float64)
        pot = force(pos, vel)[2] if diag else None
    rows = [diagnostics(pos, vel, mass, pot, step=0)] if diag else None
    for s in range(n_steps):
        xp = pos + dt * vel + (dt * dt / 2.0) * acc + (dt ** 3 / 6.0) * jerk
        vp = vel + dt * acc + (dt * dt / 2.0) * jerk
        a1, j1, pot = force(xp, vp)
        v1 = vel + (dt / 2.0) * (acc + a1) + (dt * dt / 12.0) * (jerk - j1)
        x1 = pos + (dt / 2.0) * (vel + v1) + (dt * dt / 12.0) * (acc - a1)
        pos, vel, acc, jerk = x1, v1, a1, j1
        if diag:
            rows.append(diagnostics(pos, vel, mass, pot, step=s + 1))
    return pos, vel, acc, jerk, pot, (np.array(rows) if diag else None)


def kdk(pos, vel, mass, eps, G, dt, n_steps, acc=None, accel=None, diag=True):
    """Kick-drift-kick leapfrog for ``n_steps`` steps in FP64.

    ``accel(pos) -> (acc, pot)`` defaults to the softened direct sum. If
    ``acc`` is None the first force evaluation is done here. Returns
    ``(pos, vel, acc, pot, rows)`` where ``rows`` holds a diagnostics row for
    the initial state and one after every step (None when ``diag`` is False).
    """
    if accel is None:
        def accel(x):
            return accel_pot(x, mass, eps, G)
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    if acc is None:
        acc, pot = accel(pos)
    else:
        acc = np.array(acc, dtype=np.float64)
        pot = accel(pos)[1] if diag else None
    rows = [diagnostics(pos, vel, mass, pot, step=0)] if diag else None
    h = 0.5 * dt
    for s in range(n_steps):
        vel = vel + h * acc
        pos = pos + dt * vel
        acc, pot = accel(pos)
        vel = vel + h * acc
        if diag:
            rows.append(diagnostics(pos, vel, mass, pot, step=s + 1))
    return pos, vel, acc, pot, (np.array(rows) if diag else None)


def diagnostics(pos, vel, mass, pot, step=0):
    """One diagnostics row: K, W, E, P, L, centre of mass, M, count of
    non-finite entries in (pos, vel), step index."""
    pos = np.asarray(pos, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    row = np.zeros(DIAG_LEN)
    k = 0.5 * float(np.sum(mass * np.einsum("ik,ik->i", vel, vel)))
    w = 0.5 * float(np.sum(mass * pot)) if pot is not None else np.nan
    row[D_K], row[D_W], row[D_E] = k, w, k + w
    row[D_P] = (mass[:, None] * vel).sum(axis=0)
    row[D_L] = (mass[:, None] * np.cross(pos, vel)).sum(axis=0)
    mt = float(mass.sum())
    row[D_COM] = (mass[:, None] * pos).sum(axis=0) / mt
    row[D_M] = mt
    row[D_NONFINITE] = float(np.count_nonzero(~np.isfinite(pos)) + np.count_nonzero(~np.isfinite(vel)))
    row[D_STEP] = float(step)
    return row


def energy_drift(rows):
    """Relative energy error |E_n - E_0| / |E_0| for every row."""
    e = np.asarray(rows)[:, D_E]
    return np.abs(e - e[0]) / abs(e[0])


# ---- error metrics (GPU result vs this oracle) ------------------------------

def rel_rms(x, ref):
    """sqrt(sum_i |x_i - ref_i|^2 / sum_i |ref_i|^2) over all targets."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.sum((x - ref) ** 2)
    den = np.sum(ref ** 2)
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def max_rel(x, ref):
    """max_i |x_i - ref_i| / |ref_i| (vector norms for (T, 3) arrays)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if x.ndim == 1:
        x, ref = x[:, None], ref[:, None]
    err = np.linalg.norm(x - ref, axis=1)
    mag = np.linalg.norm(ref, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(mag > 0, err / mag, np.where(err > 0, np.inf, 0.0))
    return float(r.max()) if r.size else 0.0


def paper_metric(x, ref):
    """Largest per-component error over a typical magnitude, read as the RMS
    of |ref_i| (the paper's validation criterion, Section 3)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    typ = float(np.sqrt(np.mean(np.sum(ref.reshape(len(ref), -1) ** 2, axis=1))))
    return float(np.max(np.abs(x - ref)) / typ) if typ > 0 else float(np.max(np.abs(x - ref)))


def subsample_targets(n, k=4096):
    """Evenly strided targets i_k = floor(k n / K), k = 0..K-1 (all if n <= K)."""
    if n <= k:
        return np.arange(n, dtype=np.int64)
    return (np.arange(k, dtype=np.int64) * n) // k
