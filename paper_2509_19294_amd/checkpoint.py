"""Checkpoint and resume of a simulation's state as a ``.npz`` file.

A kick-drift-kick step needs the accelerations at the current positions on
entry, so the state saved is (pos, vel, acc, mass) together with the time,
the step count and the run's parameters (eps or the per-cluster softenings,
G, dt, variant, seed, and the cluster offsets of a batched run). Saving
copies the device tensors to host memory; loading returns host arrays or,
given a device, device tensors, so that a resumed run continues from the
same bits: the forces are deterministic for a fixed tuning, and stepping
5 + 5 from a checkpoint equals stepping 10 straight.

The file holds plain arrays only (``numpy.load`` with pickling disabled
reads it back).
"""
from __future__ import annotations

import os

import numpy as np

STATE_ARRAYS = ("pos", "vel", "acc", "mass")
OPTIONAL_ARRAYS = ("jerk", "eps_k", "offsets")
SCALARS = {"t": float, "step": int, "eps": float, "G": float, "dt": float, "seed": int}
VARIANT_CODES = {"plain": 0, "comp": 1}
FORMAT_VERSION = 1


def _host(x):
    """A host numpy copy of a torch tensor or an array (no torch import needed)."""
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(x))


def save(path: str, *, pos, vel, acc, mass, t: float, step: int, eps: float = 0.0,
         G: float = 1.0, dt: float = 0.0, variant: str = "plain", seed: int = -1,
         jerk=None, eps_k=None, offsets=None) -> str:
    """Write the state to ``path`` (``.npz``; written to a temporary name and
    renamed, so a crash never leaves a half-written checkpoint). ``jerk`` is
    the Hermite integrator's extra state; ``eps_k`` and ``offsets`` describe
    a batched run. Returns the path written."""
    if variant not in VARIANT_CODES:
        raise ValueError(f"unknown variant {variant!r}")
    arrays = {k: _host(v) for k, v in (("pos", pos), ("vel", vel), ("acc", acc), ("mass", mass))}
    n = arrays["mass"].shape[0]
    for k in ("pos", "vel", "acc"):
        if arrays[k].shape != (n, 3) or arrays[k].dtype != np.float64:
            raise ValueError(f"{k} must be float64 of shape ({n}, 3)")
    if arrays["mass"].dtype != np.float64 or arrays["mass"].ndim != 1:
        raise ValueError("mass must be a float64 vector")
    if jerk is not None:
        arrays["jerk"] = _host(jerk)
        if arrays["jerk"].shape != (n, 3):
            raise ValueError(f"jerk must have shape ({n}, 3)")
    if (eps_k is None) != (offsets is None):
        raise ValueError("a batched checkpoint needs both eps_k and offsets")
    if eps_k is not None:
        arrays["eps_k"] = _host(eps_k).astype(np.float64, copy=False)
        arrays["offsets"] = _host(offsets).astype(np.int64, copy=False)
        if arrays["offsets"].shape != (arrays["eps_k"].shape[0] + 1,) or arrays["offsets"][-1] != n:
            raise ValueError("offsets must have K + 1 entries ending at n")
    meta = np.array([float(t), float(step), float(eps), float(G), float(dt), float(seed),
                     float(VARIANT_CODES[variant]), float(FORMAT_VERSION)], dtype=np.float64)
    tmp = path + ".tmp.npz"
    np.savez(tmp, meta=meta, **arrays)
    os.replace(tmp, path)
    return path


def load(path: str, device=None) -> dict:
    """Read a checkpoint written by :func:`save`. Arrays come back as numpy
    arrays, or as torch tensors on ``device`` when one is given; scalars as
    Python numbers; ``variant`` as its name."""
    with np.load(path, allow_pickle=False) as f:
        meta = f["meta"]
        if meta.shape != (8,) or int(meta[7]) != FORMAT_VERSION:
            raise ValueError(f"{path}: not a checkpoint of format {FORMAT_VERSION}")
        out = {k: f[k].copy() for k in STATE_ARRAYS}
        for k in OPTIONAL_ARRAYS:
            if k in f.files:
                out[k] = f[k].copy()
    names = {v: k for k, v in VARIANT_CODES.items()}
    out.update(t=float(meta[0]), step=int(meta[1]), eps=float(meta[2]), G=float(meta[3]),
               dt=float(meta[4]), seed=int(meta[5]), variant=names[int(meta[6])])
    if device is not None:
        import torch

        for k in STATE_ARRAYS + OPTIONAL_ARRAYS:
            if k in out and k != "offsets":
                out[k] = torch.from_numpy(out[k]).to(device)
    return out
