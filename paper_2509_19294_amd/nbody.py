"""Thin Python binding of libnbody.so (argument marshalling only).

Every step of the computation runs in the library's HIP kernels; this module
checks tensors, passes their device pointers and the current HIP stream, and
turns a non-OK status into an exception. PyTorch provides device memory and
streams. The library is loaded on first use; if it is missing, every call
raises (there is no fallback).

Names follow the C ABI of ``include/nbody.h``: ``accel`` (nbody_accel),
``step`` (nbody_step), ``Plan`` (nbody_plan_create; ``Plan.accel`` is
nbody_accel_batched), ``step_batched`` (nbody_step_batched).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbody.so")

PLAIN = 0
COMP = 1
VARIANTS = {"plain": PLAIN, "comp": COMP, PLAIN: PLAIN, COMP: COMP}

OK, EINVAL, ENOTSUP, EWORKSPACE, EHIP = 0, 1, 2, 3, 4
DIAG_LEN = 16
DIAG = dict(K=0, W=1, E=2, P=slice(3, 6), L=slice(6, 9), COM=slice(9, 12), M=12, NONFINITE=13, STEP=14)

_lib = None
_lock = threading.Lock()


class NbodyError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"nbody status {status}: {message}")
        self.status = status


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libnbody.so and declare its signatures (idempotent)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run `python -m paper_2509_19294_amd.build`")
        lib = ctypes.CDLL(path)
        c_dp = ctypes.c_void_p
        i64, i32, dbl, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        sig = {
            "nbody_workspace_bytes": (sz, [i64, i32, i32]),
            "nbody_last_error": (ctypes.c_char_p, []),
            "nbody_version": (ctypes.c_char_p, []),
            "nbody_accel": (i32, [c_dp, c_dp, i64, dbl, dbl, i32, c_dp, c_dp, c_dp, sz, c_dp]),
            "nbody_accel_noalloc": (i32, [c_dp, c_dp, i64, dbl, dbl, i32, c_dp, c_dp, c_dp]),
            "nbody_step": (i32, [c_dp, c_dp, c_dp, c_dp, c_dp, i64, dbl, dbl, dbl, i32, i32, c_dp,
                                 c_dp, c_dp, sz, c_dp]),
            "nbody_step_batched": (i32, [c_dp, c_dp, c_dp, c_dp, c_dp, i64, c_dp, c_dp, dbl, dbl, i32,
                                         i32, c_dp, c_dp, sz, c_dp]),
            "nbody_plan_create": (c_dp, [ctypes.POINTER(i64), i32, i32, ctypes.c_char_p]),
            "nbody_plan_destroy": (None, [c_dp]),
            "nbody_accel_batched": (i32, [c_dp, c_dp, c_dp, c_dp, dbl, i32, c_dp, c_dp, c_dp, sz,
                                          c_dp]),
            "nbody_plan_total": (i64, [c_dp]),
            "nbody_plan_clusters": (i32, [c_dp]),
            "nbody_plan_variant": (i32, [c_dp]),
            "nbody_plan_items": (i64, [c_dp]),
            "nbody_plan_pairs": (dbl, [c_dp]),
            "nbody_tune_count": (i32, [i32]),
            "nbody_tune_describe": (i32, [i32, i32, ctypes.POINTER(i32)]),
            "nbody_tune_set": (i32, [i32, i32, i32]),
            "nbody_tune_get": (i32, [i32, i64]),
            "nbody_tune_load": (i32, [ctypes.c_char_p]),
            "nbody_tune_reset": (i32, []),
            "nbody_workspace_bytes_jerk": (sz, [i64, i32]),
            "nbody_accel_jerk": (i32, [c_dp, c_dp, c_dp, i64, dbl, dbl, i32, c_dp, c_dp, c_dp, c_dp,
                                       sz, c_dp]),
            "nbody_step_hermite": (i32, [c_dp, c_dp, c_dp, c_dp, c_dp, c_dp, i64, dbl, dbl, dbl, i32,
                                         i32, c_dp, c_dp, sz, c_dp]),
            "nbody_tune_jerk_count": (i32, [i32]),
            "nbody_tune_jerk_describe": (i32, [i32, ctypes.POINTER(i32)]),
            "nbody_tune_jerk_set": (i32, [i32, i32]),
            "nbody_tune_jerk_get": (i32, [i32, i64]),
            "nbody_timing_enable": (i32, [i32]),
            "nbody_timing_read": (i32, [ctypes.POINTER(i64), ctypes.POINTER(dbl)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
        return lib


def last_error() -> str:
    return load().nbody_last_error().decode()


def _check(status: int):
    if status != OK:
        raise NbodyError(status, last_error())


def _variant(v) -> int:
    try:
        return VARIANTS[v]
    except KeyError:
        raise ValueError(f"unknown variant {v!r}") from None


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _vec3(t: torch.Tensor, name: str, n=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.dim() != 2 or t.shape[1] != 3 or (n is not None and t.shape[0] != n):
        raise ValueError(f"{name} must have shape ({'n' if n is None else n}, 3)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _vec1(t: torch.Tensor, name: str, n: int) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.dim() != 1 or t.shape[0] != n:
        raise ValueError(f"{name} must have shape ({n},)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def workspace_bytes(n_total: int, n_clusters: int = 1, variant="plain") -> int:
    return int(load().nbody_workspace_bytes(int(n_total), int(n_clusters), _variant(variant)))


_ws_cache: dict = {}


def workspace(n_total: int, n_clusters: int, variant, device, need: int | None = None) -> torch.Tensor:
    """A cached device workspace large enough for the call (allocated by torch)."""
    if need is None:
        need = workspace_bytes(n_total, n_clusters, variant)
    dev = torch.device(device)
    key = (dev.type, dev.index)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        _ws_cache[key] = ws
    return ws


def accel(pos: torch.Tensor, mass: torch.Tensor, eps: float, G: float = 1.0, variant="plain",
          acc: torch.Tensor | None = None, pot: torch.Tensor | bool | None = True,
          ws: torch.Tensor | None = None):
    """Softened accelerations (and potentials) of one system: nbody_accel.

    Returns ``(acc, pot)``; ``pot`` is None when ``pot=False``.
    """
    lib = load()
    _vec3(pos, "pos")
    n = pos.shape[0]
    _vec1(mass, "mass", n)
    if acc is None:
        acc = torch.empty_like(pos)
    _vec3(acc, "acc", n)
    if pot is True:
        pot = torch.empty_like(mass)
    elif pot is False:
        pot = None
    if pot is not None:
        _vec1(pot, "pot", n)
    v = _variant(variant)
    if ws is None:
        ws = workspace(n, 1, v, pos.device)
    st = lib.nbody_accel(pos.data_ptr(), mass.data_ptr(), n, float(eps), float(G), v,
                         acc.data_ptr(), pot.data_ptr() if pot is not None else None,
                         ws.data_ptr(), ws.numel(), _stream_handle(pos.device))
    _check(st)
    return acc, pot


def _diag(diag, n_steps, device):
    if diag is True:
        diag = torch.empty((max(int(n_steps), 0), DIAG_LEN), dtype=torch.float64, device=device)
    elif diag is False:
        diag = None
    if diag is not None and (diag.dtype != torch.float64 or diag.shape != (n_steps, DIAG_LEN)
                             or not diag.is_contiguous()):
        raise ValueError("diag must be a contiguous float64 tensor of shape (n_steps, 16)")
    return diag


def accel_noalloc(pos: torch.Tensor, mass: torch.Tensor, eps: float, G: float = 1.0, variant="plain",
                  acc: torch.Tensor | None = None, pot: torch.Tensor | bool | None = True):
    """nbody_accel without a workspace (the library's static scratch):
    nbody_accel_noalloc. Returns ``(acc, pot)``. Pass preallocated ``acc``
    and ``pot`` to keep the call free of allocations."""
    lib = load()
    _vec3(pos, "pos")
    n = pos.shape[0]
    _vec1(mass, "mass", n)
    acc = torch.empty_like(pos) if acc is None else _vec3(acc, "acc", n)
    if pot is True:
        pot = torch.empty_like(mass)
    elif pot is False:
        pot = None
    if pot is not None:
        _vec1(pot, "pot", n)
    st = lib.nbody_accel_noalloc(pos.data_ptr(), mass.data_ptr(), n, float(eps), float(G), _variant(variant),
                                 acc.data_ptr(), pot.data_ptr() if pot is not None else None,
                                 _stream_handle(pos.device))
    _check(st)
    return acc, pot


def step(pos, vel, acc, mass, eps: float, G: float, dt: float, n_steps: int, variant="plain",
         diag: bool | torch.Tensor = True, pot: torch.Tensor | None = None,
         ws: torch.Tensor | None = None):
    """``n_steps`` kick-drift-kick steps of one system in place on (pos, vel,
    acc): nbody_step.

    ``acc`` must hold the accelerations at ``pos`` on entry. Returns the
    diagnostics tensor of shape (n_steps, 16) (or None when ``diag=False``).
    """
    lib = load()
    _vec3(pos, "pos")
    n = pos.shape[0]
    _vec3(vel, "vel", n)
    _vec3(acc, "acc", n)
    _vec1(mass, "mass", n)
    if pot is not None:
        _vec1(pot, "pot", n)
    v = _variant(variant)
    diag = _diag(diag, n_steps, pos.device)
    if ws is None:
        ws = workspace(n, 1, v, pos.device)
    st = lib.nbody_step(pos.data_ptr(), vel.data_ptr(), acc.data_ptr(),
                        pot.data_ptr() if pot is not None else None, mass.data_ptr(), n,
                        float(eps), float(G), float(dt), int(n_steps), v, None,
                        diag.data_ptr() if (diag is not None and n_steps > 0) else None,
                        ws.data_ptr(), ws.numel(), _stream_handle(pos.device))
    _check(st)
    return diag


def step_batched(pos, vel, acc, mass, plan: "Plan", eps_k: torch.Tensor, G: float, dt: float,
                 n_steps: int, diag: bool | torch.Tensor = True, pot: torch.Tensor | None = None,
                 ws: torch.Tensor | None = None):
    """``n_steps`` kick-drift-kick steps of every cluster of ``plan`` in place,
    cluster k softened by ``eps_k[k]`` (a float64 CUDA tensor of shape (K,)):
    nbody_step_batched. ``acc`` must hold the accelerations at ``pos``."""
    lib = load()
    n = plan.n_total
    _vec3(pos, "pos", n)
    _vec3(vel, "vel", n)
    _vec3(acc, "acc", n)
    _vec1(mass, "mass", n)
    _vec1(eps_k, "eps_k", plan.K)
    if pot is not None:
        _vec1(pot, "pot", n)
    diag = _diag(diag, n_steps, pos.device)
    if ws is None:
        ws = workspace(n, plan.K, plan.variant, pos.device)
    st = lib.nbody_step_batched(pos.data_ptr(), vel.data_ptr(), acc.data_ptr(),
                                pot.data_ptr() if pot is not None else None, mass.data_ptr(), n,
                                plan.handle, eps_k.data_ptr(), float(G), float(dt), int(n_steps),
                                plan.variant,
                                diag.data_ptr() if (diag is not None and n_steps > 0) else None,
                                ws.data_ptr(), ws.numel(), _stream_handle(pos.device))
    _check(st)
    return diag


def accel_jerk(pos, vel, mass, eps: float, G: float = 1.0, variant="plain", acc=None, jerk=None,
               pot=True, ws=None):
    """Accelerations, jerks and potentials of one system: nbody_accel_jerk.
    Returns ``(acc, jerk, pot)``."""
    lib = load()
    _vec3(pos, "pos")
    n = pos.shape[0]
    _vec3(vel, "vel", n)
    _vec1(mass, "mass", n)
    acc = torch.empty_like(pos) if acc is None else _vec3(acc, "acc", n)
    jerk = torch.empty_like(pos) if jerk is None else _vec3(jerk, "jerk", n)
    if pot is True:
        pot = torch.empty_like(mass)
    elif pot is False:
        pot = None
    if pot is not None:
        _vec1(pot, "pot", n)
    v = _variant(variant)
    if ws is None:
        ws = workspace(n, 1, v, pos.device, need=int(lib.nbody_workspace_bytes_jerk(n, v)))
    st = lib.nbody_accel_jerk(pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), n, float(eps), float(G), v,
                              acc.data_ptr(), jerk.data_ptr(), pot.data_ptr() if pot is not None else None,
                              ws.data_ptr(), ws.numel(), _stream_handle(pos.device))
    _check(st)
    return acc, jerk, pot


def step_hermite(pos, vel, acc, jerk, mass, eps: float, G: float, dt: float, n_steps: int,
                 variant="plain", diag: bool | torch.Tensor = True, pot=None, ws=None):
    """``n_steps`` fourth-order Hermite steps in place: nbody_step_hermite.
    ``acc`` and ``jerk`` must hold A and J at (pos, vel) on entry."""
    lib = load()
    _vec3(pos, "pos")
    n = pos.shape[0]
    for t, name in ((vel, "vel"), (acc, "acc"), (jerk, "jerk")):
        _vec3(t, name, n)
    _vec1(mass, "mass", n)
    if pot is not None:
        _vec1(pot, "pot", n)
    v = _variant(variant)
    diag = _diag(diag, n_steps, pos.device)
    if ws is None:
        ws = workspace(n, 1, v, pos.device, need=int(lib.nbody_workspace_bytes_jerk(n, v)))
    st = lib.nbody_step_hermite(pos.data_ptr(), vel.data_ptr(), acc.data_ptr(), jerk.data_ptr(),
                                pot.data_ptr() if pot is not None else None, mass.data_ptr(), n,
                                float(eps), float(G), float(dt), int(n_steps), v,
                                diag.data_ptr() if (diag is not None and n_steps > 0) else None,
                                ws.data_ptr(), ws.numel(), _stream_handle(pos.device))
    _check(st)
    return diag


class Plan:
    """A batched plan over independent clusters (nbody_plan_create).

    ``offsets`` has K + 1 entries: cluster k owns particles
    [offsets[k], offsets[k + 1]). The per-cluster softenings are passed to
    every call (``accel``, ``step_batched``), not stored in the plan.
    """

    def __init__(self, offsets, variant="comp", tune_path: str | None = None):
        import numpy as np

        lib = load()
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        if off.ndim != 1 or off.shape[0] < 2:
            raise ValueError("offsets must have K + 1 >= 2 entries")
        self.K = int(off.shape[0] - 1)
        self.variant = _variant(variant)
        self.offsets = off
        h = lib.nbody_plan_create(off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), self.K,
                                  self.variant, tune_path.encode() if tune_path else None)
        if not h:
            raise NbodyError(EINVAL, last_error())
        self.handle = ctypes.c_void_p(h)
        self.n_total = int(lib.nbody_plan_total(self.handle))
        self.n_items = int(lib.nbody_plan_items(self.handle))
        self.pairs = float(lib.nbody_plan_pairs(self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.nbody_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def accel(self, pos, mass, eps_k, G: float = 1.0, acc=None, pot=True, ws=None):
        """Accelerations of every cluster from its own members, cluster k
        softened by ``eps_k[k]`` (float64 CUDA tensor of shape (K,)):
        nbody_accel_batched."""
        lib = load()
        n = self.n_total
        _vec3(pos, "pos", n)
        _vec1(mass, "mass", n)
        _vec1(eps_k, "eps_k", self.K)
        if acc is None:
            acc = torch.empty_like(pos)
        _vec3(acc, "acc", n)
        if pot is True:
            pot = torch.empty_like(mass)
        elif pot is False:
            pot = None
        if pot is not None:
            _vec1(pot, "pot", n)
        if ws is None:
            ws = workspace(n, self.K, self.variant, pos.device)
        st = lib.nbody_accel_batched(pos.data_ptr(), mass.data_ptr(), self.handle, eps_k.data_ptr(),
                                     float(G), self.variant, acc.data_ptr(),
                                     pot.data_ptr() if pot is not None else None,
                                     ws.data_ptr(), ws.numel(), _stream_handle(pos.device))
        _check(st)
        return acc, pot


# ---- tuning --------------------------------------------------------------

def tune_configs(variant="plain"):
    """List of (block, k, ls, sw, tile, i_per_block) of the compiled configurations."""
    lib = load()
    v = _variant(variant)
    out = []
    buf = (ctypes.c_int32 * 6)()
    for c in range(lib.nbody_tune_count(v)):
        _check(lib.nbody_tune_describe(v, c, buf))
        out.append(tuple(buf))
    return out


def batched_modes():
    lib = load()
    out = []
    buf = (ctypes.c_int32 * 6)()
    m = 0
    while lib.nbody_tune_describe(0, 1000 + m, buf) == OK:
        out.append(tuple(buf))
        m += 1
    return out


def tune_set(variant, size_class: int, cfg: int, split: int = 1):
    """Force configuration ``cfg`` with grid j-split ``split`` for a size class
    (cfg = -1 restores the table)."""
    code = -1 if cfg < 0 else cfg + 1000 * split
    _check(load().nbody_tune_set(_variant(variant), int(size_class), int(code)))


def tune_get(variant, n: int):
    code = int(load().nbody_tune_get(_variant(variant), int(n)))
    return code % 1000, max(code // 1000, 1)


def jerk_shapes(variant="plain"):
    """List of (K, SW, targets per block) of the acceleration + jerk kernel
    shapes compiled for a variant."""
    lib = load()
    buf = (ctypes.c_int32 * 3)()
    out = []
    for c in range(lib.nbody_tune_jerk_count(_variant(variant))):
        _check(lib.nbody_tune_jerk_describe(c, buf))
        out.append(tuple(buf))
    return out


def tune_jerk_set(variant, cfg: int, split: int = 0):
    """Force jerk-kernel shape ``cfg`` with grid j-split ``split`` (0 = the
    built-in rule) for every size; cfg = -1 restores the table."""
    code = -1 if cfg < 0 else cfg + 1000 * split
    _check(load().nbody_tune_jerk_set(_variant(variant), int(code)))


def tune_jerk_get(variant, n: int):
    code = int(load().nbody_tune_jerk_get(_variant(variant), int(n)))
    return code % 1000, code // 1000


def tune_load(path: str):
    _check(load().nbody_tune_load(path.encode()))


def tune_reset():
    _check(load().nbody_tune_reset())


# ---- measurement ----------------------------------------------------------

def timing_enable(on: bool = True):
    """Bracket every eager force-kernel launch with HIP events on its stream."""
    _check(load().nbody_timing_enable(1 if on else 0))


def timing_read():
    """(launches, total_ms) of the bracketed force kernels since the last read."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load().nbody_timing_read(ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)
