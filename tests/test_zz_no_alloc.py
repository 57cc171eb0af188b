"""The allocation-free entry point nbody_accel_noalloc against nbody_accel.

Called through the C ABI on the same inputs: two calls in a row, the second
on a smaller system, for both forms. Where the tuned grid j-split fits the
static scratch the two entry points must agree bit for bit; where it does
not (the compensated form at N = 262,144) they may differ only in summation
order, and both must meet the FP64 oracle's tolerances."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import cpu as ocpu
from oracle import oracle as orc
from paper_2509_19294_amd import ics, nbody

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def both(pos, mass, eps, variant):
    """(nbody_accel, nbody_accel_noalloc) results on the same inputs; the
    no-alloc outputs are preallocated so that the call itself allocates
    nothing."""
    lib = nbody.load()
    tp, tm = T(pos), T(mass)
    a_ref, p_ref = nbody.accel(tp, tm, eps, 1.0, variant)
    acc = torch.full_like(tp, np.nan)
    pot = torch.full_like(tm, np.nan)
    torch.cuda.synchronize()
    st = lib.nbody_accel_noalloc(tp.data_ptr(), tm.data_ptr(), len(mass), eps, 1.0, nbody.VARIANTS[variant],
                                 acc.data_ptr(), pot.data_ptr(), nbody._stream_handle(tp.device))
    assert st == nbody.OK, nbody.last_error()
    torch.cuda.synchronize()
    return (a_ref.cpu().numpy(), p_ref.cpu().numpy()), (acc.cpu().numpy(), pot.cpu().numpy())


def check_oracle(a, p, ref_a, ref_p):
    assert orc.rel_rms(a, ref_a) <= 1e-5 and orc.max_rel(a, ref_a) <= 1e-4
    assert orc.rel_rms(p, ref_p) <= 1e-5


@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_noalloc_equals_accel_twice_shrinking(variant):
    for n, seed in ((3001, 51), (1000, 52)):
        pos, _, mass = ics.plummer(n, seed=seed)
        (a0, p0), (a1, p1) = both(pos, mass, 0.01, variant)
        assert np.array_equal(a0, a1) and np.array_equal(p0, p1), (variant, n)
        ref_a, ref_p = orc.accel_pot(pos, mass, 0.01)
        check_oracle(a1, p1, ref_a, ref_p)


@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_noalloc_large_then_small(variant):
    """N = 262,144 (the compensated form's split is reduced to fit the
    scratch), then N = 65,536 reusing the same scratch."""
    for name in ("plummer_256k", "plummer_64k"):
        pos, _, mass, spec = ics.workload(name)
        eps = spec["eps"]
        (a0, p0), (a1, p1) = both(pos, mass, eps, variant)
        assert orc.rel_rms(a1, a0) < 2e-6 and orc.rel_rms(p1, p0) < 2e-6, (variant, name)
        tgt = orc.subsample_targets(len(mass), 4096)
        ref_a, ref_p = ocpu.accel_pot(pos, mass, eps, targets=tgt)
        check_oracle(a1[tgt], p1[tgt], ref_a, ref_p)


def test_noalloc_rejects_beyond_its_scratch():
    lib = nbody.load()
    tp = torch.zeros((8, 3), dtype=torch.float64, device=DEV)
    fake = ctypes.c_void_p(0x100000)
    st = lib.nbody_accel_noalloc(fake, ctypes.c_void_p(0x200000), 536481, 0.01, 1.0, 1,
                                 ctypes.c_void_p(0x40000000), None, nbody._stream_handle(tp.device))
    assert st == nbody.EINVAL and "scratch" in nbody.last_error()
