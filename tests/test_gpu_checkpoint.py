"""Checkpoint and resume on the GPU: ten steps straight equal five steps, a
save to .npz and a load into fresh device tensors, then five more steps, bit
for bit (KDK single system in both forms, the batched plan, and Hermite)."""
import numpy as np
import pytest
import torch

from paper_2509_19294_amd import checkpoint, ics, nbody

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def bits(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("variant", ["plain", "comp"])
def test_kdk_resume_is_bitwise(tmp_path, variant):
    pos, vel, mass = ics.plummer(3001, seed=21)
    eps, dt = 0.01, 1 / 256
    tp, tv, tm = T(pos), T(vel), T(mass)
    acc, _ = nbody.accel(tp, tm, eps, 1.0, variant)
    nbody.step(tp, tv, acc, tm, eps, 1.0, dt, 10, variant, diag=False)
    torch.cuda.synchronize()
    ref = [bits(x) for x in (tp, tv, acc)]

    tp, tv = T(pos), T(vel)
    acc, _ = nbody.accel(tp, tm, eps, 1.0, variant)
    nbody.step(tp, tv, acc, tm, eps, 1.0, dt, 5, variant, diag=False)
    torch.cuda.synchronize()
    path = checkpoint.save(str(tmp_path / "c.npz"), pos=tp, vel=tv, acc=acc, mass=tm, t=5 * dt, step=5,
                           eps=eps, dt=dt, variant=variant, seed=21)
    del tp, tv, acc
    s = checkpoint.load(path, device=DEV)
    nbody.step(s["pos"], s["vel"], s["acc"], s["mass"], s["eps"], s["G"], s["dt"], 10 - s["step"],
               s["variant"], diag=False)
    torch.cuda.synchronize()
    for got, want in zip((s["pos"], s["vel"], s["acc"]), ref):
        assert np.array_equal(bits(got), want)


def test_batched_resume_is_bitwise(tmp_path):
    ens = ics.ensemble(24, seed=9, n_min=64, n_max=1500)
    dt = 1 / 256
    plan = nbody.Plan(ens.offsets, "comp")
    te = T(ens.eps)
    tp, tv, tm = T(ens.pos), T(ens.vel), T(ens.mass)
    acc, _ = plan.accel(tp, tm, te)
    nbody.step_batched(tp, tv, acc, tm, plan, te, 1.0, dt, 10, diag=False)
    torch.cuda.synchronize()
    ref = [bits(x) for x in (tp, tv, acc)]

    tp, tv = T(ens.pos), T(ens.vel)
    acc, _ = plan.accel(tp, tm, te)
    nbody.step_batched(tp, tv, acc, tm, plan, te, 1.0, dt, 5, diag=False)
    torch.cuda.synchronize()
    path = checkpoint.save(str(tmp_path / "b.npz"), pos=tp, vel=tv, acc=acc, mass=tm, t=5 * dt, step=5,
                           dt=dt, variant="comp", eps_k=te, offsets=ens.offsets)
    plan.close()
    s = checkpoint.load(path, device=DEV)
    plan = nbody.Plan(s["offsets"], s["variant"])
    nbody.step_batched(s["pos"], s["vel"], s["acc"], s["mass"], plan, s["eps_k"], s["G"], s["dt"],
                       10 - s["step"], diag=False)
    torch.cuda.synchronize()
    for got, want in zip((s["pos"], s["vel"], s["acc"]), ref):
        assert np.array_equal(bits(got), want)
    plan.close()


def test_hermite_resume_is_bitwise(tmp_path):
    pos, vel, mass = ics.plummer(2000, seed=22)
    eps, dt = 0.01, 1 / 256
    tp, tv, tm = T(pos), T(vel), T(mass)
    acc, jerk, _ = nbody.accel_jerk(tp, tv, tm, eps, 1.0, "comp")
    nbody.step_hermite(tp, tv, acc, jerk, tm, eps, 1.0, dt, 10, "comp", diag=False)
    torch.cuda.synchronize()
    ref = [bits(x) for x in (tp, tv, acc, jerk)]

    tp, tv = T(pos), T(vel)
    acc, jerk, _ = nbody.accel_jerk(tp, tv, tm, eps, 1.0, "comp")
    nbody.step_hermite(tp, tv, acc, jerk, tm, eps, 1.0, dt, 5, "comp", diag=False)
    torch.cuda.synchronize()
    path = checkpoint.save(str(tmp_path / "h.npz"), pos=tp, vel=tv, acc=acc, mass=tm, jerk=jerk,
                           t=5 * dt, step=5, eps=eps, dt=dt, variant="comp", seed=22)
    s = checkpoint.load(path, device=DEV)
    nbody.step_hermite(s["pos"], s["vel"], s["acc"], s["jerk"], s["mass"], s["eps"], s["G"], s["dt"],
                       10 - s["step"], s["variant"], diag=False)
    torch.cuda.synchronize()
    for got, want in zip((s["pos"], s["vel"], s["acc"], s["jerk"]), ref):
        assert np.array_equal(bits(got), want)
