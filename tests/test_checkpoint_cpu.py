"""Checkpoint and resume (host side): the .npz round trip keeps every bit,
and ten oracle KDK steps equal five, a save and load, then five more."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2509_19294_amd import checkpoint, ics


def test_round_trip_keeps_every_bit(tmp_path):
    pos, vel, mass = ics.plummer(257, seed=11)
    acc, _ = orc.accel_pot(pos, mass, 0.01)
    jerk = np.random.default_rng(3).standard_normal((257, 3))
    path = checkpoint.save(str(tmp_path / "c.npz"), pos=pos, vel=vel, acc=acc, mass=mass, t=0.375,
                           step=48, eps=0.01, G=1.5, dt=1 / 128, variant="comp", seed=11, jerk=jerk)
    s = checkpoint.load(path)
    for k, ref in (("pos", pos), ("vel", vel), ("acc", acc), ("mass", mass), ("jerk", jerk)):
        assert s[k].dtype == np.float64 and np.array_equal(s[k].view(np.uint64), ref.view(np.uint64)), k
    assert (s["t"], s["step"], s["eps"], s["G"], s["dt"], s["seed"], s["variant"]) == \
        (0.375, 48, 0.01, 1.5, 1 / 128, 11, "comp")
    assert "eps_k" not in s and "offsets" not in s


def test_batched_fields_and_validation(tmp_path):
    pos, vel, mass = ics.plummer(10, seed=1)
    acc = np.zeros_like(pos)
    off = np.array([0, 4, 10], dtype=np.int64)
    ek = np.array([0.1, 0.2])
    s = checkpoint.load(checkpoint.save(str(tmp_path / "b.npz"), pos=pos, vel=vel, acc=acc, mass=mass,
                                        t=0.0, step=0, eps_k=ek, offsets=off))
    assert np.array_equal(s["offsets"], off) and np.array_equal(s["eps_k"], ek)
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "x.npz"), pos=pos, vel=vel, acc=acc, mass=mass, t=0, step=0,
                        eps_k=ek, offsets=np.array([0, 4, 9]))
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "x.npz"), pos=pos, vel=vel, acc=acc, mass=mass, t=0, step=0,
                        eps_k=ek)
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "x.npz"), pos=pos[:5], vel=vel, acc=acc, mass=mass, t=0, step=0)
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "x.npz"), pos=pos, vel=vel, acc=acc, mass=mass, t=0, step=0,
                        variant="fp16")
    assert not list(tmp_path.glob("x.npz*")), "a rejected save leaves no file"


def test_oracle_ten_steps_equal_five_save_load_five(tmp_path):
    pos, vel, mass = ics.plummer(128, seed=5)
    eps, dt = 0.01, 1 / 128
    p10, v10, a10, _, _ = orc.kdk(pos, vel, mass, eps, 1.0, dt, 10, diag=False)
    p5, v5, a5, _, _ = orc.kdk(pos, vel, mass, eps, 1.0, dt, 5, diag=False)
    path = checkpoint.save(str(tmp_path / "five.npz"), pos=p5, vel=v5, acc=a5, mass=mass, t=5 * dt,
                           step=5, eps=eps, dt=dt, seed=5)
    s = checkpoint.load(path)
    pr, vr, ar, _, _ = orc.kdk(s["pos"], s["vel"], s["mass"], s["eps"], s["G"], s["dt"], 10 - s["step"],
                               acc=s["acc"], diag=False)
    for got, ref in ((pr, p10), (vr, v10), (ar, a10)):
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
