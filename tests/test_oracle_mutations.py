"""Planted mistakes in the oracle must be caught by its pins.

Each case rewrites one line of ``oracle.accel_pot`` (a dropped term, a wrong
sign or index, a transposed operand, a missing self-term mask, a wrong power)
in a private copy, and checks that the hand-worked three-body fixtures or the
Newton's-third-law pin reject the copy. Everything runs on the CPU.
"""
import inspect
import textwrap

import numpy as np
import pytest

from oracle import oracle as orc
from tests import golden_io

MUTATIONS = {
    "wrong_sign_of_separation": ("d = pos[None, :, :] - pos[ti, None, :]", "d = pos[ti, None, :] - pos[None, :, :]"),
    "dropped_softening": ("r2 = np.einsum(\"cjk,cjk->cj\", d, d) + eps2", "r2 = np.einsum(\"cjk,cjk->cj\", d, d)"),
    "source_mass_transposed": ("w = mass[None, :] * inv", "w = mass[ti][:, None] * inv"),
    "self_term_kept": ("inv = np.where(self_mask, 0.0, inv)", "inv = np.where(self_mask & (eps2 == 0), 0.0, inv)"),
    "inverse_square_power": ("w3 = w * inv * inv", "w3 = w * inv"),
    "dropped_G_on_potential": ("pot[s:s + chunk] = -G * w.sum(axis=1)", "pot[s:s + chunk] = -w.sum(axis=1)"),
    "potential_sign": ("pot[s:s + chunk] = -G * w.sum(axis=1)", "pot[s:s + chunk] = G * w.sum(axis=1)"),
    "component_index": ("acc[s:s + chunk] = G * np.einsum(\"cj,cjk->ck\", w3, d)",
                        "acc[s:s + chunk] = G * np.einsum(\"cj,cjk->ck\", w3, d[:, :, ::-1])"),
}


def _mutant(old, new):
    src = textwrap.dedent(inspect.getsource(orc.accel_pot))
    assert old in src, old
    ns = {"np": np}
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns["accel_pot"]


def _pins_pass(f):
    for name in ("three_body_eps0.txt", "three_body_eps1.txt"):
        g = golden_io.load(name)
        pos, mass, eps = golden_io.arr(g, "pos"), golden_io.arr(g, "mass")[0], g["eps"][0][0]
        for G in (1.0, 2.0):
            acc, pot = f(pos, mass, eps, G)
            if not np.allclose(acc, G * golden_io.arr(g, "acc"), rtol=0, atol=1e-15):
                return False
            if not np.allclose(pot, G * golden_io.arr(g, "pot")[0], rtol=0, atol=1e-15):
                return False
    return True


def test_unmutated_oracle_passes():
    assert _pins_pass(orc.accel_pot)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    assert not _pins_pass(_mutant(*MUTATIONS[name]))


JERK_MUTATIONS = {
    "relative_velocity_sign": ("w = vel[None, :, :] - vel[ti, None, :]", "w = vel[ti, None, :] - vel[None, :, :]"),
    "factor_three_dropped": ("- 3.0 * np.einsum(\"cj,cjk->ck\", m5 * dw, d)", "- np.einsum(\"cj,cjk->ck\", m5 * dw, d)"),
    "second_term_sign": ("jerk[s:s + chunk] = G * (np.einsum(\"cj,cjk->ck\", m3, w) - 3.0",
                         "jerk[s:s + chunk] = G * (np.einsum(\"cj,cjk->ck\", m3, w) + 3.0"),
    "wrong_power": ("m5 = m3 * inv * inv", "m5 = m3 * inv"),
}


def _jerk_mutant(old, new):
    src = textwrap.dedent(inspect.getsource(orc.accel_jerk))
    assert old in src, old
    ns = {"np": np}
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns["accel_jerk"]


def _jerk_pin_passes(f):
    g = golden_io.load("three_body_eps0.txt")
    _, jerk, _ = f(golden_io.arr(g, "pos"), golden_io.arr(g, "vel"), golden_io.arr(g, "mass")[0], 0.0, 1.0)
    return np.allclose(jerk, golden_io.arr(g, "jerk"), rtol=0, atol=1e-15)


def test_unmutated_jerk_passes():
    assert _jerk_pin_passes(orc.accel_jerk)


@pytest.mark.parametrize("name", sorted(JERK_MUTATIONS))
def test_planted_jerk_mistake_is_caught(name):
    assert not _jerk_pin_passes(_jerk_mutant(*JERK_MUTATIONS[name]))
