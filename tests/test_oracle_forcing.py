"""Pins of the oracle's adaptive forcing terms (Algorithm 1, Eq. (12)-(13))."""
import numpy as np
import pytest

import synth
from oracle import newton as nt
from oracle import physics as ph


def _affine_model():
    """The 10x10x3 model with S_w = 0.9 inside (1 - S_or, 1), where k_rw = 1 and
    k_ro = 0 are clipped constants, constant densities (c = 0) and no gravity:
    every flux, transfer and well term is then linear, so the residual is affine
    in (p, S_w, p_b) as long as S_w stays in that interval."""
    m = synth.model_small()
    m["sw0"][:] = 0.9
    m["c_w"] = m["c_o"] = 0.0
    m["gravity"] = 0.0
    m["schedule"] = [1.0 * synth.DAY]
    return m


# a multi-level AMG (coarsest <= 20 rows) keeps the CPR-FPF inexact, so that
# GMRES stops at eta_0 = 0.1 well before the exact solution
_INEXACT = dict(amg_opts=dict(max_coarse=20))


def _first_step(m, **kw):
    geo = ph.Geometry(m)
    ctrl = [w["control"] for w in m["wells"]]
    x0 = ph.initial_state(m)
    acc = ph.accumulation(geo, x0)
    return geo, nt.newton_solve(geo, x0, acc, m["schedule"][0], ctrl, **kw)


@pytest.mark.parametrize("choice", [1, 2])
def test_affine_residual_drives_choices_1_and_2_to_the_floor(choice):
    """For affine F, b(x^1) = b(x^0) - J y exactly, so b(x^1) - r^0 = 0 and
    ||b(x^1)|| = ||r^0||: both numerators vanish (to rounding) and, with
    eta_0^phi = 0.1^1.618 < 0.1 (no safeguard), eta_1 is the floor eta_min."""
    m = _affine_model()
    geo, (x, ok, its, info) = _first_step(m, tol=1e-11, linear="cpr", forcing=choice, eta0=0.1,
                                          mb_tol=1e-12, max_newton=6, cpr_opts=_INEXACT)
    assert ok
    assert info["eta"][0] == 0.1
    assert len(info["eta"]) >= 2
    assert info["eta"][1] == 1e-8
    # the state stayed inside the affine region
    _, sw, _ = ph.unpack_state(x, geo.n)
    assert np.all((sw > 0.8) & (sw < 1.0))


def test_converged_state_does_not_depend_on_the_forcing_choice():
    """The discrete system has one solution: fixed and adaptive tolerances reach it."""
    m = synth.model_small()
    m["schedule"] = [2.0 * synth.DAY]
    states = []
    for forcing in (0, 1, 2, 3):
        geo, (x, ok, its, info) = _first_step(m, tol=1e-10, linear="cpr", eta=1e-8, forcing=forcing,
                                              max_newton=40)
        assert ok, forcing
        states.append(x)
    p0, s0, b0 = ph.unpack_state(states[0], geo.n)
    for x in states[1:]:
        p, s, b = ph.unpack_state(x, geo.n)
        assert np.max(np.abs(p - p0) / np.abs(p0)) <= 1e-8
        assert np.max(np.abs(s - s0)) <= 1e-8
        assert np.max(np.abs(b - b0) / np.abs(b0)) <= 1e-8


@pytest.mark.parametrize("choice", [1, 2, 3])
def test_forcing_sequence_respects_clamp_and_safeguards(choice):
    """Along a nonlinear solve every eta lies in [eta_min, eta_max] and never drops
    below the safeguard of its choice once that safeguard exceeds 0.1."""
    m = synth.model_small()
    m["schedule"] = [5.0 * synth.DAY]
    geo, (x, ok, its, info) = _first_step(m, tol=1e-8, linear="cpr", forcing=choice, max_newton=40)
    eta = info["eta"]
    assert len(eta) >= 3
    assert all(1e-8 <= e <= 0.9 for e in eta)
    for a, b in zip(eta[:-1], eta[1:]):
        guard = a ** nt.GOLDEN if choice in (1, 2) else 0.9 * a ** 2.0
        if guard > 0.1:
            assert b >= min(guard, 0.9) * (1 - 1e-15)
