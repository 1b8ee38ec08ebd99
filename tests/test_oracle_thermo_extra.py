"""Pins of the oracle's enthalpy inversion and primitive-variable routine:
h - e = R T sum_k Y_k/W_k, dh/dT = c_p, a constant-cp closed form, round
trips through the enthalpy and through conserved variables."""

import numpy as np
import pytest

import mechs
from oracle import eos, newton, primitive, thermo
from oracle.constants import GAS_CONSTANT as RU
from pyro_synth.states import draw_states


@pytest.mark.parametrize("cfg", [0, 1])
def test_enthalpy_minus_energy_is_RT_over_W(cfg):
    """h = e + p/rho for an ideal gas: h - e = R T sum_k Y_k/W_k."""
    m = mechs.load_config(cfg)
    T, p, Y = draw_states(cfg, 200, m.S)
    d = thermo.mixture_enthalpy(m, T, Y) - thermo.mixture_internal_energy(m, T, Y)
    ref = RU * T * (Y / m.W[:, None]).sum(axis=0)
    scale = np.abs(Y * thermo.species_enthalpy(m, T)).sum(axis=0)
    assert np.all(np.abs(d - ref) <= 1e-13 * scale)


def test_cp_is_dh_dT(mech1):
    T, p, Y = draw_states(1, 50, mech1.S)
    T = np.where(np.abs(T - 1000.0) < 1.0, T + 5.0, T)
    h = 1e-3
    fd = (thermo.mixture_enthalpy(mech1, T + h, Y) - thermo.mixture_enthalpy(mech1, T - h, Y)) / (2 * h)
    np.testing.assert_allclose(fd, thermo.mixture_cp(mech1, T, Y), rtol=1e-7)


def test_enthalpy_newton_constant_cp_closed_form(tmp_path):
    """Constant cp: h = sum Y R (a1 T + a6)/W, so T = (h - sum Y R a6/W) /
    (sum Y R a1/W), reached in at most two updates."""
    S = 3
    a1 = np.array([3.5, 4.5, 2.5])
    a6 = np.array([-800.0, 1500.0, 300.0])
    a = mechs.constant_cp(S, a1, a6, 20.0)
    m = mechs.make(str(tmp_path / "h.pyromech"), W=[0.002, 0.028, 0.032], nasa_low=a,
                   reactions=[dict(reac=[(0, 1)], prod=[(1, 1)], arrh=(0.0, 0.0, 0.0))])
    Y = np.array([[0.1, 0.3], [0.5, 0.2], [0.4, 0.5]])
    hmix = np.array([2.0e5, 9.0e5])
    x = Y / m.W[:, None]
    T_ref = (hmix - RU * (x * a6[:, None]).sum(axis=0)) / (RU * (x * a1[:, None]).sum(axis=0))
    T, st = newton.temperature_from_enthalpy(m, hmix, Y, 1200.0)
    np.testing.assert_allclose(T, T_ref, rtol=1e-13)
    assert np.all((st >= 1) & (st <= 2))


@pytest.mark.parametrize("cfg", [0, 1])
def test_enthalpy_round_trip(cfg):
    m = mechs.load_config(cfg)
    T, p, Y = draw_states(cfg, 300, m.S, first=77)
    h = thermo.mixture_enthalpy(m, T, Y)
    Tn, st = newton.temperature_from_enthalpy(m, h, Y, 1200.0)
    assert np.all(st > 0)
    np.testing.assert_allclose(Tn, T, rtol=1e-12)


def test_primitive_round_trip(mech1):
    """Conserved variables built from a primitive state (rho, Y, u, T) give
    that state back, with p from the equation of state."""
    m = mech1
    n = 120
    T, p, Y = draw_states(1, n, m.S, first=500)
    rho = eos.density(m, p, T, Y)
    rng = np.random.default_rng(3)
    u = rng.uniform(-400, 400, (3, n))
    E = thermo.mixture_internal_energy(m, T, Y) + 0.5 * (u ** 2).sum(axis=0)
    out = primitive.primitive_from_conserved(m, rho * Y, rho * u, rho * E, 1200.0)
    r2, Y2, u2, T2, p2, st = out
    assert np.all(st > 0)
    np.testing.assert_allclose(r2, rho, rtol=1e-14)
    np.testing.assert_allclose(Y2, Y, rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(u2, u, rtol=1e-13)
    np.testing.assert_allclose(T2, T, rtol=1e-11)
    np.testing.assert_allclose(p2, p, rtol=1e-11)
