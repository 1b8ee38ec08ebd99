"""Pins of the oracle's chemical Jacobian (oracle/jacobian.py) to facts from
outside it: a closed form through the energy constraint, conservation of
mass and atoms in every column, the implicit-function form of the fixed-
energy Jacobian, and central differences of the source terms through the
real Newton solve."""

import numpy as np
import pytest

import mechs
from oracle import eos, jacobian, kinetics, newton, thermo
from oracle.constants import GAS_CONSTANT as RU
from pyro_synth.states import draw_states


def _state(m, cfg, n, first=0):
    T, p, Y = draw_states(cfg, n, m.S, first=first)
    return T, eos.density(m, p, T, Y), Y


def test_single_reaction_closed_form(tmp_path):
    """A + B -> C + D with k = A T (b = 1, Ea = 0), constant cp, W = 1:
    S_C = -S_A = A T rho^2 Y_A Y_B.  At fixed energy T moves with Y through
    dT/dY_k = -e_k/c_v, e_k = R((a1_k - 1) T + a6_k), c_v = sum Y R (a1 - 1)."""
    S = 4
    a1 = np.array([3.5, 4.0, 2.5, 3.0])
    a6 = np.array([-1000.0, 2000.0, 500.0, -300.0])
    a = mechs.constant_cp(S, a1, a6, 20.0)
    m = mechs.make(str(tmp_path / "j.pyromech"), W=[1.0] * S, nasa_low=a,
                   reactions=[dict(reac=[(0, 1), (1, 1)], prod=[(2, 1), (3, 1)],
                                   arrh=(np.log(3.0), 1.0, 0.0), reversible=False)])
    T = np.array([900.0, 1700.0])
    Y = np.array([[0.3, 0.05], [0.2, 0.6], [0.4, 0.1], [0.1, 0.25]])
    rho = np.array([1.7, 0.6])
    r = 3.0 * T * rho**2                       # dS_C/d(Y_A Y_B)
    JT = np.zeros((S, S, 2))
    for j, sgn in ((0, -1), (1, -1), (2, 1), (3, 1)):
        JT[j, 0] = sgn * r * Y[1]
        JT[j, 1] = sgn * r * Y[0]
    np.testing.assert_allclose(jacobian.jacobian(m, rho, T, Y, fixed="temperature"), JT,
                               rtol=4e-15, atol=0)
    dSdT = np.array([-1, -1, 1, 1])[:, None] * 3.0 * rho**2 * Y[0] * Y[1]
    ek = RU * ((a1[:, None] - 1) * T + a6[:, None])
    cv = (Y * RU * (a1[:, None] - 1)).sum(axis=0)
    JE = JT + dSdT[:, None, :] * (-ek / cv)[None, :, :]
    np.testing.assert_allclose(jacobian.jacobian(m, rho, T, Y), JE, rtol=1e-13, atol=0)


@pytest.mark.parametrize("cfg", [0, 1])
def test_columns_conserve_mass_and_atoms(cfg):
    """sum_j S_j = sum_j W_j omega_j = 0 and sum_j a_ej omega_j = 0 for every
    state, so every column of J sums to zero (both weightings)."""
    m = mechs.load_config(cfg)
    T, rho, Y = _state(m, cfg, 6, first=123)
    J = jacobian.jacobian(m, rho, T, Y)
    scale = np.abs(J).sum(axis=0)                       # (S, n) per column
    assert np.all(np.abs(J.sum(axis=0)) <= 1e-12 * scale + 1e-300)
    atoms = np.einsum("ej,jkn->ekn", m.composition / m.W[None, :], J)
    ascale = np.einsum("ej,jkn->ekn", np.abs(m.composition) / m.W[None, :], np.abs(J))
    assert np.all(np.abs(atoms) <= 1e-12 * ascale + 1e-300)


def test_fixed_energy_is_the_implicit_function_form(mech0):
    """dS/dY at fixed e equals dS/dY at fixed T plus dS/dT times
    dT/dY_k = -e_k(T)/c_v(T, Y), the derivative of the root of e(T, Y) = e;
    dS/dT by its own complex step."""
    m = mech0
    T, rho, Y = _state(m, 0, 5, first=77)
    JE = jacobian.jacobian(m, rho, T, Y)
    JT = jacobian.jacobian(m, rho, T, Y, fixed="temperature")
    dSdT = kinetics.source_terms(m, rho, T + 1e-30j, Y).imag / 1e-30
    dTdY = -thermo.species_internal_energy(m, T) / thermo.mixture_cv(m, T, Y)
    ref = JT + dSdT[:, None, :] * dTdY[None, :, :]
    scale = np.abs(JT) + np.abs(dSdT[:, None, :] * dTdY[None, :, :])
    assert np.all(np.abs(JE - ref) <= 1e-12 * scale.max(axis=(0, 1)) + 1e-300)


def test_central_differences_through_the_newton_solve(mech0):
    """Column k against (S(Y + h e_k) - S(Y - h e_k))/(2h), T from the real
    Newton solve at the state's energy; h = 1e-6 max(Y_k, 1e-3)."""
    m = mech0
    T, rho, Y = _state(m, 0, 4, first=9)
    e = thermo.mixture_internal_energy(m, T, Y)
    J = jacobian.jacobian(m, rho, T, Y)

    def S_of(Yx):
        Tx, st = newton.temperature(m, e, Yx, T)
        assert np.all(st > 0)
        return kinetics.source_terms(m, rho, Tx, Yx)

    for k in range(m.S):
        h = 1e-6 * np.maximum(Y[k], 1e-3)
        Yp, Ym = Y.copy(), Y.copy()
        Yp[k] += h
        Ym[k] -= h
        fd = (S_of(Yp) - S_of(Ym)) / (2 * h)
        ok = Y[k] > 2 * h
        err = np.abs(fd - J[:, k, :])[:, ok]
        assert np.all(err <= 1e-5 * np.abs(J).max(axis=(0, 1))[ok]), (k, err.max())


def test_zero_mass_fraction_has_no_concentration_part(mech0):
    """C_k = rho max(Y_k, 0)/W_k: with Y_k = 0 its column holds only the
    temperature part at fixed energy, and nothing at fixed temperature."""
    m = mech0
    T, rho, Y = _state(m, 0, 3, first=5)
    Y[2] = 0.0
    JT = jacobian.jacobian(m, rho, T, Y, fixed="temperature")
    assert np.all(JT[:, 2, :] == 0.0)
    JE = jacobian.jacobian(m, rho, T, Y)
    dSdT = kinetics.source_terms(m, rho, T + 1e-30j, Y).imag / 1e-30
    dTdY = -thermo.species_internal_energy(m, T)[2] / thermo.mixture_cv(m, T, Y)
    np.testing.assert_allclose(JE[:, 2, :], dSdT * dTdY, rtol=1e-12, atol=1e-300)
