"""Pins of the oracle's reactor steps (oracle/reactor.py): closed-form
amplification factors of both steppers on linear reactions whose temperature
cannot change, conservation of mass and elements, the Crank-Nicolson
residual at the Newton solution, and the local-error orders (5 and 3)."""

import numpy as np
import pytest

import mechs
from oracle import eos, kinetics, reactor, thermo
from pyro_synth.states import draw_states

A_FIT = np.array([3.5, 2e-4, -1e-7, 3e-11, -2e-15, -1000.0, 4.0])


def _isothermal_pair(tmp_path, reversible):
    """A -> B (or A <=> B) and an inert C, all with the same molar mass and
    NASA7 coefficients: e_k is the same function of T for every species, so
    converting A to B leaves T unchanged; K_c = 1 for A <=> B."""
    nasa = np.tile(A_FIT, (3, 1))
    return mechs.make(str(tmp_path / "pair.pyromech"), W=[0.03, 0.03, 0.03],
                      nasa_low=nasa,
                      reactions=[{"reac": [(0, 1)], "prod": [(1, 1)],
                                  "arrh": (np.log(2.0e4), 0.3, 3.0e4),
                                  "reversible": reversible}])


def _state(m, n=5):
    rng = np.random.default_rng(3)
    Y = rng.dirichlet(np.ones(3), n).T
    T = rng.uniform(900.0, 1800.0, n)
    rho = rng.uniform(0.2, 3.0, n)
    return rho, T, Y


def _k(m, T):
    return kinetics.arrhenius(m.arrhenius, T)[0]


@pytest.mark.parametrize("stepper", ["rk4", "cn"])
def test_irreversible_first_order_closed_form(tmp_path, stepper):
    """dY_A/dt = -k Y_A: RK4 multiplies Y_A by 1 - z + z^2/2 - z^3/6 +
    z^4/24, Crank-Nicolson by (1 - z/2)/(1 + z/2), z = k dt."""
    m = _isothermal_pair(tmp_path, reversible=False)
    rho, T, Y = _state(m)
    e = thermo.mixture_internal_energy(m, T, Y)
    k = _k(m, T)
    dt = np.array([0.05, 0.3, 1.0, 0.7, 0.01]) / k
    z = k * dt
    if stepper == "rk4":
        Yn, Tn = reactor.rk4_step(m, rho, e, Y, T, dt)
        g = 1 - z + z**2 / 2 - z**3 / 6 + z**4 / 24
    else:
        Yn, Tn, st = reactor.cn_step(m, rho, e, Y, T, dt)
        assert np.all(st > 0)
        g = (1 - z / 2) / (1 + z / 2)
    np.testing.assert_allclose(Yn[0], Y[0] * g, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(Yn[1], Y[1] + Y[0] * (1 - g), rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(Yn[2], Y[2])
    np.testing.assert_allclose(Tn, T, rtol=1e-12)


@pytest.mark.parametrize("stepper", ["rk4", "cn"])
def test_reversible_pair_closed_form(tmp_path, stepper):
    """A <=> B with K_c = 1: Y_A + Y_B is conserved and Y_A - Y_B decays by
    the stepper's factor at z = 2 k dt."""
    m = _isothermal_pair(tmp_path, reversible=True)
    rho, T, Y = _state(m)
    e = thermo.mixture_internal_energy(m, T, Y)
    k = _k(m, T)
    dt = np.array([0.05, 0.3, 1.0, 0.7, 0.01]) / k
    z = 2 * k * dt
    if stepper == "rk4":
        Yn, Tn = reactor.rk4_step(m, rho, e, Y, T, dt)
        g = 1 - z + z**2 / 2 - z**3 / 6 + z**4 / 24
    else:
        Yn, Tn, st = reactor.cn_step(m, rho, e, Y, T, dt)
        g = (1 - z / 2) / (1 + z / 2)
    np.testing.assert_allclose(Yn[0] + Yn[1], Y[0] + Y[1], rtol=1e-14)
    np.testing.assert_allclose(Yn[0] - Yn[1], (Y[0] - Y[1]) * g, rtol=1e-11, atol=1e-14)


def _cfg0_state(n=6, first=40):
    m = mechs.load_config(0)
    T, p, Y = draw_states(0, n, m.S, first=first)
    rho = eos.density(m, p, T, Y)
    e = thermo.mixture_internal_energy(m, T, Y)
    f, _ = reactor.rhs(m, rho, e, Y, T)
    # a step well inside the fastest local time scale of each cell
    with np.errstate(divide="ignore"):
        tau = np.min(np.where(np.abs(f) > 0, np.maximum(Y, 1e-3) / np.abs(f), np.inf), axis=0)
    return m, rho, e, T, Y, 0.05 * tau


@pytest.mark.parametrize("stepper", ["rk4", "cn"])
def test_mass_and_elements_conserved(stepper):
    m, rho, e, T, Y, dt = _cfg0_state()
    if stepper == "rk4":
        Yn, Tn = reactor.rk4_step(m, rho, e, Y, T, dt)
    else:
        Yn, Tn, st = reactor.cn_step(m, rho, e, Y, T, dt)
        assert np.all(st > 0)
    np.testing.assert_allclose(Yn.sum(axis=0), Y.sum(axis=0), rtol=1e-13)
    A = m.composition / m.W[None, :]        # moles of element per kg of species
    np.testing.assert_allclose(A @ Yn, A @ Y, rtol=1e-12)
    np.testing.assert_allclose(thermo.mixture_internal_energy(m, Tn, Yn), e, rtol=1e-12)


def test_crank_nicolson_residual_vanishes():
    m, rho, e, T, Y, dt = _cfg0_state()
    Yn, Tn, st = reactor.cn_step(m, rho, e, Y, T, 20 * dt)
    assert np.all(st > 0)
    f0, _ = reactor.rhs(m, rho, e, Y, T)
    f1, _ = reactor.rhs(m, rho, e, Yn, Tn)
    F = Yn - Y - 0.5 * 20 * dt * (f0 + f1)
    scale = np.abs(Y) + 10 * dt * (np.abs(f0) + np.abs(f1))
    assert np.max(np.abs(F) / scale) < 1e-10


@pytest.mark.parametrize("stepper,order", [("rk4", 5), ("cn", 3)])
def test_local_error_order(stepper, order):
    """One step of dt against two of dt/2: the difference falls by
    2^order when dt is halved (local error O(dt^(p+1)))."""
    m, rho, e, T, Y, dt = _cfg0_state(n=4, first=90)

    def step(Y0, T0, h):
        if stepper == "rk4":
            return reactor.rk4_step(m, rho, e, Y0, T0, h)
        Yn, Tn, st = reactor.cn_step(m, rho, e, Y0, T0, h)
        return Yn, Tn

    def defect(h):
        Y1, _ = step(Y, T, h)
        Yh, Th = step(Y, T, h / 2)
        Y2, _ = step(Yh, Th, h / 2)
        return np.max(np.abs(Y1 - Y2), axis=0)

    d1 = defect(dt)
    d2 = defect(dt / 2)
    ratio = d1 / d2
    assert np.all(ratio > 0.6 * 2**order) and np.all(ratio < 1.6 * 2**order), ratio
