"""Pins of the CPU oracle to facts that do not come from the oracle itself:
the paper's worked example, textbook closed forms, quadrature, chemical
equilibrium from the chemical potentials, conservation laws, complex step
against finite differences, and equivariance under relabelling.
"""

import os
import subprocess
import sys

import numpy as np
import pytest
from scipy import integrate, optimize

import mechs
from oracle import eos, gradients, kinetics, mechfile, newton, thermo
from oracle.constants import GAS_CONSTANT as RU, ONE_ATM
from pyro_synth.states import draw_states

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


def _state(m, cfg, n):
    T, p, Y = draw_states(cfg, n, m.S)
    return T, p, Y, eos.density(m, p, T, Y)


# ---------------------------------------------------------------- worked example

def test_arrhenius_worked_example(tmp_path):
    """Sec. 2.2-2.4: A = 35127309770106.477, b = -0.7, theta = 8590 K renders
    to exp(31.19 - 0.7 log T - 8590/T) C0 C1 on the demo grid."""
    g = _golden("arrhenius_worked_example.txt")
    lnA = np.log(g["pre_exponential_factor"])
    assert round(lnA, int(g["printed_log_a_decimals"])) == g["printed_log_a"]
    b = g["temperature_exponent"]
    Ea = g["activation_temperature"] * RU
    m = mechs.make(str(tmp_path / "ex.pyromech"), W=[1.0] * 4,
                   nasa_low=mechs.constant_cp(4, 3.5, 0.0, 0.0),
                   reactions=[dict(reac=[(0, 1), (1, 1)], prod=[(2, 1), (3, 1)],
                                   arrh=(lnA, b, Ea), reversible=False)])
    T = np.linspace(g["grid_start"], g["grid_stop"], int(g["grid_num"]),
                    endpoint=False)
    Y = np.zeros((4, T.size))
    Y[0] = g["concentration_m"]
    Y[1] = g["concentration_n"]
    Rf, Rr, phi, q = kinetics.rates_of_progress(m, np.ones_like(T), T, Y)
    printed = (np.exp(g["printed_log_a"] + b * np.log(T)
                      - g["activation_temperature"] / T)
               * g["concentration_m"] * g["concentration_n"])
    # the printed ln A is rounded to two decimals
    np.testing.assert_allclose(q[0], printed * np.exp(lnA - g["printed_log_a"]),
                               rtol=1e-14)
    np.testing.assert_allclose(q[0], printed, rtol=abs(lnA - 31.19) * 1.01 + 1e-14)
    assert np.all(Rr == 0)
    # the same rate as a power law: A T^b exp(-theta/T)
    np.testing.assert_allclose(
        q[0], g["pre_exponential_factor"] * T**b
        * np.exp(-g["activation_temperature"] / T) * 0.16, rtol=1e-13)


# ---------------------------------------------------------------- thermo

def test_constant_cp_closed_forms():
    """a2..a5 = 0: cp = R a1, h = R (a1 T + a6), s = R (a1 ln T + a7)."""
    rng = np.random.default_rng(5)
    a = mechs.constant_cp(6, rng.uniform(2.5, 5, 6), rng.uniform(-3e4, 3e4, 6),
                          rng.uniform(-5, 30, 6))
    T = np.linspace(250.0, 3400.0, 37)
    np.testing.assert_allclose(thermo.cp_R_poly(a, T),
                               np.broadcast_to(a[:, :1], (6, T.size)), rtol=0)
    scale = np.abs(a[:, :1] * T) + np.abs(a[:, 5:6])
    assert np.all(np.abs(thermo.h_RT_poly(a, T) * T - (a[:, :1] * T + a[:, 5:6]))
                  <= 1e-14 * scale)
    np.testing.assert_allclose(thermo.s_R_poly(a, T),
                               a[:, :1] * np.log(T) + a[:, 6:7], rtol=1e-14)


@pytest.mark.parametrize("cfg", [0, 1])
def test_enthalpy_entropy_are_integrals_of_cp(cfg):
    """h(T2) - h(T1) = int cp dT and s(T2) - s(T1) = int cp/T dT, inside each
    range, by adaptive quadrature; plus central differences dh/dT = cp."""
    m = mechs.load_config(cfg)
    for T1, T2 in [(310.0, 940.0), (1060.0, 3300.0)]:
        Tp = np.array([T1, T2])
        h = thermo.species_h_RT(m, Tp) * Tp
        s = thermo.species_s_R(m, Tp)
        for k in range(m.S):
            cp = lambda t: thermo.species_cp_R(m, np.array([t]))[k, 0]  # noqa: E731
            ih = integrate.quad(cp, T1, T2, epsabs=0, epsrel=1e-13)[0]
            is_ = integrate.quad(lambda t: cp(t) / t, T1, T2, epsabs=0, epsrel=1e-13)[0]
            assert abs((h[k, 1] - h[k, 0]) - ih) <= 1e-11 * abs(ih) + 1e-9
            assert abs((s[k, 1] - s[k, 0]) - is_) <= 1e-11 * abs(is_) + 1e-12
    T = np.array([500.0, 800.0, 1500.0, 2800.0])
    d = 1e-3
    dh = (thermo.species_h_RT(m, T + d) * (T + d)
          - thermo.species_h_RT(m, T - d) * (T - d)) / (2 * d)
    np.testing.assert_allclose(dh, thermo.species_cp_R(m, T), rtol=1e-8)
    ds = (thermo.species_s_R(m, T + d) - thermo.species_s_R(m, T - d)) / (2 * d)
    np.testing.assert_allclose(ds, thermo.species_cp_R(m, T) / T, rtol=1e-8)


@pytest.mark.parametrize("cfg", [0, 1, 3])
def test_stored_mechanisms_continuous_at_T_mid(cfg):
    m = mechs.load_config(cfg)
    Tm = m.T_mid[0]
    assert np.all(m.T_mid == Tm)
    for poly, scale in [(thermo.cp_R_poly, 1.0), (thermo.h_RT_poly, Tm),
                        (thermo.s_R_poly, 1.0)]:
        lo = poly(m.nasa_low, np.array([Tm]))[:, 0] * scale
        hi = poly(m.nasa_high, np.array([Tm]))[:, 0] * scale
        np.testing.assert_allclose(lo, hi, rtol=1e-12, atol=1e-9)
    Tg = np.linspace(200.0, 3500.0, 200)
    # cp > R keeps c_v > 0, so e(T) is strictly increasing
    assert np.all(thermo.species_cp_R(m, Tg) > 1.0)


def test_range_selection_at_and_around_T_mid(tmp_path):
    """T <= T_mid uses the low set (a tie goes low)."""
    lo = mechs.constant_cp(1, 3.0, 0.0, 0.0)
    hi = mechs.constant_cp(1, 4.0, 0.0, 0.0)
    m = mechs.make(str(tmp_path / "r.pyromech"), W=[0.03], nasa_low=lo,
                   nasa_high=hi, reactions=[dict(reac=[(0, 1)], prod=[(0, 1)],
                                                 arrh=(0, 0, 0))])
    cp = thermo.species_cp_R(m, np.array([999.0, 1000.0, 1000.0000001, 2000.0]))
    assert cp[0].tolist() == [3.0, 3.0, 4.0, 4.0]


# ---------------------------------------------------------------- EOS / [M]

def test_third_body_unit_efficiencies_equal_total_concentration(mech1):
    """With every efficiency 1, [M] = sum C_k = rho/W = p/(R T) (eq. eos)."""
    T, p, Y, rho = _state(mech1, 1, 64)
    C = kinetics.concentrations(mech1, rho, Y)
    np.testing.assert_allclose(C.sum(axis=0), p / (RU * T), rtol=1e-13)
    np.testing.assert_allclose(eos.pressure(mech1, rho, T, Y), p, rtol=1e-14)
    single = np.zeros_like(Y)
    single[7] = 1.0
    np.testing.assert_allclose(eos.mixture_molar_mass(mech1, single),
                               mech1.W[7], rtol=1e-15)


# ---------------------------------------------------------------- conservation

@pytest.mark.parametrize("cfg", [0, 1])
def test_element_and_mass_conservation(cfg):
    m = mechs.load_config(cfg)
    T, p, Y, rho = _state(m, cfg, 200)
    Rf, Rr, phi, q = kinetics.rates_of_progress(m, rho, T, Y)
    w = kinetics.net_production_rates(m, rho, T, Y)
    term = np.abs(m.nu) @ np.abs(q)                    # (S, n) magnitude of the sum
    atoms = m.composition @ w
    np.testing.assert_array_less(np.abs(atoms), 1e-13 * (np.abs(m.composition) @ term) + 1e-300)
    mass = m.W @ w
    np.testing.assert_array_less(np.abs(mass), 1e-13 * (m.W @ term) + 1e-300)
    inert = np.nonzero(np.abs(m.nu).sum(axis=1) == 0)[0]
    if cfg == 1:
        assert inert.size == 1
    assert np.all(w[inert] == 0.0)


# ---------------------------------------------------------------- equilibrium

def _equilibrium_state(m, T, C_given, last):
    """Concentrations at chemical equilibrium of the single reaction of ``m``:
    sum_k nu_k mu_k = 0 with mu_k/(R T) = g0_k/(R T) + ln(C_k R T/p0), solved
    for the concentration of species ``last``."""
    g = thermo.species_g_RT(m, np.array([T]))[:, 0]
    nu = m.nu[:, 0]
    acc = 0.0
    for k in range(m.S):
        if k != last and nu[k] != 0:
            acc += nu[k] * (g[k] + np.log(C_given[k] * RU * T / ONE_ATM))
    lnC = (-acc / nu[last]) - g[last] - np.log(RU * T / ONE_ATM)
    C = np.array(C_given, float)
    C[last] = np.exp(lnC)
    return C


@pytest.mark.parametrize("reac,prod,rtype", [
    ([(0, 1), (1, 1)], [(2, 1)], 0),            # A + B <=> C    (dnu = -1)
    ([(0, 1), (1, 1)], [(2, 1), (3, 1)], 0),    # A + B <=> C + D (dnu = 0)
    ([(0, 1)], [(1, 1), (2, 1)], 0),            # A <=> B + C    (dnu = +1)
    ([(0, 2)], [(1, 1)], 0),                    # 2A <=> B
    ([(0, 1), (1, 1)], [(2, 1)], 1),            # A + B + M <=> C + M
])
def test_detailed_balance_at_gibbs_equilibrium(tmp_path, reac, prod, rtype):
    rng = np.random.default_rng(11)
    S = 4
    a = mechs.constant_cp(S, rng.uniform(2.5, 5, S), rng.uniform(-2e4, 2e4, S),
                          rng.uniform(15, 30, S))
    m = mechs.make(str(tmp_path / "eq.pyromech"), W=[0.002, 0.016, 0.018, 0.03],
                   nasa_low=a, nasa_high=a,
                   reactions=[dict(reac=reac, prod=prod, type=rtype,
                                   arrh=(np.log(3e9), 0.4, 5e4),
                                   eff=rng.uniform(0.5, 12, S))])
    for T in (450.0, 1200.0, 2700.0):
        last = prod[-1][0]
        C = _equilibrium_state(m, T, rng.uniform(0.5, 5.0, S), last)
        rho = 1.3
        Y = (C * m.W / rho)[:, None]
        Rf, Rr, phi, q = kinetics.rates_of_progress(m, np.array([rho]),
                                                    np.array([T]), Y)
        assert abs(Rf[0, 0] - Rr[0, 0]) <= 1e-12 * Rf[0, 0]
        assert abs(q[0, 0]) <= 1e-12 * Rf[0, 0] * phi[0, 0]
    # the reverse reaction has the reciprocal constant
    m2 = mechs.make(str(tmp_path / "eq2.pyromech"), W=m.W, nasa_low=a,
                    nasa_high=a, reactions=[dict(reac=prod, prod=reac,
                                                 arrh=(0, 0, 0))])
    Tg = np.array([400.0, 1500.0])
    np.testing.assert_allclose(kinetics.equilibrium_constants(m, Tg)
                               * kinetics.equilibrium_constants(m2, Tg), 1.0,
                               rtol=1e-13)


# ---------------------------------------------------------------- closed forms

def test_single_reaction_closed_forms(tmp_path):
    S = 4
    a = mechs.constant_cp(S, 3.5, 0.0, 20.0)
    T = np.array([700.0, 1900.0])
    Y = np.array([[0.3, 0.05], [0.2, 0.6], [0.4, 0.1], [0.1, 0.25]])
    rho = np.array([1.7, 0.6])
    C = rho * Y                   # W = 1 kg/mol
    # A + B -> C + D, k = A exactly (b = 0, Ea = 0)
    m = mechs.make(str(tmp_path / "a.pyromech"), W=[1.0] * S, nasa_low=a,
                   reactions=[dict(reac=[(0, 1), (1, 1)], prod=[(2, 1), (3, 1)],
                                   arrh=(np.log(2.5), 0, 0), reversible=False)])
    w = kinetics.net_production_rates(m, rho, T, Y)
    r = 2.5 * C[0] * C[1]
    np.testing.assert_allclose(w, np.stack([-r, -r, r, r]), rtol=1e-15)
    # 2A -> B
    m = mechs.make(str(tmp_path / "b.pyromech"), W=[1.0] * S, nasa_low=a,
                   reactions=[dict(reac=[(0, 2)], prod=[(1, 1)],
                                   arrh=(np.log(2.5), 0, 0), reversible=False)])
    w = kinetics.net_production_rates(m, rho, T, Y)
    r = 2.5 * C[0] ** 2
    np.testing.assert_allclose(w[:2], np.stack([-2 * r, r]), rtol=1e-15)
    assert np.all(w[2:] == 0)
    # the same with a third body of unit efficiencies: times sum C = rho/W
    m = mechs.make(str(tmp_path / "c.pyromech"), W=[1.0] * S, nasa_low=a,
                   reactions=[dict(reac=[(0, 1), (1, 1)], prod=[(2, 1), (3, 1)],
                                   type=1, arrh=(np.log(2.5), 0, 0),
                                   reversible=False)])
    w = kinetics.net_production_rates(m, rho, T, Y)
    np.testing.assert_allclose(w[0], -2.5 * C[0] * C[1] * C.sum(axis=0), rtol=1e-15)
    # negative mass fractions count as zero
    Yn = Y.copy()
    Yn[1, 0] = -0.2
    w = kinetics.net_production_rates(m, rho, T, Yn)
    assert w[0, 0] == 0.0


def _falloff_mech(path, rtype, A_inf, A0, troe=(0.5, 100.0, 1000.0, 1000.0)):
    a = mechs.constant_cp(3, 3.5, 0.0, 20.0)
    return mechs.make(path, W=[1.0] * 3, nasa_low=a,
                      reactions=[dict(reac=[(0, 1), (1, 1)], prod=[(2, 1)],
                                      type=rtype, arrh=(np.log(A_inf), 0, 0),
                                      low=(np.log(A0), 0, 0), troe=troe,
                                      reversible=False)])


def test_lindemann_closed_form_and_limits(tmp_path):
    T = np.array([900.0])
    Y = np.array([[0.2], [0.3], [0.5]])
    rho = np.array([1.6])
    C = rho * Y[:, 0]                          # [M] = 1.6 with unit efficiencies
    for A0, A_inf in [(1e3, 5.0), (1e-3, 5.0), (7.0, 5.0)]:
        m = _falloff_mech(str(tmp_path / "l.pyromech"), 2, A_inf, A0)
        k, M = kinetics.rate_coefficients(m, T, rho * Y)
        Pr = A0 * 1.6 / A_inf
        np.testing.assert_allclose(k[0], A_inf * Pr / (1 + Pr), rtol=1e-14)
        w = kinetics.net_production_rates(m, rho, T, Y)
        # [M] enters only through P_r
        np.testing.assert_allclose(w[2], k[0] * C[0] * C[1], rtol=1e-15)
    m = _falloff_mech(str(tmp_path / "hi.pyromech"), 2, 5.0, 1e12)
    np.testing.assert_allclose(kinetics.rate_coefficients(m, T, rho * Y)[0][0], 5.0, rtol=1e-11)
    m = _falloff_mech(str(tmp_path / "lo.pyromech"), 2, 5.0, 1e-12)
    np.testing.assert_allclose(kinetics.rate_coefficients(m, T, rho * Y)[0][0],
                               1.6e-12, rtol=1e-11)


def test_troe_special_cases(tmp_path):
    T = np.array([900.0])
    Y = np.array([[0.2], [0.3], [0.5]])
    # F_cent = 1 (alpha = 0, T*** and T** huge): Troe reduces to Lindemann
    big = 1e300
    mt = _falloff_mech(str(tmp_path / "t.pyromech"), 3, 5.0, 7.0,
                       troe=(0.0, big, 100.0, big))
    ml = _falloff_mech(str(tmp_path / "l.pyromech"), 2, 5.0, 7.0)
    np.testing.assert_allclose(kinetics.rate_coefficients(mt, T, Y)[0],
                               kinetics.rate_coefficients(ml, T, Y)[0], rtol=1e-15)
    # alpha = 1, T* = T/ln 2, T** huge: F_cent = 1/2; at log10 Pr = -c the
    # broadening factor equals F_cent, and far from it F -> F_cent^(d^2/(1+d^2))
    troe = (1.0, 1e3, 900.0 / np.log(2.0), big)
    c = -0.4 - 0.67 * np.log10(0.5)
    F = kinetics.troe_factor(troe, T, np.array([10.0 ** (-c)]))
    np.testing.assert_allclose(F, 0.5, rtol=1e-14)
    for Pr in (1e200, 1e-200):
        F = kinetics.troe_factor(troe, T, np.array([Pr]))
        np.testing.assert_allclose(F, 0.5 ** (0.14**2 / (1 + 0.14**2)), rtol=2e-3)
    assert kinetics.troe_factor(troe, T, np.array([0.0]))[0] > 0
    # in a rate: at that P_r the Troe coefficient is half the Lindemann one
    Y = np.array([[0.2], [0.3], [0.5]])
    A0 = 10.0 ** (-c) * 5.0 / 1.6
    mt = _falloff_mech(str(tmp_path / "t2.pyromech"), 3, 5.0, A0, troe=troe)
    ml = _falloff_mech(str(tmp_path / "l2.pyromech"), 2, 5.0, A0)
    np.testing.assert_allclose(kinetics.rate_coefficients(mt, T, 1.6 * Y)[0],
                               0.5 * kinetics.rate_coefficients(ml, T, 1.6 * Y)[0],
                               rtol=1e-13)


def test_troe_hand_evaluated_values(tmp_path):
    """F_cent = 1/2 (alpha = 1, T* = T/ln 2, T*** and T** huge), evaluated by
    hand: log10 F_cent = -0.30102999566398120, c = -0.4 - 0.67 log10 F_cent =
    -0.19830990290513262, n = 0.75 - 1.27 log10 F_cent = 1.1323080944932562,
    d = 0.14.  At x = log10 P_r + c = 1: f1 = 1/(n - d) = 1.0077515295394943 and
    F = 2^(-1/(1 + f1^2)) = 0.70900157806297...; at x = -2: f1 = -2/(n + 2d) =
    -1.4161216010856406, F = 0.79403011576779...  The pole of f1 at x = n/d
    gives F = 1, and f1 = +-1 at x = n/(1 + d) and x = -n/(1 - d) gives
    F = sqrt(F_cent): both place n and d independently of the centre value."""
    big = 1e300
    T = np.array([900.0])
    troe = (1.0, big, 900.0 / np.log(2.0), big)
    c = -0.19830990290513262
    n = 1.1323080944932562
    for x, F_hand in ((1.0, 0.709001578062973), (-2.0, 0.794030115767798)):
        Pr = np.array([10.0 ** (x - c)])
        np.testing.assert_allclose(kinetics.troe_factor(troe, T, Pr), F_hand, rtol=1e-13)
    # next to the pole of f1 the factor is one
    Pr = np.array([10.0 ** (n / 0.14 * (1 - 1e-9) - c)])
    assert abs(kinetics.troe_factor(troe, T, Pr)[0] - 1.0) <= 1e-12
    for x in (n / 1.14, -n / 0.86):
        F = kinetics.troe_factor(troe, T, np.array([10.0 ** (x - c)]))
        np.testing.assert_allclose(F, np.sqrt(0.5), rtol=1e-12)
    # the same factor inside a falloff rate coefficient: k = k_inf Pr/(1+Pr) F
    Y = np.array([[0.2], [0.3], [0.5]])
    rho = 1.6                                  # W = 1: [M] = rho sum Y = 1.6
    Pr = 10.0 ** (1.0 - c)
    A0 = Pr * 5.0 / 1.6
    mt = _falloff_mech(str(tmp_path / "t.pyromech"), 3, 5.0, A0, troe=troe)
    k, M = kinetics.rate_coefficients(mt, T, rho * Y)
    np.testing.assert_allclose(M[0], 1.6, rtol=1e-15)
    np.testing.assert_allclose(k[0], 5.0 * Pr / (1 + Pr) * 0.709001578062973, rtol=1e-13)


def _eff_mech(path, eff_a, eff_b, rtype_b=1, A0=None):
    """A + B + M -> C + M (efficiencies eff_a) and B + C + M -> A + D + M
    or a falloff B + C -> D (efficiencies eff_b), constant rates."""
    a = mechs.constant_cp(4, 3.5, 0.0, 20.0)
    r2 = dict(reac=[(1, 1), (2, 1)], prod=[(0, 1), (3, 1)], type=rtype_b,
              arrh=(np.log(0.75), 0, 0), eff=eff_b, reversible=False)
    if rtype_b >= 2:
        r2.update(prod=[(3, 1)], low=(np.log(A0), 0, 0))
    return mechs.make(path, W=[1.0] * 4, nasa_low=a, reactions=[
        dict(reac=[(0, 1), (1, 1)], prod=[(2, 1)], type=1,
             arrh=(np.log(2.5), 0, 0), eff=eff_a, reversible=False), r2])


def test_third_body_efficiencies_hand_evaluated(tmp_path):
    """Each third-body reaction weights the concentrations with its own
    efficiency row: q = k C_A C_B (2 C_A + 0.5 C_B + 7 C_C + 3 C_D) for the
    first reaction and k C_B C_C (4 C_A + 1.5 C_B + 0.25 C_C + 9 C_D) for the
    second (W = 1 kg/mol, so C = rho Y)."""
    T = np.array([700.0, 1900.0])
    Y = np.array([[0.3, 0.05], [0.2, 0.6], [0.4, 0.1], [0.1, 0.25]])
    rho = np.array([1.7, 0.6])
    C = rho * Y
    m = _eff_mech(str(tmp_path / "e.pyromech"), (2.0, 0.5, 7.0, 3.0), (4.0, 1.5, 0.25, 9.0))
    Rf, Rr, phi, q = kinetics.rates_of_progress(m, rho, T, Y)
    M1 = 2.0 * C[0] + 0.5 * C[1] + 7.0 * C[2] + 3.0 * C[3]
    M2 = 4.0 * C[0] + 1.5 * C[1] + 0.25 * C[2] + 9.0 * C[3]
    np.testing.assert_allclose(q[0], 2.5 * C[0] * C[1] * M1, rtol=1e-15)
    np.testing.assert_allclose(q[1], 0.75 * C[1] * C[2] * M2, rtol=1e-15)
    w = kinetics.net_production_rates(m, rho, T, Y)
    np.testing.assert_allclose(w[2], 2.5 * C[0] * C[1] * M1 - 0.75 * C[1] * C[2] * M2,
                               rtol=1e-14)
    np.testing.assert_allclose(w[3], 0.75 * C[1] * C[2] * M2, rtol=1e-15)


@pytest.mark.parametrize("rtype", [2, 3])
def test_falloff_efficiencies_hand_evaluated(tmp_path, rtype):
    """Falloff B + C (+M) -> D: P_r = k0 [M]/k_inf with [M] = 4 C_A + 1.5 C_B
    + 0.25 C_C + 9 C_D; Lindemann k = k_inf P_r/(1 + P_r); Troe with F_cent = 1
    (alpha = 0, T*** and T** huge) gives the same; [M] does not multiply q."""
    T = np.array([900.0, 1500.0])
    Y = np.array([[0.3, 0.05], [0.2, 0.6], [0.4, 0.1], [0.1, 0.25]])
    rho = np.array([1.7, 0.6])
    C = rho * Y
    A0 = 3.0
    m = _eff_mech(str(tmp_path / "f.pyromech"), (2.0, 0.5, 7.0, 3.0),
                  (4.0, 1.5, 0.25, 9.0), rtype_b=rtype, A0=A0)
    if rtype == 3:
        big = 1e300
        m = mechs.make(str(tmp_path / "f3.pyromech"), W=m.W,
                       nasa_low=mechs.constant_cp(4, 3.5, 0.0, 20.0),
                       reactions=[dict(reac=[(1, 1), (2, 1)], prod=[(3, 1)], type=3,
                                       arrh=(np.log(0.75), 0, 0), low=(np.log(A0), 0, 0),
                                       troe=(0.0, big, 100.0, big),
                                       eff=(4.0, 1.5, 0.25, 9.0), reversible=False)])
    Rf, Rr, phi, q = kinetics.rates_of_progress(m, rho, T, Y)
    M = 4.0 * C[0] + 1.5 * C[1] + 0.25 * C[2] + 9.0 * C[3]
    Pr = A0 * M / 0.75
    j = m.R - 1
    np.testing.assert_allclose(q[j], 0.75 * Pr / (1 + Pr) * C[1] * C[2], rtol=1e-14)


# ---------------------------------------------------------------- Newton

@pytest.mark.parametrize("cfg", [0, 1])
def test_newton_round_trip(cfg):
    m = mechs.load_config(cfg)
    T, p, Y, rho = _state(m, cfg, 300)
    e = thermo.mixture_internal_energy(m, T, Y)
    for guess in (1200.0, T * np.random.default_rng(1).uniform(0.7, 1.3, T.size)):
        Tn, st = newton.temperature(m, e, Y, guess)
        assert np.all(st > 0)
        np.testing.assert_allclose(Tn, T, rtol=1e-12)


def test_newton_constant_cp_closed_form(tmp_path):
    """e = sum Y_k R ((a1_k - 1) T + a6_k)/W_k is linear in T: one update
    lands on the root, the second confirms it."""
    rng = np.random.default_rng(3)
    S = 5
    a = mechs.constant_cp(S, rng.uniform(2.5, 5, S), rng.uniform(-2e4, 2e4, S), 10.0)
    W = rng.uniform(0.002, 0.05, S)
    m = mechs.make(str(tmp_path / "n.pyromech"), W=W, nasa_low=a,
                   reactions=[dict(reac=[(0, 1)], prod=[(1, 1)], arrh=(0, 0, 0))])
    Y = rng.dirichlet(np.ones(S), size=50).T
    e = rng.uniform(-5e6, 5e6, 50)
    X = Y / W[:, None]
    T_exact = (e - RU * (X * a[:, 5:6]).sum(0)) / (RU * (X * (a[:, :1] - 1)).sum(0))
    ok = (T_exact > 250) & (T_exact < 3000)
    Tn, st = newton.temperature(m, e[ok], Y[:, ok], 1200.0)
    np.testing.assert_allclose(Tn, T_exact[ok], rtol=1e-13)
    assert np.all((st >= 1) & (st <= 2))


def test_newton_reports_non_convergence(mech0):
    T, p, Y, rho = _state(mech0, 0, 8)
    e = thermo.mixture_internal_energy(mech0, T, Y)
    Tn, st = newton.temperature(mech0, e, Y, 300.0, max_iter=1)
    assert np.all(st == -1)


# ---------------------------------------------------------------- gradients

def _L(m, rho, T, Y, wbar, P):
    return (wbar * kinetics.net_production_rates(m, rho, T, Y, P)).sum()


def _tame(m, path):
    """The reaction network of ``m`` with thermo and rate parameters drawn in
    narrow ranges, so that no term dwarfs the others and finite differences
    resolve almost every derivative."""
    rng = np.random.default_rng(21)
    rs = _as_reactions(m)
    for r in rs:
        r["arrh"] = (rng.uniform(2, 6), rng.uniform(-0.5, 0.5), rng.uniform(0, 2e4))
        if "low" in r:
            r["low"] = (rng.uniform(2, 6), rng.uniform(-0.5, 0.5), rng.uniform(0, 2e4))
            r["troe"] = (0.6, 300.0, 1500.0, 2500.0)
    # every species gets the heat capacity of species 0 and nearby
    # integration constants, which keeps ln K_c of order one
    lo = np.repeat(m.nasa_low[:1], m.S, axis=0)
    hi = np.repeat(m.nasa_high[:1], m.S, axis=0)
    d6 = rng.uniform(-300, 300, m.S)
    d7 = rng.uniform(-0.5, 0.5, m.S)
    lo[:, 5] += d6
    hi[:, 5] += d6
    lo[:, 6] += d7
    hi[:, 6] += d7
    return mechs.make(path, W=m.W, nasa_low=lo, nasa_high=hi, reactions=rs)


@pytest.mark.parametrize("tame", [False, True])
def test_complex_step_matches_central_differences(mech0, tmp_path, tame):
    """Central differences (h = 1e-6 relative; floors ln A 1, b 1, Ea 1e4 J/mol,
    Y 1e-20) agree with the complex step to 1e-5 relative, above the
    differences' own rounding floor 30 eps |L_cell|_abs / h.  On the tame
    variant of the network most entries must sit far above that floor."""
    m = _tame(mech0, str(tmp_path / "tame.pyromech")) if tame else mech0
    T, p, Y, rho = _state(m, 0, 3)
    wbar = np.random.default_rng(2).standard_normal((m.S, 3))
    P = m.parameters()
    Ybar, Tbar, pbar = gradients.vjp(m, rho, T, Y, wbar, P)
    eps = np.finfo(float).eps
    checked = resolved = 0

    def cellL(Tc, Yc, Pc):
        return (wbar * kinetics.net_production_rates(m, rho, Tc, Yc, Pc)).sum(axis=0)

    Labs = np.abs(wbar * kinetics.net_production_rates(m, rho, T, Y, P)).sum(axis=0)

    def check(fd, g, floor):
        nonlocal checked, resolved
        checked += 1
        resolved += abs(g) > 1e3 * floor
        assert abs(fd - g) <= 1e-5 * abs(g) + floor

    for c in range(3):
        for k in range(m.S):
            h = 1e-6 * max(Y[k, c], 1e-20)
            Yp, Ym = Y.copy(), Y.copy()
            Yp[k, c] += h
            Ym[k, c] -= h
            fd = (cellL(T, Yp, P)[c] - cellL(T, Ym, P)[c]) / (2 * h)
            check(fd, Ybar[k, c], 30 * eps * Labs[c] / h)
        h = 1e-6 * T[c]
        Tp, Tm = T.copy(), T.copy()
        Tp[c] += h
        Tm[c] -= h
        fd = (cellL(Tp, Y, P)[c] - cellL(Tm, Y, P)[c]) / (2 * h)
        check(fd, Tbar[c], 30 * eps * Labs[c] / h)
    # a parameter acts on L only through the rate of progress of its own
    # reaction, L = sum_j qbar_j q_j, so its difference quotient is taken on
    # qbar_j q_j, whose rounding floor is far below that of L
    floors = (1.0, 1.0, 1e4)
    qbar = m.nu.T @ wbar
    owner = list(range(m.R)) + [int(j) for j in m.falloff_reactions]
    for i in range(P.shape[0]):
        j = owner[i]
        for c in range(3):
            h = 1e-6 * max(abs(P[i, c]), floors[c])
            Pp, Pm = P.copy(), P.copy()
            Pp[i, c] += h
            Pm[i, c] -= h
            qp = kinetics.rates_of_progress(m, rho, T, Y, Pp)[3][j]
            qm = kinetics.rates_of_progress(m, rho, T, Y, Pm)[3][j]
            fd = (qbar[j] * (qp - qm)).sum() / (2 * h)
            q0 = kinetics.rates_of_progress(m, rho, T, Y, P)[3][j]
            check(fd, pbar[i, c], 30 * eps * np.abs(qbar[j] * q0).sum() / h)
    assert resolved >= (0.8 if tame else 0.5) * checked, (resolved, checked)


@pytest.mark.parametrize("weights", ["mass", "element"])
def test_gradients_vanish_for_conserved_combinations(mech1, weights):
    """sum_k W_k omega_k and sum_k a_ek omega_k vanish for every state, so
    every derivative of them does."""
    m = mech1
    T, p, Y, rho = _state(m, 1, 4)
    if weights == "mass":
        wbar = np.repeat(m.W[:, None], 4, axis=1)
    else:
        wbar = np.repeat(m.composition[1][:, None].astype(float), 4, axis=1)
    Ybar, Tbar, pbar = gradients.vjp(m, rho, T, Y, wbar)
    Ybar_ref, Tbar_ref, pbar_ref = gradients.vjp(
        m, rho, T, Y, np.random.default_rng(0).standard_normal(wbar.shape) * wbar)
    assert np.max(np.abs(Ybar)) <= 1e-11 * np.max(np.abs(Ybar_ref))
    assert np.max(np.abs(Tbar)) <= 1e-11 * np.max(np.abs(Tbar_ref))
    assert np.max(np.abs(pbar)) <= 1e-11 * np.max(np.abs(pbar_ref))


def test_parameter_gradients_of_elementary_reactions(mech1):
    """q_j = k_j (...) with k_j = exp(ln A + b ln T - Ea/(R T)):
    dL/d ln A = sum qbar q, dL/db = sum qbar q ln T, dL/dEa = -sum qbar q/(R T)."""
    m = mech1
    T, p, Y, rho = _state(m, 1, 6)
    wbar = np.random.default_rng(4).standard_normal((m.S, 6))
    _, _, pbar = gradients.vjp(m, rho, T, Y, wbar)
    _, _, _, q = kinetics.rates_of_progress(m, rho, T, Y)
    qbar = m.nu.T @ wbar
    elem = np.nonzero(m.rtype == 0)[0]
    gq = qbar[elem] * q[elem]
    np.testing.assert_allclose(pbar[elem, 0], gq.sum(1), rtol=1e-10,
                               atol=1e-12 * np.abs(gq).sum(1).max())
    np.testing.assert_allclose(pbar[elem, 1], (gq * np.log(T)).sum(1), rtol=1e-10,
                               atol=1e-12 * np.abs(gq * np.log(T)).sum(1).max())
    np.testing.assert_allclose(pbar[elem, 2], -(gq / (RU * T)).sum(1), rtol=1e-10,
                               atol=1e-12 * np.abs(gq / (RU * T)).sum(1).max())


# ---------------------------------------------------------------- relabelling

def _as_reactions(m):
    fo = {int(j): f for f, j in enumerate(m.falloff_reactions)}
    pd = {int(j): i for i, j in enumerate(m.pd_reactions)}
    out = []
    for j in range(m.R):
        r = dict(reac=[(int(k), int(m.nu_f[k, j])) for k in np.nonzero(m.nu_f[:, j])[0]],
                 prod=[(int(k), int(m.nu_r[k, j])) for k in np.nonzero(m.nu_r[:, j])[0]],
                 arrh=tuple(m.arrhenius[j]), type=int(m.rtype[j]),
                 reversible=bool(m.reversible[j]))
        if j in pd:
            r["eff"] = m.efficiency[pd[j]]
        if j in fo:
            r["low"] = tuple(m.falloff_low[fo[j]])
            r["troe"] = tuple(m.troe[fo[j]])
        out.append(r)
    return out


def test_relabelling_species_and_reactions(tmp_path, mech0):
    m = mech0
    T, p, Y, rho = _state(m, 0, 16)
    w = kinetics.net_production_rates(m, rho, T, Y)
    rng = np.random.default_rng(9)
    sp = rng.permutation(m.S)          # new species i is old species sp[i]
    inv = np.argsort(sp)
    rx = rng.permutation(m.R)
    rs = _as_reactions(m)
    new = []
    for j in rx:
        r = dict(rs[j])
        r["reac"] = [(int(inv[k]), v) for k, v in r["reac"]]
        r["prod"] = [(int(inv[k]), v) for k, v in r["prod"]]
        if "eff" in r:
            r["eff"] = r["eff"][sp]
        new.append(r)
    m2 = mechs.make(str(tmp_path / "perm.pyromech"), W=m.W[sp],
                    nasa_low=m.nasa_low[sp], nasa_high=m.nasa_high[sp],
                    reactions=new)
    w2 = kinetics.net_production_rates(m2, rho, T, Y[sp])
    scale = np.abs(m.nu) @ np.abs(kinetics.rates_of_progress(m, rho, T, Y)[3])
    np.testing.assert_array_less(np.abs(w2 - w[sp]), 1e-13 * scale[sp] + 1e-300)


# ---------------------------------------------------------------- the file

def test_reader_rejects_damaged_files(tmp_path):
    blob = open(mechs.config_path(0), "rb").read()
    for bad in (blob[:-9], blob[:40], b"PYROMECX" + blob[8:],
                blob[:8] + b"\x02" + blob[9:],
                blob[:200] + bytes([blob[200] ^ 1]) + blob[201:]):
        with pytest.raises(mechfile.MechanismFileError):
            mechfile.parse(bad)


def test_stored_mechanisms_are_reproducible():
    script = os.path.join(mechs.MECH_DIR, "make_mechanisms.py")
    r = subprocess.run([sys.executable, script, "--check"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
