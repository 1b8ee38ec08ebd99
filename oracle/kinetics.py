"""Net production rates (Sec. A.1): concentrations (eq. concentrations), rate
coefficients (eq. rate_coeff, plus third-body and falloff forms), equilibrium
constants (eq. equil_constants), rates of progress (eq. reaction_rates) and
net production rates (eq. production_rates), evaluated in that order.

Readings:

* negative mass fractions: C_k = rho max(Y_k, 0)/W_k (the paper only
  evaluates positive states).
* Arrhenius: theta_a = Ea/R with Ea in J/mol, k = exp(ln A + b ln T - Ea/(R T)),
  as the paper's own symbolic construction of the expression does (Sec. 2.3).
* third-body reactions (named, not written, in Sec. A.1): the rate of progress
  is multiplied by [M]_j = sum_k eps_jk C_k with one efficiency per species.
* falloff reactions (cited to Troe, not written): P_r = k0 [M]/k_inf,
  k = k_inf P_r/(1 + P_r) F with F = 1 (Lindemann) or the Troe form
  log10 F = log10 F_cent / (1 + f1^2),
  F_cent = (1-alpha) e^(-T/T***) + alpha e^(-T/T*) + e^(-T**/T),
  f1 = (log10 P_r + c)/(n - d (log10 P_r + c)),
  c = -0.4 - 0.67 log10 F_cent, n = 0.75 - 1.27 log10 F_cent, d = 0.14;
  P_r and F_cent are floored at 1e-300 before their logarithms; [M] does not
  multiply the rate of progress of a falloff reaction.
* equilibrium constant exponent: the printed sum has garbled limits; it is
  read as Delta nu_j = sum_k nu_kj over the species (the third body is no
  species), with p0 = 1 atm.
* irreversible reactions have no reverse term.
"""

import numpy as np

from .constants import GAS_CONSTANT, ONE_ATM
from . import thermo

FLOOR = 1e-300


def _real(x):
    return np.real(x)


def concentrations(mech, rho, Y):
    """C_k = rho Y_k / W_k (eq. concentrations), (S, n)."""
    Ypos = np.where(_real(Y) > 0, Y, 0.0)
    return rho * Ypos / mech.W[:, None]


def arrhenius(params, T):
    """k = A T^b exp(-theta_a/T) (eq. rate_coeff) for rows (ln A, b, Ea) of
    ``params``; returns (rows, n)."""
    lnA = params[:, 0][:, None]
    b = params[:, 1][:, None]
    Ea = params[:, 2][:, None]
    return np.exp(lnA + b * np.log(T) - Ea / (GAS_CONSTANT * T))


def third_body_concentrations(mech, C):
    """[M]_i = sum_k eps_ik C_k for the reactions of class >= 1, in the order
    of ``mech.pd_reactions``; (n_pd, n)."""
    M = np.zeros((len(mech.pd_reactions), C.shape[1]), dtype=C.dtype)
    for i in range(len(mech.pd_reactions)):
        for k in range(mech.S):
            M[i] = M[i] + mech.efficiency[i, k] * C[k]
    return M


def troe_factor(troe, T, Pr):
    """Broadening factor F of one Troe falloff reaction, per cell."""
    alpha, T3, T1, T2 = troe
    Fcent = ((1 - alpha) * np.exp(-T / T3) + alpha * np.exp(-T / T1)
             + np.exp(-T2 / T))
    Fcent = np.where(_real(Fcent) > FLOOR, Fcent, FLOOR)
    log_Fcent = np.log10(Fcent)
    c = -0.4 - 0.67 * log_Fcent
    n = 0.75 - 1.27 * log_Fcent
    d = 0.14
    Pr = np.where(_real(Pr) > FLOOR, Pr, FLOOR)
    x = np.log10(Pr) + c
    with np.errstate(divide="ignore", invalid="ignore"):
        f1 = x / (n - d * x)
        log_F = log_Fcent / (1 + f1 * f1)
    return 10.0 ** log_F


def rate_coefficients(mech, T, C, params=None):
    """Forward rate coefficients k_j of every reaction, (R, n), and the
    third-body concentrations [M] of the class >= 1 reactions.

    ``params`` overrides the Arrhenius triples: rows 0..R-1 are the main
    (high-pressure for falloff) triples, rows R..R+n_fo-1 the low-pressure
    triples of the falloff reactions in order.
    """
    if params is None:
        params = mech.parameters()
    k = arrhenius(params[:mech.R], T)
    M = third_body_concentrations(mech, C)
    pd_row = {int(j): i for i, j in enumerate(mech.pd_reactions)}
    k = k.astype(np.result_type(k, M))
    for f, j in enumerate(mech.falloff_reactions):
        j = int(j)
        k_inf = k[j]
        k0 = arrhenius(params[mech.R + f][None, :], T)[0]
        Pr = k0 * M[pd_row[j]] / k_inf
        if mech.rtype[j] == 3:
            F = troe_factor(mech.troe[f], T, Pr)
        else:
            F = 1.0
        k[j] = k_inf * (Pr / (1 + Pr)) * F
    return k, M


def equilibrium_constants(mech, T):
    """K_j = (p0/(R T))^(Delta nu_j) exp(-sum_k nu_kj g0_k/(R T))
    (eq. equil_constants, eq. gibbs); (R, n)."""
    T = np.asarray(T)
    g = thermo.species_g_RT(mech, T)
    nu = mech.nu
    K = []
    for j in range(mech.R):
        dnu = nu[:, j].sum()
        s = 0.0
        for k in range(mech.S):
            if nu[k, j] != 0:
                s = s + nu[k, j] * g[k]
        K.append((ONE_ATM / (GAS_CONSTANT * T)) ** dnu * np.exp(-s))
    return np.array(K)


def _power_product(C, nu_col):
    """prod_k C_k^nu_k by repeated multiplication (integer nu >= 0)."""
    out = np.ones(C.shape[1], dtype=C.dtype)
    for k in np.nonzero(nu_col)[0]:
        for _ in range(int(nu_col[k])):
            out = out * C[k]
    return out


def rates_of_progress(mech, rho, T, Y, params=None):
    """Rates of progress of eq. reaction_rates.

    Returns ``(Rf, Rr, phi, q)``, each (R, n): the forward term
    k_j prod C^nu', the reverse term k_j/K_j prod C^nu'' (zero when
    irreversible), the third-body factor phi_j ([M]_j for class 1, else 1)
    and q_j = (Rf - Rr) phi.
    """
    T = np.asarray(T)
    C = concentrations(mech, rho, Y)
    k, M = rate_coefficients(mech, T, C, params)
    K = equilibrium_constants(mech, T)
    dt = np.result_type(C, k, K)
    Rf = np.zeros((mech.R, C.shape[1]), dtype=dt)
    Rr = np.zeros_like(Rf)
    phi = np.ones_like(Rf)
    pd_row = {int(j): i for i, j in enumerate(mech.pd_reactions)}
    for j in range(mech.R):
        Rf[j] = k[j] * _power_product(C, mech.nu_f[:, j])
        if mech.reversible[j]:
            Rr[j] = k[j] / K[j] * _power_product(C, mech.nu_r[:, j])
        if mech.rtype[j] == 1:
            phi[j] = M[pd_row[j]]
    q = (Rf - Rr) * phi
    return Rf, Rr, phi, q


def net_production_rates(mech, rho, T, Y, params=None):
    """omega_i = sum_j nu_ij q_j (eq. production_rates), mol m^-3 s^-1, (S, n)."""
    _, _, _, q = rates_of_progress(mech, rho, T, Y, params)
    nu = mech.nu
    w = np.zeros((mech.S, q.shape[1]), dtype=q.dtype)
    for i in range(mech.S):
        for j in range(mech.R):
            if nu[i, j] != 0:
                w[i] = w[i] + nu[i, j] * q[j]
    return w


def source_terms(mech, rho, T, Y, params=None):
    """Chemical source terms S_k = W_k omega_k (eq. massfrac_ode), kg m^-3 s^-1."""
    return mech.W[:, None] * net_production_rates(mech, rho, T, Y, params)
