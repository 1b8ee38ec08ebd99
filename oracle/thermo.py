"""Species thermodynamics from two-range NASA7 polynomials (Sec. A.1,
eq. nasa_poly, eq. nasa_poly_c, eq. gibbs) and the mixture internal energy
(Sec. A.3.1, eq. int_energy, eq. cv).

Readings (the printed formulas are garbled):

* cp: the printed sum runs to m = 4 with a factor m/m; the standard NASA7 form
  cp/R = sum_{m=1..5} a_m T^(m-1) is taken, pinned by dh/dT = cp.
* entropy: the printed form puts the log on alpha_h and T^m on the higher
  terms; the standard form s/R = a1 ln T + sum_{m=2..5} a_m T^(m-1)/(m-1) + a7
  is taken (alpha_h = a6, alpha_s = a7), pinned by ds/dT = cp/T.
* range: coefficient set "low" when T <= T_mid of the species, else "high";
  no clamping outside [T_low, T_high].
* units: J/mol throughout (the paper mixes J/mol and J/kmol); the internal
  energy and c_v are per unit mass, e_k = (h_k - R T)/W_k with W_k in kg/mol.
* mass-specific c_v: the printed "c_v = c_p - R" is read on the mass basis,
  c_v = sum_k Y_k (cp_k - R)/W_k.
"""

import numpy as np

from .constants import GAS_CONSTANT


def _col(a, m):
    """Coefficient a_m (1-based) of every species as a column (S, 1)."""
    return a[:, m - 1][:, None]


def cp_R_poly(a, T):
    """cp/R = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4 for coefficient rows
    ``a`` (S, 7) at temperatures ``T`` (n,); returns (S, n)."""
    return (_col(a, 1) + _col(a, 2) * T + _col(a, 3) * T**2
            + _col(a, 4) * T**3 + _col(a, 5) * T**4)


def h_RT_poly(a, T):
    """h/(RT) = a1 + a2 T/2 + a3 T^2/3 + a4 T^3/4 + a5 T^4/5 + a6/T."""
    return (_col(a, 1) + _col(a, 2) * T / 2 + _col(a, 3) * T**2 / 3
            + _col(a, 4) * T**3 / 4 + _col(a, 5) * T**4 / 5 + _col(a, 6) / T)


def s_R_poly(a, T):
    """s/R = a1 ln T + a2 T + a3 T^2/2 + a4 T^3/3 + a5 T^4/4 + a7."""
    return (_col(a, 1) * np.log(T) + _col(a, 2) * T + _col(a, 3) * T**2 / 2
            + _col(a, 4) * T**3 / 3 + _col(a, 5) * T**4 / 4 + _col(a, 7))


def _by_range(mech, poly, T):
    T = np.asarray(T)
    low = poly(mech.nasa_low, T)
    high = poly(mech.nasa_high, T)
    use_low = np.real(T)[None, :] <= mech.T_mid[:, None]
    return np.where(use_low, low, high)


def species_cp_R(mech, T):
    """cp_k/R of every species, (S, n)."""
    return _by_range(mech, cp_R_poly, T)


def species_h_RT(mech, T):
    """h_k/(R T), (S, n)."""
    return _by_range(mech, h_RT_poly, T)


def species_s_R(mech, T):
    """s0_k/R, (S, n)."""
    return _by_range(mech, s_R_poly, T)


def species_g_RT(mech, T):
    """Standard Gibbs function g0_k/(R T) = h_k/(R T) - s0_k/R (eq. gibbs)."""
    return species_h_RT(mech, T) - species_s_R(mech, T)


def species_internal_energy(mech, T):
    """e_k = (h_k - R T)/W_k in J/kg (Sec. A.3.1), (S, n)."""
    T = np.asarray(T)
    h = species_h_RT(mech, T) * GAS_CONSTANT * T
    return (h - GAS_CONSTANT * T) / mech.W[:, None]


def species_cv(mech, T):
    """c_v,k = (cp_k - R)/W_k in J/(kg K), the T-derivative of e_k."""
    cp = species_cp_R(mech, T) * GAS_CONSTANT
    return (cp - GAS_CONSTANT) / mech.W[:, None]


def mixture_internal_energy(mech, T, Y):
    """e = Y . e(T) (eq. int_energy), summed over species in index order."""
    ek = species_internal_energy(mech, T)
    total = np.zeros(np.broadcast(np.asarray(T), Y[0]).shape, dtype=np.result_type(ek, Y))
    for k in range(mech.S):
        total = total + Y[k] * ek[k]
    return total


def mixture_cv(mech, T, Y):
    """c_v = sum_k Y_k c_v,k (eq. cv on the mass basis)."""
    cvk = species_cv(mech, T)
    total = np.zeros(np.broadcast(np.asarray(T), Y[0]).shape, dtype=np.result_type(cvk, Y))
    for k in range(mech.S):
        total = total + Y[k] * cvk[k]
    return total


def species_enthalpy(mech, T):
    """h_k/W_k in J/kg (eq. nasa_poly), (S, n)."""
    T = np.asarray(T)
    return species_h_RT(mech, T) * GAS_CONSTANT * T / mech.W[:, None]


def mixture_enthalpy(mech, T, Y):
    """h = sum_k Y_k h_k/W_k, summed in species order."""
    hk = species_enthalpy(mech, T)
    total = np.zeros(np.broadcast(np.asarray(T), Y[0]).shape, dtype=np.result_type(hk, Y))
    for k in range(mech.S):
        total = total + Y[k] * hk[k]
    return total


def mixture_cp(mech, T, Y):
    """c_p = sum_k Y_k cp_k/W_k = dh/dT (mass basis)."""
    cpk = species_cp_R(mech, T) * GAS_CONSTANT / mech.W[:, None]
    total = np.zeros(np.broadcast(np.asarray(T), Y[0]).shape, dtype=np.result_type(cpk, Y))
    for k in range(mech.S):
        total = total + Y[k] * cpk[k]
    return total
