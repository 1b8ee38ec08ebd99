"""Mixture-averaged transport properties (appendix "Extensions to Flow &
Transport": eq. mixavg_viscosity, eq. mixavg_conductivity,
eq. diff_mix_rule and the species polynomial fits), evaluated per cell in the
paper's notation.

Readings: "log T" is the natural logarithm; the binary diffusivities are the
printed polynomial sqrt(T) sum_m a_ijm (log T)^m with no pressure factor; the
mixture rule uses X_k = W Y_k/W_k with W = (sum_k Y_k/W_k)^-1 from the
mass fractions as given (the sum is not renormalised); a pure species has a
zero numerator and an infinite sum in eq. diff_mix_rule, which is left to
IEEE arithmetic (NaN).
"""

import numpy as np

from . import eos


def _poly(coef, L):
    """sum_{m=0..4} coef[..., m] L^m for each row of coef, (rows, n)."""
    out = np.zeros(coef.shape[:-1] + L.shape)
    for m in range(coef.shape[-1]):
        out = out + coef[..., m, None] * L ** m
    return out


def species_viscosities(visc, T):
    """mu_i = sqrt(T) (sum_m b_im (log T)^m)^2, (S, n)."""
    T = np.asarray(T, dtype=float)
    return np.sqrt(T) * _poly(visc, np.log(T)) ** 2


def species_conductivities(cond, T):
    """kappa_i = sqrt(T) sum_m c_im (log T)^m (eq. species_cond), (S, n)."""
    T = np.asarray(T, dtype=float)
    return np.sqrt(T) * _poly(cond, np.log(T))


def binary_diffusivities(diff, T):
    """D_ij = sqrt(T) sum_m a_ijm (log T)^m, (S, S, n)."""
    T = np.asarray(T, dtype=float)
    return np.sqrt(T) * _poly(diff, np.log(T))


def mole_fractions(mech, Y):
    """X_k = W Y_k/W_k (W the mixture molar mass), (S, n)."""
    return eos.mixture_molar_mass(mech, Y) * Y / mech.W[:, None]


def mixture_viscosity(mech, visc, T, Y):
    """mu = sum_k X_k mu_k / sum_j Phi_kj X_j with
    Phi_kj = (1 + sqrt((mu_k/mu_j) sqrt(W_j/W_k)))^2 / sqrt(8 (1 + W_k/W_j))."""
    mu = species_viscosities(visc, T)
    X = mole_fractions(mech, Y)
    W = mech.W
    S = mech.S
    total = np.zeros(X.shape[1])
    for k in range(S):
        den = np.zeros(X.shape[1])
        for j in range(S):
            phi = ((1.0 + np.sqrt((mu[k] / mu[j]) * np.sqrt(W[j] / W[k]))) ** 2
                   / np.sqrt(8.0 * (1.0 + W[k] / W[j])))
            den = den + phi * X[j]
        total = total + X[k] * mu[k] / den
    return total


def mixture_conductivity(mech, cond, T, Y):
    """kappa = (sum_k X_k kappa_k + (sum_k X_k/kappa_k)^-1)/2."""
    kap = species_conductivities(cond, T)
    X = mole_fractions(mech, Y)
    a = np.zeros(X.shape[1])
    b = np.zeros(X.shape[1])
    for k in range(mech.S):
        a = a + X[k] * kap[k]
        b = b + X[k] / kap[k]
    return 0.5 * (a + 1.0 / b)


def mixture_diffusivities(mech, diff, T, Y):
    """D_k,m = (W - X_k W_k)/W (sum_{j != k} X_j/D_kj)^-1, (S, n)."""
    D = binary_diffusivities(diff, T)
    X = mole_fractions(mech, Y)
    Wmix = eos.mixture_molar_mass(mech, Y)
    out = np.zeros_like(X)
    with np.errstate(divide="ignore", invalid="ignore"):
        for k in range(mech.S):
            s = np.zeros(X.shape[1])
            for j in range(mech.S):
                if j != k:
                    s = s + X[j] / D[k, j]
            out[k] = (Wmix - X[k] * mech.W[k]) / Wmix / s
    return out
