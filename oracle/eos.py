"""Ideal-gas equation of state (Sec. A.1, eq. eos)."""

import numpy as np

from .constants import GAS_CONSTANT


def mixture_molar_mass(mech, Y):
    """W = (sum_i Y_i/W_i)^-1 in kg/mol, summed in species order."""
    acc = np.zeros(Y.shape[1:], dtype=Y.dtype)
    for i in range(mech.S):
        acc = acc + Y[i] / mech.W[i]
    return 1.0 / acc


def pressure(mech, rho, T, Y):
    """p = rho R T / W (eq. eos)."""
    return rho * GAS_CONSTANT * T / mixture_molar_mass(mech, Y)


def density(mech, p, T, Y):
    """rho = p W / (R T), eq. eos solved for the density."""
    return p * mixture_molar_mass(mech, Y) / (GAS_CONSTANT * T)
