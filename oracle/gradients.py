"""Reverse-mode products of the net production rates, by the complex step.

L = sum over cells and species of wbar_k(cell) * omega_k(cell), at fixed
density (omega is a function of rho, T and Y; eq. production_rates).  The
gradient with respect to an input x is Im(L(x + i h))/h with h = 1e-30, exact
to rounding because no difference of nearby values is formed.

* dL/dY_k and dL/dT are per cell (cells are independent): one complex pass per
  species with Y_k of every cell perturbed, and one pass with T perturbed.
* The parameters enter reaction by reaction: q_j depends only on its own
  triples (ln A, b, Ea), and for a falloff reaction also on its low-pressure
  triple.  With qbar_j = sum_k nu_kj wbar_k, dL/dp = sum_cells qbar_j dq_j/dp.
  One pass with a parameter column of every reaction perturbed at once yields
  dq_j/dp_j for all j together; main and low-pressure triples get separate
  passes because a falloff q_j depends on both.

Gradients with respect to Ea are per J/mol.  Troe shape parameters and
third-body efficiencies get no gradient.  A cell with Y_k <= 0 has
dL/dY_k = 0 (C_k = rho max(Y_k, 0)/W_k).
"""

import numpy as np

from . import kinetics

STEP = 1e-30


def vjp(mech, rho, T, Y, wbar, params=None):
    """Returns ``(Ybar (S, n), Tbar (n,), pbar (R + n_fo, 3))``."""
    if params is None:
        params = mech.parameters()
    params = np.asarray(params, dtype=float)
    T = np.asarray(T, dtype=float)
    S, n = Y.shape

    def cell_L(Tc, Yc, P):
        w = kinetics.net_production_rates(mech, rho, Tc, Yc, P)
        return (wbar * w).sum(axis=0)

    Ybar = np.zeros((S, n))
    for k in range(S):
        Yc = Y.astype(complex)
        Yc[k] += 1j * STEP
        Ybar[k] = cell_L(T, Yc, params).imag / STEP
    Tbar = cell_L(T + 1j * STEP, Y, params).imag / STEP

    qbar = mech.nu.T @ wbar                   # (R, n)
    R = mech.R
    pbar = np.zeros_like(params)
    for c in range(3):
        P = params.astype(complex)
        P[:R, c] += 1j * STEP
        _, _, _, q = kinetics.rates_of_progress(mech, rho, T, Y, P)
        dq = q.imag / STEP
        pbar[:R, c] = (qbar * dq).sum(axis=1)
        if mech.n_falloff:
            P = params.astype(complex)
            P[R:, c] += 1j * STEP
            _, _, _, q = kinetics.rates_of_progress(mech, rho, T, Y, P)
            dq = q.imag / STEP
            for f, j in enumerate(mech.falloff_reactions):
                pbar[R + f, c] = (qbar[j] * dq[j]).sum()
    return Ybar, Tbar, pbar
