"""Parity metrics between the GPU library and the oracle.

omega_k and q_j are differences of large terms, so a componentwise relative
error is ill conditioned.  Two measures are used, per cell:

* scaled: max_k |w_gpu - w_ref| / (sum_j |nu_kj| (|Rf_j| + |Rr_j|) phi_j),
  the error relative to the magnitudes that are summed (condition free);
* normwise: ||w_gpu - w_ref||_2 / ||w_ref||_2 (the paper's eq. verif_errors
  with p = 2 over the species axis), asserted for cells whose condition
  number kappa = || |nu| (|Rf| + |Rr|) phi ||_2 / ||w_ref||_2 is <= 1e3.
"""

import numpy as np

from oracle import kinetics, thermo
from oracle.constants import GAS_CONSTANT as RU

TOL_F64 = 1e-12
KAPPA_MAX = 1e3


def wdot_metrics(m, rho, T, Y, w_gpu, params=None):
    Rf, Rr, phi, q = kinetics.rates_of_progress(m, rho, T, Y, params)
    w_ref = kinetics.net_production_rates(m, rho, T, Y, params)
    mag = np.abs(m.nu) @ ((np.abs(Rf) + np.abs(Rr)) * np.abs(phi))
    diff = np.abs(w_gpu - w_ref)
    with np.errstate(invalid="ignore", divide="ignore"):
        scaled = np.where(mag > 0, diff / np.where(mag > 0, mag, 1.0), diff)
    scaled = scaled.max(axis=0)
    nref = np.linalg.norm(w_ref, axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        normwise = np.linalg.norm(w_gpu - w_ref, axis=0) / nref
        kappa = np.linalg.norm(mag, axis=0) / nref
    return dict(scaled=scaled, normwise=normwise, kappa=kappa, w_ref=w_ref)


def assert_wdot_parity(m, rho, T, Y, w_gpu, tol=TOL_F64, params=None):
    r = wdot_metrics(m, rho, T, Y, w_gpu, params)
    assert np.all(np.isfinite(w_gpu)), "non-finite GPU result"
    worst = int(np.argmax(r["scaled"]))
    assert r["scaled"].max() <= tol, (
        f"scaled error {r['scaled'].max():.3e} at cell {worst}")
    well = r["kappa"] <= KAPPA_MAX
    if well.any():
        assert r["normwise"][well].max() <= tol, (
            f"normwise error {r['normwise'][well].max():.3e}")
    return r


def vjp_scales(m, rho, T, Y, wbar, abs_qbar=False):
    """Magnitudes of the terms summed into each gradient (no cancellation):
    the reference the errors are measured against.  With ``abs_qbar`` the
    cotangent of each rate of progress is taken as |nu|^T |wbar|, the size of
    the terms that cancel in nu^T wbar."""
    Rf, Rr, phi, q = kinetics.rates_of_progress(m, rho, T, Y)
    qbar = np.abs(m.nu).T @ np.abs(wbar) if abs_qbar else m.nu.T @ wbar
    Dbar = np.abs(qbar * phi)
    a = Dbar * np.abs(Rf)
    b = Dbar * np.abs(Rr)
    ab = a + b
    pos = Y > 0
    sY = (m.nu_f @ a + m.nu_r @ b) / np.where(pos, Y, 1.0)
    M = np.zeros_like(Rf)
    pd = m.pd_reactions
    if len(pd):
        M[pd] = np.abs(qbar[pd]) * (np.abs(Rf[pd]) + np.abs(Rr[pd]))
        eps = np.zeros((m.S, m.R))
        eps[:, pd] = m.efficiency.T
        sY = sY + (rho / m.W[:, None]) * (eps @ M)
    sY = np.where(pos, sY, 0.0)     # dL/dY_k = 0 exactly where Y_k <= 0
    h = np.abs(thermo.species_h_RT(m, T)).max(axis=0)
    coef = (np.abs(m.arrhenius[:, 1])[:, None] + m.arrhenius[:, 2][:, None] / (RU * T)
            + np.abs(m.nu.sum(axis=0))[:, None] + 2.0 + 2.0 * h[None, :])
    sT = (ab * coef).sum(axis=0) / T
    sP = np.zeros((m.R + m.n_falloff, 3))
    sP[:m.R, 0] = ab.sum(axis=1)
    sP[:m.R, 1] = (ab * np.abs(np.log(T))).sum(axis=1)
    sP[:m.R, 2] = (ab / (RU * T)).sum(axis=1)
    for f, j in enumerate(m.falloff_reactions):
        sP[m.R + f] = sP[j]
    return sY, sT, sP
