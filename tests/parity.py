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

from oracle import kinetics

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
