"""Chemical Jacobian J = dS/dY of the source terms S_k = W_k omega_k
(eq. jacobian and eq. chem_jacobian, Sec. "Automatic Differentiation Enables
Implicit Time Marching"), by the complex step.

Reading: the paper differentiates the function Y -> W * omega(rho, T, Y) in
which T comes from the Newton inversion of the internal energy at the given
(fixed) density and energy.  Here that function is evaluated with complex
mass fractions: the Newton iteration of eq. delta_temp runs in complex
arithmetic from the real guess until the real and imaginary parts of the
update have both converged, and column k of J is Im S(Y + i h e_k)/h with
h = 1e-30 (exact to rounding).  ``fixed="temperature"`` gives the partial
derivative at fixed T instead (no Newton solve).

Cells lie on the last axis; J has shape (S, S, n) with J[j, k] = dS_j/dY_k.
A mass fraction Y_k <= 0 enters the concentrations as zero, so its column has
no concentration part (only the temperature part at fixed energy).
"""

import numpy as np

from . import kinetics, thermo

STEP = 1e-30


def source_terms(mech, rho, T, Y, params=None):
    """S_k = W_k omega_k (eq. massfrac_ode's chemical source), (S, n)."""
    return kinetics.source_terms(mech, rho, T, Y, params)


def temperature_complex(mech, e, Y, T_guess, rtol=1e-12, max_iter=100):
    """The Newton iteration T <- T - (Y.e(T) - e)/c_v(T) in complex
    arithmetic (complex Y); stops once |Re dT| <= rtol |Re T| and
    |Im dT| <= rtol |Im T| + 1e-300 hold for every cell."""
    n = Y.shape[1]
    T = np.broadcast_to(np.asarray(T_guess, dtype=complex), (n,)).copy()
    for _ in range(max_iter):
        resid = thermo.mixture_internal_energy(mech, T, Y) - e
        dT = -resid / thermo.mixture_cv(mech, T, Y)
        T = T + dT
        if (np.all(np.abs(dT.real) <= rtol * np.abs(T.real))
                and np.all(np.abs(dT.imag) <= rtol * np.abs(T.imag) + 1e-300)):
            return T
    raise RuntimeError("complex Newton iteration did not converge")


def jacobian(mech, rho, T, Y, fixed="energy", params=None):
    """J[j, k, cell] = dS_j/dY_k at fixed density and, by default, fixed
    internal energy e = e(T, Y) (T the converged temperature of the state)."""
    if fixed not in ("energy", "temperature"):
        raise ValueError("fixed must be 'energy' or 'temperature'")
    T = np.asarray(T, dtype=float)
    S, n = Y.shape
    e = thermo.mixture_internal_energy(mech, T, Y)
    J = np.zeros((S, S, n))
    for k in range(S):
        Yc = Y.astype(complex)
        Yc[k] += 1j * STEP
        Tc = temperature_complex(mech, e, Yc, T) if fixed == "energy" else T
        J[:, k, :] = source_terms(mech, rho, Tc, Yc, params).imag / STEP
    return J
