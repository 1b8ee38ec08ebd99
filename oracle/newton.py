"""Newton inversion of the temperature from the internal energy (Sec. A.3.1,
eq. int_energy, eq. delta_temp, eq. cv).

Readings: the paper stops on a "data-dependent tolerance" and mentions
limiting the iteration count without numbers; here each cell iterates
T_{m+1} = T_m - (Y.e(T_m) - e)/c_v(T_m) until the first update with
|Delta T| <= rtol |T_{m+1}| (rtol = 1e-12) or ``max_iter`` updates (50), with
no damping or clamping.  ``status`` holds the number of updates taken, negated
when the tolerance was not met.
"""

import numpy as np

from . import thermo


def temperature_from_enthalpy(mech, h, Y, T_guess, rtol=1e-12, max_iter=50):
    """The same iteration on the enthalpy: T <- T - (Y.h(T) - h)/c_p(T) (the
    enthalpy variant the paper names at the end of Sec. A.3.1)."""
    return _newton(mech, h, Y, T_guess, rtol, max_iter, thermo.mixture_enthalpy,
                   thermo.mixture_cp)


def temperature(mech, e, Y, T_guess, rtol=1e-12, max_iter=50):
    return _newton(mech, e, Y, T_guess, rtol, max_iter, thermo.mixture_internal_energy,
                   thermo.mixture_cv)


def _newton(mech, e, Y, T_guess, rtol, max_iter, value, slope):
    e = np.asarray(e, dtype=float)
    n = e.shape[0]
    T = np.broadcast_to(np.asarray(T_guess, dtype=float), (n,)).copy()
    status = np.full(n, -max_iter, dtype=np.int32)
    active = np.ones(n, dtype=bool)
    for m in range(max_iter):
        if not active.any():
            break
        idx = np.nonzero(active)[0]
        Ti = T[idx]
        Yi = Y[:, idx]
        resid = value(mech, Ti, Yi) - e[idx]
        dT = -resid / slope(mech, Ti, Yi)
        Tn = Ti + dT
        T[idx] = Tn
        done = np.abs(dT) <= rtol * np.abs(Tn)
        status[idx[done]] = m + 1
        active[idx[done]] = False
    return T, status
