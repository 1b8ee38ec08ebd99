"""Homogeneous adiabatic isochoric reactor: one time step of the mass
fraction ODE rho dY_k/dt = W_k omega_k (eq. massfrac_ode) at constant density
and internal energy, the temperature of every evaluation following from the
Newton inversion of the energy (eq. delta_temp).

Two steppers, as in the paper's reactor demonstrations:

* the classical fourth-order Runge-Kutta step (Sec. "Application: Simulations
  of Autoignition and Flame Propagation", explicit marching);
* the Crank-Nicolson step solved by Newton's method (Sec. "Time Integration &
  Spatial Discretization": eq. crank_nicol_rhs, eq. crank_nicol_newton_system,
  eq. crank_nicol_newton_update, eq. crank_nicol_jac, eq. chem_jacobian).

Readings: the printed Crank-Nicolson residual omits the density of
eq. massfrac_ode; here F = Y^{m+1} - Y^m - dt/(2 rho) (S^{m+1} + S^m) and its
Jacobian delta_jk - dt/(2 rho) J_jk, J = dS/dY at fixed density and energy.
The paper gives no Newton stopping rule for this system: iterate from
Y^{m+1}_0 = Y^m until the first update with max_k |Delta Y_k| <= tol
(1e-12; mass fractions are O(1)), at most ``max_iter`` (20) updates; the
count is returned per cell, negated if tol was not met.  The step size may
differ per cell (an array of n values).
"""

import numpy as np

from . import jacobian, kinetics, newton


def rhs(mech, rho, e, Y, T_guess):
    """dY/dt = S/rho with T from the energy; returns (dY/dt (S, n), T)."""
    T, status = newton.temperature(mech, e, Y, T_guess)
    if not np.all(status > 0):
        raise RuntimeError("temperature inversion did not converge")
    return kinetics.source_terms(mech, rho, T, Y) / rho, T


def rk4_step(mech, rho, e, Y, T, dt):
    """One classical Runge-Kutta step; returns (Y_new, T of Y_new)."""
    k1, T1 = rhs(mech, rho, e, Y, T)
    k2, T2 = rhs(mech, rho, e, Y + 0.5 * dt * k1, T1)
    k3, T3 = rhs(mech, rho, e, Y + 0.5 * dt * k2, T2)
    k4, T4 = rhs(mech, rho, e, Y + dt * k3, T3)
    Yn = Y + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    Tn, status = newton.temperature(mech, e, Yn, T4)
    return Yn, Tn


def cn_step(mech, rho, e, Y, T, dt, tol=1e-12, max_iter=20):
    """One Crank-Nicolson step by Newton's method; returns (Y_new, T_new,
    status).  Cells are independent: each solves its own S x S system."""
    S, n = Y.shape
    dt = np.broadcast_to(np.asarray(dt, dtype=float), (n,))
    f0, T0 = rhs(mech, rho, e, Y, T)
    Yk = Y.copy()
    Tk = T0.copy()
    status = np.full(n, -max_iter, dtype=np.int32)
    active = np.ones(n, dtype=bool)
    for it in range(max_iter):
        if not active.any():
            break
        idx = np.nonzero(active)[0]
        Ya, ra, ea, ha = Yk[:, idx], rho[idx], e[idx], dt[idx]
        fa, Ta = rhs(mech, ra, ea, Ya, Tk[idx])
        F = Ya - Y[:, idx] - 0.5 * ha * (fa + f0[:, idx])
        J = jacobian.jacobian(mech, ra, Ta, Ya)            # dS/dY, fixed rho and e
        for c in range(len(idx)):
            A = np.eye(S) - (0.5 * ha[c] / ra[c]) * J[:, :, c]
            dY = np.linalg.solve(A, -F[:, c])
            Ya[:, c] = Ya[:, c] + dY
            if np.max(np.abs(dY)) <= tol:
                status[idx[c]] = it + 1
                active[idx[c]] = False
        Yk[:, idx] = Ya
        Tk[idx] = Ta
    Tn, st = newton.temperature(mech, e, Yk, Tk)
    return Yk, Tn, status
