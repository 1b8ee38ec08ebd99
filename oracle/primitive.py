"""Primitive from conserved variables: the per-cell equation-of-state routine
of the paper's flame solver (Sec. "Python Code Generation and Immediate
Execution using NumPy"), in its order: density as the sum of the partial
densities, mass fractions, velocity, internal energy as total energy per
mass minus the kinetic part, temperature by the Newton inversion
(eq. delta_temp), pressure by the equation of state (eq. eos).
"""

import numpy as np

from . import eos, newton


def primitive_from_conserved(mech, densities, momentum, total_energy, T_guess,
                             rtol=1e-12, max_iter=50):
    """densities (S, n), momentum (dim, n), total_energy (n,) ->
    (density, mass_fractions, velocity, temperature, pressure, status)."""
    density = np.zeros(densities.shape[1])
    for k in range(densities.shape[0]):
        density = density + densities[k]
    mass_fractions = densities / density
    velocity = momentum / density
    kinetic = np.zeros_like(density)
    for d in range(velocity.shape[0]):
        kinetic = kinetic + velocity[d] ** 2
    energy = total_energy / density - 0.5 * kinetic
    temperature, status = newton.temperature(mech, energy, mass_fractions, T_guess, rtol, max_iter)
    pressure = eos.pressure(mech, density, temperature, mass_fractions)
    return density, mass_fractions, velocity, temperature, pressure, status
