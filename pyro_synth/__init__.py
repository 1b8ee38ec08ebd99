"""Seeded synthetic inputs shared by the tests, the benchmark and the mechanism
builder.

This package only draws random numbers and arranges them into mechanisms and
cell states.  It holds none of the thermochemistry arithmetic (no NASA
polynomial, rate, equilibrium or equation-of-state evaluation): quantities that
need that arithmetic (thermo integration constants, the equilibrium-constant
guard, densities, internal energies) are computed by whoever consumes the
draws.
"""

from .configs import CONFIGS, SEEDS, mechanism_config  # noqa: F401
