"""MI355X-native per-cell thermochemistry (arXiv:2503.24286, Appendix A).

Python binding of libpyro.so: every computation runs in the library's HIP
kernels; this package only marshals torch tensors into the C ABI of
include/pyro.h.
"""

from ._lib import PyroError  # noqa: F401
from .api import (Mechanism, ProductionRates, Transport, chemical_jacobian,  # noqa: F401
                  density, internal_energy, mixture_transport, pressure,
                  primitive_from_conserved, production_rates, reactor_step,
                  production_rates_autograd, production_rates_vjp, temperature,
                  temperature_from_enthalpy)
