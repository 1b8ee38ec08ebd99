"""MI355X-native per-cell thermochemistry (arXiv:2503.24286, Appendix A).

Python binding of libpyro.so: every computation runs in the library's HIP
kernels; this package only marshals torch tensors into the C ABI of
include/pyro.h.
"""

from ._lib import PyroError  # noqa: F401
from .api import (Mechanism, ProductionRates, density, internal_energy,  # noqa: F401
                  pressure, production_rates, production_rates_autograd,
                  production_rates_vjp, temperature)
