"""CPU FP64 oracle of the ideal-gas kinetics and thermodynamics formulation.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference the GPU library is checked against.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
path never does, and it shares no code, tables or constants generator with the
HIP library.

It follows Appendix A of the paper (Sec. A.1 governing equations, Sec. A.3.1
temperature inversion) step by step and in the paper's notation: molar
concentrations (eq. concentrations), NASA7 thermodynamics (eq. nasa_poly,
eq. nasa_poly_c, eq. gibbs), Arrhenius rate coefficients (eq. rate_coeff),
equilibrium constants (eq. equil_constants), rates of progress
(eq. reaction_rates), net production rates (eq. production_rates), the
equation of state (eq. eos) and the Newton inversion of T from the internal
energy (eq. int_energy, eq. delta_temp, eq. cv).  Cells lie on the last array
axis, as in the paper's NumPy execution of its generated code (Sec. 4.1);
arithmetic is FP64, or complex128 when a caller perturbs an input along the
imaginary axis for complex-step derivatives.

Readings of passages the paper leaves garbled or silent are listed in the
docstrings of the functions that take them.  Every function is pinned by the
"not gpu" tests (closed forms, invariants, quadrature, complex step vs. finite
differences, detailed balance, conservation, hand-evaluated third-body and Troe
values with distinct efficiencies and a finite reduced pressure).  What no pin
can fix is the agreement of the third-body and Troe conventions with other
kinetics packages: the paper names these forms without writing them.
"""

from . import eos, kinetics, mechfile, newton, thermo, gradients, jacobian, primitive  # noqa: F401
from .constants import GAS_CONSTANT, ONE_ATM  # noqa: F401
