"""Physical constants of the oracle (SI, mole basis)."""

# universal gas constant, J mol^-1 K^-1 (CODATA 2018, exact)
GAS_CONSTANT = 8.314462618
# reference pressure p0 of the equilibrium constants, 1 atm (eq. equil_constants)
ONE_ATM = 101325.0
