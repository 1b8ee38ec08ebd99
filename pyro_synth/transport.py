"""Seeded synthetic transport fits: coefficients of the species viscosity,
conductivity and binary-diffusivity polynomials in ln T (the mixture-averaged
transport model of the paper's "Extensions to Flow & Transport" appendix).

Each fit is drawn as a smooth, positive polynomial around T0 = 1000 K,
p(L) = beta (1 + sum_{m=1..4} e_m ((L - L0)/2)^m) with |e_m| <= 0.3/m,
L = ln T, L0 = ln T0, then written in the monomial basis sum_m c_m L^m the
model uses.  The levels match gases at 1000 K: viscosity 1e-5..6e-5 Pa s
(through its square root, the model squares the polynomial), conductivity
0.02..0.3 W/(m K), binary diffusivity 1e-5..3e-4 m^2/s (symmetric in the
pair), each divided by sqrt(T0) as the model multiplies by sqrt(T).
"""

import numpy as np

T0 = 1000.0
SEED = 5000


def _fits(rng, levels):
    """Monomial coefficients (..., 5) of positive quartics in L = ln T."""
    L0 = np.log(T0)
    shift = np.polynomial.Polynomial([-L0 / 2.0, 0.5])          # (L - L0)/2
    out = np.empty(levels.shape + (5,))
    e = rng.uniform(-1.0, 1.0, levels.shape + (4,)) * (0.3 / np.arange(1, 5))
    for idx in np.ndindex(levels.shape):
        p = np.polynomial.Polynomial([1.0])
        for m in range(4):
            p = p + e[idx + (m,)] * shift ** (m + 1)
        out[idx] = levels[idx] * p.coef
    return out


def draw_transport(S, seed=SEED):
    """Returns (viscosity (S, 5), conductivity (S, 5), diffusivity (S, S, 5))."""
    rng = np.random.default_rng(seed)
    mu = np.exp(rng.uniform(np.log(1e-5), np.log(6e-5), S))
    kappa = np.exp(rng.uniform(np.log(0.02), np.log(0.3), S))
    D = np.exp(rng.uniform(np.log(1e-5), np.log(3e-4), (S, S)))
    D = np.triu(D) + np.triu(D, 1).T
    sq = np.sqrt(T0)
    visc = _fits(rng, np.sqrt(mu / sq))
    cond = _fits(rng, kappa / sq)
    diff = _fits(rng, D / sq)
    iu = np.triu_indices(S, 1)
    diff[iu[1], iu[0]] = diff[iu[0], iu[1]]
    return visc, cond, diff
