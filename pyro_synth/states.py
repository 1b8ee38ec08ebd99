"""Seeded cell states.

Cells are drawn in chunks of ``CHUNK`` consecutive cells, chunk ``c`` from
``default_rng([seed, c])``, so any range of cells can be regenerated without
drawing the ones before it.  Arrays are structure-of-arrays and
species-major: ``Y[k, i]``.
"""

import numpy as np

from .configs import CONFIGS, SEEDS

CHUNK = 1 << 16


def _chunk_rng(seed, c):
    return np.random.default_rng([seed, c])


def draw_states(cfg, n, S, seed=None, first=0):
    """Temperature (K), pressure (Pa) and mass fractions for cells
    ``first .. first+n-1`` of workload ``cfg``.

    T ~ U[T_range]; p is fixed or log10 p ~ U[log10p_range]; Y ~ Dirichlet
    with the configured concentration, drawn as normalised Gamma variates.
    Returns ``(T, p, Y)`` with shapes ``(n,)``, ``(n,)``, ``(S, n)``.
    """
    c = CONFIGS[cfg]
    if seed is None:
        seed = SEEDS["states"] + cfg
    T = np.empty(n)
    p = np.empty(n)
    Y = np.empty((S, n))
    end = first + n
    c0 = first // CHUNK
    c1 = (end + CHUNK - 1) // CHUNK
    for ch in range(c0, c1):
        lo = ch * CHUNK
        rng = _chunk_rng(seed, ch)
        Tc = rng.uniform(*c["T_range"], size=CHUNK)
        if c["p_fixed"] is not None:
            pc = np.full(CHUNK, c["p_fixed"])
        else:
            pc = 10.0 ** rng.uniform(*c["log10p_range"], size=CHUNK)
        G = rng.standard_gamma(c["dirichlet_alpha"], size=(S, CHUNK))
        Yc = G / G.sum(axis=0)
        a, b = max(first, lo), min(end, lo + CHUNK)
        T[a - first:b - first] = Tc[a - lo:b - lo]
        p[a - first:b - first] = pc[a - lo:b - lo]
        Y[:, a - first:b - first] = Yc[:, a - lo:b - lo]
    return T, p, Y


def draw_guess_factors(cfg, n, seed=None):
    """Multipliers U[0.7, 1.3] for a per-cell Newton initial guess T*f."""
    if seed is None:
        seed = SEEDS["states"] + 100 + cfg
    return np.random.default_rng(seed).uniform(0.7, 1.3, size=n)


def draw_cotangent(cfg, n, S, seed=None):
    """w ~ N(0, 1) of shape (S, n): the weights of L = sum w_k wdot_k."""
    if seed is None:
        seed = SEEDS["vjp_weights"] + cfg
    return np.random.default_rng(seed).standard_normal((S, n))
