"""Random draws that make up a synthetic reaction mechanism.

Every function takes a ``numpy.random.Generator`` and returns plain arrays; the
order of the calls fixes the stream, so a mechanism is a pure function of its
seed.  Reactions are atom balanced by construction: candidate product sets are
looked up among the multisets of species whose summed element vector equals
that of the reactants.
"""

import itertools
from collections import defaultdict

import numpy as np

from .configs import ATOMIC_WEIGHTS

SIDE_SIZE_P = (0.25, 0.60, 0.15)   # probability of 1, 2, 3 molecules per side
T_LOW, T_MID, T_HIGH = 200.0, 1000.0, 3500.0


def draw_species(rng, cfg):
    """Element compositions of the species.

    Returns ``(elements, comp, reactive)``: ``comp[e, k]`` is the number of
    atoms of element ``e`` in species ``k``; ``reactive`` lists the species
    that may take part in reactions (all but the inert argon).
    """
    elements = list(cfg["elements"])
    E = len(elements)
    S = cfg["n_species"]
    fixed = []
    n2 = [0] * E
    n2[elements.index("N")] = 2
    fixed.append(tuple(n2))
    inert = None
    if cfg["inert_argon"]:
        ar = [0] * E
        ar[elements.index("Ar")] = 1
        inert = tuple(ar)
    # every composition inside the per-element bounds, in a fixed order
    bounded = [e for e in elements if e != "Ar"]
    ranges = [range(cfg["bounds"][e][0], cfg["bounds"][e][1] + 1) for e in bounded]
    pool = []
    for counts in itertools.product(*ranges):
        total = sum(counts)
        if not 1 <= total <= cfg["max_atoms"]:
            continue
        vec = [0] * E
        for e, c in zip(bounded, counts):
            vec[elements.index(e)] = c
        vec = tuple(vec)
        if vec not in fixed:
            pool.append(vec)
    n_random = S - len(fixed) - (1 if inert is not None else 0)
    if n_random > len(pool):
        raise ValueError("not enough distinct compositions")
    pick = rng.permutation(len(pool))[:n_random]
    comps = fixed + [pool[i] for i in sorted(pick)]
    if inert is not None:
        comps.append(inert)
    comp = np.array(comps, dtype=np.int32).T.copy()          # (E, S)
    reactive = np.arange(S - (1 if inert is not None else 0))
    return elements, comp, reactive


def molecular_weights(elements, comp):
    """W_k from the atom counts and standard atomic weights (kg/mol)."""
    aw = np.array([ATOMIC_WEIGHTS[e] for e in elements])
    return aw @ comp, aw


def species_names(elements, comp):
    names = []
    for k in range(comp.shape[1]):
        parts = []
        for e, c in zip(elements, comp[:, k]):
            if c:
                parts.append(e + (str(c) if c > 1 else ""))
        names.append("".join(parts))
    return names


def draw_thermo(rng, S):
    """Raw draws behind the two-range NASA7 fits.

    ``a1_lo`` ~ U[2.5, 5]; the higher coefficients of each range are
    ``u (1e-3/3.5)^(m-1) / 8`` with ``u`` ~ U[-1, 1] (m = 2..5), which keeps
    each term within 1/8 in magnitude up to 3500 K.  ``h298_R`` and ``s298_R``
    are the targets h(298.15 K)/R ~ U[-2e4, 2e4] K and s(298.15 K)/R ~
    U[15, 35]; the integration constants that hit them, and the high-range
    constants that make cp, h and s continuous at ``T_MID``, are solved for by
    the mechanism builder.
    """
    scale = (1e-3 / 3.5) ** np.arange(1, 5) / 8.0
    a1_lo = rng.uniform(2.5, 5.0, size=S)
    higher_lo = rng.uniform(-1.0, 1.0, size=(S, 4)) * scale
    higher_hi = rng.uniform(-1.0, 1.0, size=(S, 4)) * scale
    h298_R = rng.uniform(-2e4, 2e4, size=S)
    s298_R = rng.uniform(15.0, 35.0, size=S)
    return dict(a1_lo=a1_lo, higher_lo=higher_lo, higher_hi=higher_hi,
                h298_R=h298_R, s298_R=s298_R)


def _multisets_by_elements(comp, reactive, max_size=3):
    """Map element vector -> {size: [sorted species tuples]}."""
    E = comp.shape[0]
    base = int(comp.max()) * max_size + 1
    weights = base ** np.arange(E, dtype=np.int64)
    table = defaultdict(lambda: defaultdict(list))
    idx = np.asarray(reactive)
    for size in range(1, max_size + 1):
        combos = np.array(list(itertools.combinations_with_replacement(idx, size)),
                          dtype=np.int64).reshape(-1, size)
        vec = comp[:, combos].sum(axis=2)                     # (E, n_combos)
        keys = weights @ vec
        for key, c in zip(keys.tolist(), combos.tolist()):
            table[key][size].append(tuple(c))
    return table, weights


def reaction_candidates(rng, comp, reactive):
    """Endless stream of atom-balanced candidate reactions.

    Each candidate is ``(reactants, products)``, two sorted tuples of species
    indices in which a repeated index means a stoichiometric coefficient of 2
    or 3.  The reactant count is drawn from ``SIDE_SIZE_P``, the reactants
    uniformly with replacement; the product count is drawn from the same law
    and the products uniformly among the multisets of that size that carry
    the same atoms and share no species with the reactants.  A draw with no
    such multiset is discarded.
    """
    table, weights = _multisets_by_elements(comp, reactive)
    reactive = np.asarray(reactive)
    sizes = np.array([1, 2, 3])
    while True:
        nr = int(rng.choice(sizes, p=SIDE_SIZE_P))
        reac = tuple(sorted(int(x) for x in rng.choice(reactive, size=nr)))
        npr = int(rng.choice(sizes, p=SIDE_SIZE_P))
        key = int(weights @ comp[:, list(reac)].sum(axis=1))
        rset = set(reac)
        matches = [m for m in table[key][npr] if not rset.intersection(m)]
        if not matches:
            continue
        yield reac, matches[int(rng.integers(len(matches)))]


def draw_classes(rng, R, n_third_body, n_falloff, n_irreversible):
    """Reaction classes: 0 elementary, 1 third-body, 3 Troe falloff.

    Returns ``(rtype, reversible)``.  Irreversible reactions are drawn among
    the elementary ones.
    """
    perm = rng.permutation(R)
    rtype = np.zeros(R, dtype=np.int32)
    rtype[perm[:n_third_body]] = 1
    rtype[perm[n_third_body:n_third_body + n_falloff]] = 3
    reversible = np.ones(R, dtype=np.int32)
    elementary = np.sort(perm[n_third_body + n_falloff:])
    irr = rng.choice(elementary, size=n_irreversible, replace=False)
    reversible[irr] = 0
    return rtype, reversible


def draw_kinetics(rng, R, n_falloff, n_pd, S):
    """Arrhenius triples (ln A, b, Ea), low-pressure triples, Troe parameters
    and dense third-body efficiencies.

    ln A ~ U[ln 1e6, ln 1e14] (SI), b ~ U[-1.5, 1.5], Ea ~ U[0, 2e5] J/mol;
    Troe alpha ~ U[0.5, 0.8] and T***, T*, T** log-uniform on [1e1, 1e4] K;
    efficiencies ~ U[0.5, 12] for every species.
    """
    def triples(m):
        return np.stack([rng.uniform(np.log(1e6), np.log(1e14), size=m),
                         rng.uniform(-1.5, 1.5, size=m),
                         rng.uniform(0.0, 2e5, size=m)], axis=1)
    arrh = triples(R)
    low = triples(n_falloff)
    troe = np.stack([rng.uniform(0.5, 0.8, size=n_falloff),
                     10.0 ** rng.uniform(1.0, 4.0, size=n_falloff),
                     10.0 ** rng.uniform(1.0, 4.0, size=n_falloff),
                     10.0 ** rng.uniform(1.0, 4.0, size=n_falloff)], axis=1)
    eff = rng.uniform(0.5, 12.0, size=(n_pd, S))
    return arrh, low, troe, eff
