"""Builds the synthetic mechanism files ``cfg0.pyromech``, ``cfg1.pyromech``
and ``cfg3.pyromech`` in this directory from their seeds.

The random draws come from ``pyro_synth``; the thermodynamic integration
constants and the equilibrium-constant guard are evaluated with the oracle, so
every stored number is either a seeded draw or an oracle result.

* NASA7 low range: a6 and a7 are set so that h(298.15 K)/R and s(298.15 K)/R
  hit their drawn targets; high range: a1, a6 and a7 are set so that cp, h and
  s are continuous at T_mid = 1000 K.
* Guard: a candidate reaction is redrawn when |ln K_c(T)| > 230 anywhere on 64
  points spanning [300, 3000] K, which keeps every FP64 rate finite.

Usage: ``python mechanisms/make_mechanisms.py [--check]``; ``--check``
rebuilds into a temporary directory and compares bytes with the stored files.
"""

import argparse
import filecmp
import os
import sys
import tempfile
from types import SimpleNamespace

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from pyro_synth import CONFIGS, SEEDS  # noqa: E402
from pyro_synth import mechanism as draws  # noqa: E402
from pyro_synth import mechfile  # noqa: E402
from oracle import kinetics, thermo  # noqa: E402

GUARD_LNK = 230.0
GUARD_T = np.linspace(300.0, 3000.0, 64)
BUILT = (0, 1, 3)


def _nasa(th, S):
    T298 = np.array([298.15])
    Tm = np.array([draws.T_MID])
    lo = np.zeros((S, 7))
    lo[:, 0] = th["a1_lo"]
    lo[:, 1:5] = th["higher_lo"]
    lo[:, 5] = th["h298_R"] - 298.15 * thermo.h_RT_poly(lo, T298)[:, 0]
    lo[:, 6] = th["s298_R"] - thermo.s_R_poly(lo, T298)[:, 0]
    hi = np.zeros((S, 7))
    hi[:, 1:5] = th["higher_hi"]
    hi[:, 0] = thermo.cp_R_poly(lo, Tm)[:, 0] - thermo.cp_R_poly(hi, Tm)[:, 0]
    hi[:, 5] = Tm[0] * (thermo.h_RT_poly(lo, Tm) - thermo.h_RT_poly(hi, Tm))[:, 0]
    hi[:, 6] = (thermo.s_R_poly(lo, Tm) - thermo.s_R_poly(hi, Tm))[:, 0]
    return lo, hi


def build(cfg, path):
    c = CONFIGS[cfg]
    rng = np.random.default_rng(SEEDS["mechanism"] + cfg)
    elements, comp, reactive = draws.draw_species(rng, c)
    W, aw = draws.molecular_weights(elements, comp)
    S = comp.shape[1]
    lo, hi = _nasa(draws.draw_thermo(rng, S), S)
    T_range = np.tile([draws.T_LOW, draws.T_MID, draws.T_HIGH], (S, 1))
    thermo_view = SimpleNamespace(S=S, nasa_low=lo, nasa_high=hi,
                                  T_mid=T_range[:, 1])

    R = c["n_reactions"]
    accepted = []
    seen = set()
    for reac, prod in draws.reaction_candidates(rng, comp, reactive):
        if (reac, prod) in seen or (prod, reac) in seen:
            continue
        nu = np.zeros((S, 1))
        for k in prod:
            nu[k, 0] += 1
        for k in reac:
            nu[k, 0] -= 1
        view = SimpleNamespace(R=1, S=S, nu=nu, nasa_low=lo, nasa_high=hi,
                               T_mid=T_range[:, 1])
        with np.errstate(over="ignore", divide="ignore"):
            lnK = np.log(kinetics.equilibrium_constants(view, GUARD_T)[0])
        if not np.all(np.abs(lnK) <= GUARD_LNK):
            continue
        seen.add((reac, prod))
        accepted.append((reac, prod))
        if len(accepted) == R:
            break
    del thermo_view

    rtype, reversible = draws.draw_classes(
        rng, R, c["n_third_body"], c["n_falloff"], c["n_irreversible"])
    n_fo = int((rtype >= 2).sum())
    n_pd = int((rtype >= 1).sum())
    arrh, low, troe, eff = draws.draw_kinetics(rng, R, n_fo, n_pd, S)

    def side(t):
        ks, counts = np.unique(t, return_counts=True)
        return list(zip(ks.tolist(), counts.tolist()))

    mechfile.write(path, element_weight=aw, composition=comp, W=W,
                   T_range=T_range, nasa=np.stack([lo, hi], axis=1),
                   rtype=rtype, reversible=reversible, arrhenius=arrh,
                   reactants=[side(r) for r, _ in accepted],
                   products=[side(p) for _, p in accepted],
                   falloff_low=low, troe=troe, efficiency=eff)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--check", action="store_true")
    args = ap.parse_args()
    if args.check:
        with tempfile.TemporaryDirectory() as tmp:
            ok = True
            for cfg in BUILT:
                p = os.path.join(tmp, f"cfg{cfg}.pyromech")
                build(cfg, p)
                same = filecmp.cmp(p, os.path.join(HERE, f"cfg{cfg}.pyromech"),
                                   shallow=False)
                print(f"cfg{cfg}: {'identical' if same else 'DIFFERENT'}")
                ok &= same
        sys.exit(0 if ok else 1)
    for cfg in BUILT:
        p = os.path.join(HERE, f"cfg{cfg}.pyromech")
        build(cfg, p)
        print("wrote", p, os.path.getsize(p), "bytes")


if __name__ == "__main__":
    main()
