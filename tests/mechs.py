"""Small hand-made mechanisms for the tests.

Each is written to a ``.pyromech`` file with the input writer and read back
with the oracle's parser, so the same file can be handed to the GPU library.
"""

import os

import numpy as np

from pyro_synth import mechfile as writer
from oracle import mechfile

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MECH_DIR = os.path.join(REPO, "mechanisms")


def config_path(cfg):
    return os.path.join(MECH_DIR, f"cfg{cfg}.pyromech")


def load_config(cfg):
    return mechfile.load(config_path(cfg))


def constant_cp(S, a1, a6, a7):
    """NASA7 rows with only a1, a6, a7 (constant heat capacity)."""
    a = np.zeros((S, 7))
    a[:, 0] = a1
    a[:, 5] = a6
    a[:, 6] = a7
    return a


def make(path, W, nasa_low, reactions, nasa_high=None, T_mid=1000.0,
         composition=None, element_weight=None):
    """Write a mechanism.

    ``reactions`` is a list of dicts with keys ``reac``, ``prod`` (lists of
    ``(species, nu)``), ``arrh`` (ln A, b, Ea) and optionally ``type``
    (0, 1, 2, 3), ``reversible``, ``low``, ``troe``, ``eff``.
    """
    W = np.asarray(W, float)
    S = len(W)
    nasa_low = np.asarray(nasa_low, float)
    nasa_high = nasa_low if nasa_high is None else np.asarray(nasa_high, float)
    if composition is None:
        composition = np.ones((1, S), np.int32)
        element_weight = np.array([1.0])
    rtype = [r.get("type", 0) for r in reactions]
    low = [r["low"] for r in reactions if r.get("type", 0) >= 2]
    troe = [r.get("troe", (0.5, 100.0, 1000.0, 1000.0)) for r in reactions
            if r.get("type", 0) >= 2]
    eff = [r.get("eff", np.ones(S)) for r in reactions if r.get("type", 0) >= 1]
    writer.write(path, element_weight=element_weight, composition=composition,
                 W=W, T_range=np.tile([200.0, T_mid, 3500.0], (S, 1)),
                 nasa=np.stack([nasa_low, nasa_high], axis=1), rtype=rtype,
                 reversible=[int(r.get("reversible", True)) for r in reactions],
                 arrhenius=[r["arrh"] for r in reactions],
                 reactants=[r["reac"] for r in reactions],
                 products=[r["prod"] for r in reactions],
                 falloff_low=np.array(low).reshape(-1, 3),
                 troe=np.array(troe).reshape(-1, 4),
                 efficiency=np.array(eff).reshape(-1, S))
    return mechfile.load(path)
