"""Shared pieces of the GPU tests: device checks and seeded inputs."""

import json
import os
import sys

import numpy as np
import pytest

import mechs
from oracle import eos, thermo
from pyro_synth.states import draw_states


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def announce(msg):
    """Write a case name straight to the process's stderr, past pytest's
    capture, before a GPU step."""
    sys.__stderr__.write(f"[gpu-case] {msg}\n")
    sys.__stderr__.flush()


def record(case, quantity, value, tol):
    """Announce an achieved error level and, when PYRO_PARITY_LOG names a
    file, append it there as one JSON line (case, quantity, value, bar) so
    that a run's margins can be kept."""
    announce(f"  {case}: {quantity} {value:.3e} (bar {tol:.0e})")
    path = os.environ.get("PYRO_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps({"case": case, "quantity": quantity,
                                "value": float(value), "bar": float(tol)}) + "\n")


def states(cfg, n, S, first=0):
    """Seeded (T, p, Y) and the oracle's density for cells first..first+n-1."""
    T, p, Y = draw_states(cfg, n, S, first=first)
    m = mechs.load_config(1 if cfg in (2, 4) else cfg)
    rho = eos.density(m, p, T, Y)
    return T, p, Y, rho


def energies(m, T, Y):
    return thermo.mixture_internal_energy(m, T, Y)


def to_dev(torch, *arrays, dtype=None):
    out = []
    for a in arrays:
        t = torch.from_numpy(np.ascontiguousarray(a))
        if dtype is not None:
            t = t.to(dtype)
        out.append(t.cuda())
    return out
