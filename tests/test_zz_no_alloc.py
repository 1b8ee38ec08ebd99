"""The allocation-free VJP entry point (pyro_production_rates_vjp_noalloc)
against pyro_production_rates_vjp, called through the C ABI: two calls in a
row on the fixed scratch, the second with fewer cells, then n = 0."""

import ctypes

import numpy as np
import pytest

import mechs
from gpu_util import announce, states, to_dev, torch_cuda
from pyro_synth.states import draw_cotangent

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _call(lib, name, gm, r, t, y, wb, Yb, Tb, pb, w):
    S, n = y.shape
    return getattr(lib, name)(gm.handle, n, y.stride(0), _ptr(r), _ptr(t), _ptr(y), _ptr(wb),
                              _ptr(Yb), _ptr(Tb), _ptr(pb), _ptr(w), None, None)


def test_noalloc_vjp_matches_the_allocating_entry_point():
    torch = torch_cuda()
    import paper_2503_24286_amd as pyro
    from paper_2503_24286_amd import _lib
    lib = _lib.lib()
    gm = pyro.Mechanism(mechs.config_path(1))
    m = mechs.load_config(1)
    try:
        for n in (70_001, 1_000):              # the second call is smaller
            announce(f"no-alloc vjp n={n}")
            T, p, Y, rho = states(1, n, m.S, first=12)
            wbar = draw_cotangent(2, n, m.S, seed=n)
            r, t, y, wb = to_dev(torch, rho, T, Y, wbar)
            outs = []
            for name in ("pyro_production_rates_vjp", "pyro_production_rates_vjp_noalloc"):
                Yb = torch.full_like(y, 3.0)
                Tb = torch.full_like(t, 3.0)
                pb = torch.full((gm.n_params, 3), 3.0, dtype=torch.float64, device="cuda")
                w = torch.full_like(y, 3.0)
                assert _call(lib, name, gm, r, t, y, wb, Yb, Tb, pb, w) == _lib.PYRO_OK
                torch.cuda.synchronize()
                outs.append([x.cpu().numpy() for x in (Yb, Tb, pb, w)])
            for a, b in zip(*outs):
                assert np.array_equal(a, b)
        # no cells: the parameter gradients are zeroed without a memset
        e = torch.empty(0, dtype=torch.float64, device="cuda")
        Z = torch.empty((m.S, 0), dtype=torch.float64, device="cuda")
        pb = torch.full((gm.n_params, 3), 3.0, dtype=torch.float64, device="cuda")
        assert _call(lib, "pyro_production_rates_vjp_noalloc", gm, e, e, Z, Z, Z, e, pb,
                     None) == _lib.PYRO_OK
        torch.cuda.synchronize()
        assert bool((pb == 0).all())
    finally:
        gm.close()
