"""Torch-facing wrappers of libpyro: argument marshalling only.

Every array is a CUDA (HIP) tensor; per-species arrays are species-major
``(S, n)`` views whose row stride is ``ld`` (any ``ld >= n``), per-cell arrays
are contiguous ``(n,)``.  Calls are enqueued on torch's current stream.
"""

import ctypes
import os

import numpy as np
import torch

from . import _lib
from ._lib import PyroError, check, lib  # noqa: F401


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _species_major(Y, S, dtype, name):
    if Y.dim() != 2 or Y.shape[0] != S:
        raise ValueError(f"{name} must have shape (S={S}, n)")
    if Y.dtype != dtype or not Y.is_cuda:
        raise ValueError(f"{name} must be a {dtype} CUDA tensor")
    if Y.stride(1) != 1 or (S > 1 and Y.stride(0) < Y.shape[1]):
        raise ValueError(f"{name} must have unit cell stride and row stride >= n")
    return Y.stride(0) if S > 1 else max(Y.shape[1], 1)


def _cells(x, n, dtype, name):
    if x.dim() != 1 or x.shape[0] != n or x.dtype != dtype or not x.is_cuda:
        raise ValueError(f"{name} must be a contiguous ({n},) {dtype} CUDA tensor")
    if x.stride(0) != 1:
        raise ValueError(f"{name} must be contiguous")


class Mechanism:
    """A loaded mechanism (``pyro_mech_load``) on the current device."""

    def __init__(self, path):
        handle = ctypes.c_void_p()
        check(lib().pyro_mech_load(os.fsencode(path), ctypes.byref(handle)))
        self._h = handle
        info = _lib.MechInfo()
        check(lib().pyro_mech_get_info(handle, ctypes.byref(info)))
        self.n_species = info.n_species
        self.n_reactions = info.n_reactions
        self.n_elements = info.n_elements
        self.n_third_body = info.n_third_body
        self.n_falloff = info.n_falloff
        self.n_params = info.n_params
        self.nnz_reactant = info.nnz_reactant
        self.nnz_product = info.nnz_product
        self.nnz_net = info.nnz_net
        W = np.empty(self.n_species)
        check(lib().pyro_mech_molecular_weights(handle, W.ctypes.data_as(ctypes.c_void_p)))
        self.molecular_weights = W
        P = np.empty((self.n_params, 3))
        check(lib().pyro_mech_arrhenius(handle, P.ctypes.data_as(ctypes.c_void_p)))
        self.arrhenius = P
        self.device = torch.cuda.current_device()

    @property
    def handle(self):
        return self._h

    @property
    def wdot_variant(self):
        """The production-rate kernel variant (``_lib.PYRO_WDOT_*``)."""
        info = _lib.MechInfo()
        check(lib().pyro_mech_get_info(self._h, ctypes.byref(info)))
        return info.wdot_variant

    @wdot_variant.setter
    def wdot_variant(self, variant):
        check(lib().pyro_mech_set_wdot_variant(self._h, int(variant)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pyro_mech_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def production_rates(mech, rho, T, Y, out=None, params=None):
    """omega (S, n) from rho (n,), T (n,), Y (S, n); FP64 or FP32 tensors."""
    dtype = Y.dtype
    if dtype not in (torch.float64, torch.float32):
        raise ValueError("Y must be float64 or float32")
    S = mech.n_species
    n = Y.shape[1]
    ld = _species_major(Y, S, dtype, "Y")
    _cells(rho, n, dtype, "rho")
    _cells(T, n, dtype, "T")
    if out is None:
        out = torch.empty((S, ld), dtype=dtype, device=Y.device)[:, :n]
    if _species_major(out, S, dtype, "out") != ld:
        raise ValueError("out must have the row stride of Y")
    if params is not None:
        if params.dtype != torch.float64 or params.numel() != 3 * mech.n_params:
            raise ValueError("params must hold 3*n_params float64 values")
        params = params.contiguous()
    code = lib().pyro_production_rates(
        mech.handle, n, ld, _lib.PYRO_F64 if dtype == torch.float64 else _lib.PYRO_F32,
        _ptr(rho), _ptr(T), _ptr(Y), _ptr(out), _ptr(params), _stream(Y.device))
    check(code)
    return out


def temperature(mech, e, Y, T_guess=1200.0, max_iter=50, rtol=1e-12, out=None, status=None):
    """Newton inversion T(e, Y); returns (T, status)."""
    S = mech.n_species
    n = Y.shape[1]
    ld = _species_major(Y, S, torch.float64, "Y")
    _cells(e, n, torch.float64, "e")
    tg = None
    tg_value = 0.0
    if isinstance(T_guess, torch.Tensor):
        _cells(T_guess, n, torch.float64, "T_guess")
        tg = T_guess
    else:
        tg_value = float(T_guess)
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=Y.device)
    if status is None:
        status = torch.empty(n, dtype=torch.int32, device=Y.device)
    check(lib().pyro_temperature(mech.handle, n, ld, _ptr(e), _ptr(Y), _ptr(tg), tg_value,
                                 _ptr(out), _ptr(status), int(max_iter), float(rtol),
                                 _stream(Y.device)))
    return out, status


def temperature_from_enthalpy(mech, h, Y, T_guess=1200.0, max_iter=50, rtol=1e-12, out=None,
                              status=None):
    """Newton inversion T(h, Y) from the mass-specific enthalpy; returns
    (T, status)."""
    S = mech.n_species
    n = Y.shape[1]
    ld = _species_major(Y, S, torch.float64, "Y")
    _cells(h, n, torch.float64, "h")
    tg = None
    tg_value = 0.0
    if isinstance(T_guess, torch.Tensor):
        _cells(T_guess, n, torch.float64, "T_guess")
        tg = T_guess
    else:
        tg_value = float(T_guess)
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=Y.device)
    if status is None:
        status = torch.empty(n, dtype=torch.int32, device=Y.device)
    check(lib().pyro_temperature_from_enthalpy(mech.handle, n, ld, _ptr(h), _ptr(Y), _ptr(tg),
                                               tg_value, _ptr(out), _ptr(status), int(max_iter),
                                               float(rtol), _stream(Y.device)))
    return out, status


def primitive_from_conserved(mech, partial_densities, momentum, total_energy, T_guess=1200.0,
                             max_iter=50, rtol=1e-12):
    """(rho, Y, u, T, p, status) from the partial densities (S, n), the
    momentum (dim, n) with the row stride of the densities (or None) and the
    total energy (n,)."""
    S = mech.n_species
    n = partial_densities.shape[1]
    ld = _species_major(partial_densities, S, torch.float64, "partial_densities")
    _cells(total_energy, n, torch.float64, "total_energy")
    dim = 0 if momentum is None else momentum.shape[0]
    if dim:
        if (momentum.dim() != 2 or momentum.shape[1] != n or momentum.dtype != torch.float64
                or not momentum.is_cuda or momentum.stride(1) != 1
                or (dim > 1 and momentum.stride(0) != ld)):
            raise ValueError("momentum must be a (dim, n) float64 view with the row stride "
                             "of the densities")
    tg = None
    tg_value = 0.0
    if isinstance(T_guess, torch.Tensor):
        _cells(T_guess, n, torch.float64, "T_guess")
        tg = T_guess
    else:
        tg_value = float(T_guess)
    dev = partial_densities.device
    rho = torch.empty(n, dtype=torch.float64, device=dev)
    Y = torch.empty((S, ld), dtype=torch.float64, device=dev)[:, :n]
    u = torch.empty((max(dim, 1), ld), dtype=torch.float64, device=dev)[:dim, :n]
    T = torch.empty(n, dtype=torch.float64, device=dev)
    p = torch.empty(n, dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    check(lib().pyro_primitive_from_conserved(
        mech.handle, n, ld, dim, _ptr(partial_densities), _ptr(momentum if dim else None),
        _ptr(total_energy), _ptr(tg), tg_value, _ptr(rho), _ptr(Y), _ptr(u if dim else None),
        _ptr(T), _ptr(p), _ptr(status), int(max_iter), float(rtol), _stream(dev)))
    return rho, Y, u, T, p, status


def reactor_step(mech, method, rho, e, Y, T, dt, tol=1e-12, max_newton=20, status=None):
    """One reactor step in place on Y (S, n) and T (n,): ``method`` "rk4" or
    "cn"; dt a float or an (n,) tensor.  Returns status (n,) int32."""
    S = mech.n_species
    n = Y.shape[1]
    ld = _species_major(Y, S, torch.float64, "Y")
    _cells(rho, n, torch.float64, "rho")
    _cells(e, n, torch.float64, "e")
    _cells(T, n, torch.float64, "T")
    code = {"rk4": _lib.PYRO_REACTOR_RK4, "cn": _lib.PYRO_REACTOR_CN}[method]
    dtp, dtv = None, 0.0
    if isinstance(dt, torch.Tensor):
        _cells(dt, n, torch.float64, "dt")
        dtp = dt
    else:
        dtv = float(dt)
    if status is None:
        status = torch.empty(n, dtype=torch.int32, device=Y.device)
    size = lib().pyro_reactor_workspace_size(mech.handle, n, ld, code)
    ws = torch.empty(max(size, 1) + 256, dtype=torch.uint8, device=Y.device)
    off = (-ws.data_ptr()) % 256
    check(lib().pyro_reactor_step(mech.handle, code, n, ld, _ptr(rho), _ptr(e), _ptr(Y), _ptr(T),
                                  _ptr(dtp), dtv, float(tol), int(max_newton), _ptr(status),
                                  ctypes.c_void_p(ws.data_ptr() + off), size, _stream(Y.device)))
    return status


class Transport:
    """Device tables of a set of transport fits for a mechanism
    (``pyro_transport_create``): visc (S, 5), cond (S, 5), diff (S, S, 5)."""

    def __init__(self, mech, visc, cond, diff):
        S = mech.n_species
        visc = np.ascontiguousarray(visc, dtype=np.float64)
        cond = np.ascontiguousarray(cond, dtype=np.float64)
        diff = np.ascontiguousarray(diff, dtype=np.float64)
        if visc.shape != (S, 5) or cond.shape != (S, 5) or diff.shape != (S, S, 5):
            raise ValueError("fits must have shapes (S, 5), (S, 5) and (S, S, 5)")
        handle = ctypes.c_void_p()
        vp = ctypes.c_void_p
        check(lib().pyro_transport_create(mech.handle, visc.ctypes.data_as(vp),
                                          cond.ctypes.data_as(vp), diff.ctypes.data_as(vp),
                                          ctypes.byref(handle)))
        self._h = handle
        self.mech = mech

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pyro_transport_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mixture_transport(mech, tr, T, Y):
    """(mu (n,), kappa (n,), D (S, n)) of the mixture-averaged model."""
    S = mech.n_species
    n = Y.shape[1]
    ld = _species_major(Y, S, torch.float64, "Y")
    _cells(T, n, torch.float64, "T")
    mu = torch.empty(n, dtype=torch.float64, device=Y.device)
    kappa = torch.empty(n, dtype=torch.float64, device=Y.device)
    D = torch.empty((S, ld), dtype=torch.float64, device=Y.device)[:, :n]
    check(lib().pyro_mixture_transport(mech.handle, tr.handle, n, ld, _ptr(T), _ptr(Y), _ptr(mu),
                                       _ptr(kappa), _ptr(D), _stream(Y.device)))
    return mu, kappa, D


def density(mech, p, T, Y, out=None):
    S = mech.n_species
    n = Y.shape[1]
    ld = _species_major(Y, S, torch.float64, "Y")
    _cells(p, n, torch.float64, "p")
    _cells(T, n, torch.float64, "T")
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=Y.device)
    check(lib().pyro_density(mech.handle, n, ld, _ptr(p), _ptr(T), _ptr(Y), _ptr(out),
                             _stream(Y.device)))
    return out


def pressure(mech, rho, T, Y, out=None):
    S = mech.n_species
    n = Y.shape[1]
    ld = _species_major(Y, S, torch.float64, "Y")
    _cells(rho, n, torch.float64, "rho")
    _cells(T, n, torch.float64, "T")
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=Y.device)
    check(lib().pyro_pressure(mech.handle, n, ld, _ptr(rho), _ptr(T), _ptr(Y), _ptr(out),
                              _stream(Y.device)))
    return out


def internal_energy(mech, T, Y, out=None):
    S = mech.n_species
    n = Y.shape[1]
    ld = _species_major(Y, S, torch.float64, "Y")
    _cells(T, n, torch.float64, "T")
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=Y.device)
    check(lib().pyro_internal_energy(mech.handle, n, ld, _ptr(T), _ptr(Y), _ptr(out),
                                     _stream(Y.device)))
    return out


def production_rates_vjp(mech, rho, T, Y, wbar, params=None, Ybar=None, Tbar=None,
                         params_bar=None, wdot=None):
    """Gradients of L = sum wbar * omega (fixed rho): returns (Ybar, Tbar,
    params_bar) with params_bar of shape (n_params, 3) = dL/d(ln A, b, Ea).
    ``wdot``, an (S, n) view with the row stride of Y, also receives omega
    from the same pass."""
    S = mech.n_species
    n = Y.shape[1]
    ld = _species_major(Y, S, torch.float64, "Y")
    if _species_major(wbar, S, torch.float64, "wbar") != ld:
        raise ValueError("wbar must have the row stride of Y")
    _cells(rho, n, torch.float64, "rho")
    _cells(T, n, torch.float64, "T")
    if Ybar is None:
        Ybar = torch.empty((S, ld), dtype=torch.float64, device=Y.device)[:, :n]
    if _species_major(Ybar, S, torch.float64, "Ybar") != ld:
        raise ValueError("Ybar must have the row stride of Y")
    if Tbar is None:
        Tbar = torch.empty(n, dtype=torch.float64, device=Y.device)
    if params_bar is None:
        params_bar = torch.empty((mech.n_params, 3), dtype=torch.float64, device=Y.device)
    if params is not None:
        if params.dtype != torch.float64 or params.numel() != 3 * mech.n_params:
            raise ValueError("params must hold 3*n_params float64 values")
        params = params.contiguous()
    if wdot is not None and _species_major(wdot, S, torch.float64, "wdot") != ld:
        raise ValueError("wdot must have the row stride of Y")
    check(lib().pyro_production_rates_vjp(
        mech.handle, n, ld, _ptr(rho), _ptr(T), _ptr(Y), _ptr(wbar), _ptr(Ybar), _ptr(Tbar),
        _ptr(params_bar), _ptr(wdot), _ptr(params), _stream(Y.device)))
    return Ybar, Tbar, params_bar


def chemical_jacobian(mech, rho, T, Y, fixed_energy=True, params=None, out=None, dSdT=None):
    """J (S, S, n) with J[j, k] = dS_j/dY_k, S_j = W_j omega_j, at fixed
    density and (default) fixed internal energy, T being the state's
    temperature.  ``out`` may be an (S, S, n) view whose innermost rows have
    the row stride of Y; ``dSdT`` an (S, n) view with that stride."""
    S = mech.n_species
    n = Y.shape[1]
    ld = _species_major(Y, S, torch.float64, "Y")
    _cells(rho, n, torch.float64, "rho")
    _cells(T, n, torch.float64, "T")
    if out is None:
        out = torch.empty((S, S, ld), dtype=torch.float64, device=Y.device)[:, :, :n]
    if (out.shape != (S, S, n) or out.dtype != torch.float64 or not out.is_cuda
            or out.stride() != (S * ld, ld, 1)):
        raise ValueError("out must be an (S, S, n) float64 view with strides (S*ld, ld, 1)")
    if dSdT is not None and _species_major(dSdT, S, torch.float64, "dSdT") != ld:
        raise ValueError("dSdT must have the row stride of Y")
    if params is not None:
        if params.dtype != torch.float64 or params.numel() != 3 * mech.n_params:
            raise ValueError("params must hold 3*n_params float64 values")
        params = params.contiguous()
    check(lib().pyro_chemical_jacobian(mech.handle, n, ld, _ptr(rho), _ptr(T), _ptr(Y),
                                       1 if fixed_energy else 0, _ptr(out), _ptr(dSdT),
                                       _ptr(params), _stream(Y.device)))
    return out


class ProductionRates(torch.autograd.Function):
    """omega(rho, T, Y; params) with a reverse mode from the library's VJP
    kernel.  The density gets no gradient (omega is differentiated at fixed
    rho).  ``params`` is the (n_params, 3) tensor of (ln A, b, Ea)."""

    @staticmethod
    def forward(ctx, mech, rho, T, Y, params):
        ctx.mech = mech
        ctx.save_for_backward(rho, T, Y, params)
        return production_rates(mech, rho, T, Y,
                                params=None if params is None else params.detach().reshape(-1))

    @staticmethod
    def backward(ctx, grad_w):
        rho, T, Y, params = ctx.saved_tensors
        S, n = Y.shape
        wbar = torch.empty((S, Y.stride(0) if S > 1 else n), dtype=torch.float64,
                           device=Y.device)[:, :n]
        wbar.copy_(grad_w)
        Ybar, Tbar, pbar = production_rates_vjp(
            ctx.mech, rho, T, Y, wbar,
            params=None if params is None else params.detach().reshape(-1))
        return (None, None, Tbar if ctx.needs_input_grad[2] else None,
                Ybar if ctx.needs_input_grad[3] else None,
                pbar if params is not None and ctx.needs_input_grad[4] else None)


def production_rates_autograd(mech, rho, T, Y, params=None):
    return ProductionRates.apply(mech, rho, T, Y, params)
