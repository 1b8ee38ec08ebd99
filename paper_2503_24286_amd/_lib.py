"""ctypes loader of libpyro.so with the signatures of include/pyro.h.

The library must have been built (``__graft_entry__.build()`` or
``python -m paper_2503_24286_amd.build``); there is no fallback.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpyro.so")

PYRO_OK = 0
PYRO_E_ARG = -1
PYRO_E_IO = -2
PYRO_E_FORMAT = -3
PYRO_E_HIP = -4
PYRO_E_NOMEM = -5
PYRO_E_UNSUPPORTED = -6
STATUS_NAMES = {0: "PYRO_OK", -1: "PYRO_E_ARG", -2: "PYRO_E_IO", -3: "PYRO_E_FORMAT",
                -4: "PYRO_E_HIP", -5: "PYRO_E_NOMEM", -6: "PYRO_E_UNSUPPORTED"}
PYRO_F64 = 0
PYRO_F32 = 1
PYRO_WDOT_SPECIES_EQUILIBRIUM = 0
PYRO_WDOT_REACTION_EQUILIBRIUM = 1
PYRO_WDOT_MFMA_THIRD_BODY = 2
PYRO_WDOT_MFMA_NET_RATES = 4
PYRO_WDOT_LOG_SPACE = 8
PYRO_WDOT_MFMA_LOG_PRODUCTS = 16
PYRO_REACTOR_RK4 = 0
PYRO_REACTOR_CN = 1


class PyroError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


class MechInfo(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_reactions", ctypes.c_int32),
                ("n_elements", ctypes.c_int32), ("n_third_body", ctypes.c_int32),
                ("n_falloff", ctypes.c_int32), ("n_params", ctypes.c_int32),
                ("nnz_reactant", ctypes.c_int32), ("nnz_product", ctypes.c_int32),
                ("nnz_net", ctypes.c_int32), ("wdot_variant", ctypes.c_int32)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double

SIGNATURES = {
    "pyro_last_error": (ctypes.c_char_p, []),
    "pyro_mech_load": (_I, [ctypes.c_char_p, ctypes.POINTER(_P)]),
    "pyro_mech_free": (None, [_P]),
    "pyro_mech_get_info": (_I, [_P, ctypes.POINTER(MechInfo)]),
    "pyro_mech_set_wdot_variant": (_I, [_P, _I]),
    "pyro_mech_molecular_weights": (_I, [_P, _P]),
    "pyro_mech_arrhenius": (_I, [_P, _P]),
    "pyro_production_rates": (_I, [_P, _I64, _I64, _I, _P, _P, _P, _P, _P, _P]),
    "pyro_production_rates_vjp": (_I, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "pyro_temperature": (_I, [_P, _I64, _I64, _P, _P, _P, _D, _P, _P, _I, _D, _P]),
    "pyro_chemical_jacobian": (_I, [_P, _I64, _I64, _P, _P, _P, _I, _P, _P, _P, _P]),
    "pyro_production_rates_vjp_noalloc": (_I, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P,
                                               _P, _P]),
    "pyro_temperature_from_enthalpy": (_I, [_P, _I64, _I64, _P, _P, _P, _D, _P, _P, _I, _D, _P]),
    "pyro_primitive_from_conserved": (_I, [_P, _I64, _I64, _I, _P, _P, _P, _P, _D, _P, _P, _P,
                                           _P, _P, _P, _I, _D, _P]),
    "pyro_reactor_workspace_size": (ctypes.c_size_t, [_P, _I64, _I64, _I]),
    "pyro_reactor_step": (_I, [_P, _I, _I64, _I64, _P, _P, _P, _P, _P, _D, _D, _I, _P, _P,
                               ctypes.c_size_t, _P]),
    "pyro_transport_create": (_I, [_P, _P, _P, _P, ctypes.POINTER(_P)]),
    "pyro_transport_free": (None, [_P]),
    "pyro_mixture_transport": (_I, [_P, _P, _I64, _I64, _P, _P, _P, _P, _P, _P]),
    "pyro_density": (_I, [_P, _I64, _I64, _P, _P, _P, _P, _P]),
    "pyro_pressure": (_I, [_P, _I64, _I64, _P, _P, _P, _P, _P]),
    "pyro_internal_energy": (_I, [_P, _I64, _I64, _P, _P, _P, _P]),
}

class Surrogate(ctypes.Structure):
    _fields_ = [("n_members", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("weights", ctypes.c_void_p), ("biases", ctypes.c_void_p),
                ("feat_shift", ctypes.c_void_p), ("feat_scale", ctypes.c_void_p),
                ("target_scale", ctypes.c_void_p), ("target_mean", ctypes.c_void_p),
                ("target_std", ctypes.c_void_p)]


_SZ = ctypes.c_size_t
_F = ctypes.c_float
SIGNATURES.update({
    "pyro_mlp_param_counts": (_SZ, [_I, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "pyro_mlp_forward": (_I, [_I, _I64, _P, _P, _P, _P, _P, _P]),
    "pyro_mlp_backward": (_I, [_I, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _I, _P]),
    "pyro_mlp_loss_partials": (_I64, [_I64]),
    "pyro_mlp_mse": (_I, [_I64, _I, _P, _P, _P, _P, _P]),
    "pyro_adamw_step": (_I, [_I64, _P, _P, _P, _P, _P, _F, _F, _F, _F, _F, _I, _P]),
    "pyro_to_bf16": (_I, [_I64, _P, _P, _P]),
    "pyro_surrogate_features": (_I, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P]),
    "pyro_surrogate_targets": (_I, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P]),
    "pyro_surrogate_workspace_size": (_SZ, [_P, _I64, _I, _I]),
    "pyro_surrogate_eval": (_I, [_P, ctypes.POINTER(Surrogate), _I64, _I64, _P, _P, _P, _D, _D,
                                 _P, _P, _P, _P, _P, _SZ, _P]),
    "pyro_surrogate_outputs": (_I, [_P, ctypes.POINTER(Surrogate), _I64, _I64, _P, _P, _P, _P, _P,
                                    _SZ, _P]),
})

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(there is no CPU fallback)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            # a symbol this build of the library lacks stays unbound: calling
            # it raises AttributeError, the other entry points still work
            fn = getattr(handle, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def last_error():
    return lib().pyro_last_error().decode()


def check(code):
    if code != PYRO_OK:
        raise PyroError(code, last_error())
    return code
