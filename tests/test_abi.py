"""The C ABI without a GPU: the library loads, exports every symbol declared in
include/pyro.h, and rejects bad arguments and bad mechanism files before any
device work."""

import ctypes
import os
import re

import numpy as np
import pytest

import mechs
from pyro_synth import mechfile as writer

REPO = mechs.REPO
HEADER = os.path.join(REPO, "include", "pyro.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2503_24286_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.lib()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"PYRO_API\s+[\w\s\*]+?\b(pyro_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("pyro_mech_load", "pyro_production_rates", "pyro_temperature",
                 "pyro_last_error", "pyro_mech_free"):
        assert name in syms


def test_every_declared_symbol_is_exported(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name
    from paper_2503_24286_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared_symbols())


def _load(lib, path):
    h = ctypes.c_void_p()
    rc = lib.pyro_mech_load(os.fsencode(path), ctypes.byref(h))
    if rc == 0:
        lib.pyro_mech_free(h)
    return rc, lib.pyro_last_error().decode()


def test_load_errors(lib, tmp_path):
    from paper_2503_24286_amd import _lib
    h = ctypes.c_void_p()
    assert lib.pyro_mech_load(None, ctypes.byref(h)) == _lib.PYRO_E_ARG
    assert lib.pyro_last_error()
    rc, msg = _load(lib, str(tmp_path / "missing.pyromech"))
    assert rc == _lib.PYRO_E_IO and "cannot open" in msg
    blob = open(mechs.config_path(1), "rb").read()
    cases = {
        "truncated": blob[:-100],
        "magic": b"PYROMECX" + blob[8:],
        "version": blob[:8] + b"\x07" + blob[9:],
        "checksum": blob[:500] + bytes([blob[500] ^ 0x10]) + blob[501:],
        "short": blob[:30],
    }
    for name, b in cases.items():
        p = tmp_path / f"{name}.pyromech"
        p.write_bytes(b)
        rc, msg = _load(lib, str(p))
        assert rc == _lib.PYRO_E_FORMAT, (name, rc, msg)
        assert msg


def _write(path, reactions, W=(0.002, 0.032, 0.034), arrh_nan=False):
    S = len(W)
    a = mechs.constant_cp(S, 3.5, 0.0, 20.0)
    arrh = [r["arrh"] for r in reactions]
    if arrh_nan:
        arrh[0] = (np.nan, 0.0, 0.0)
    writer.write(path, element_weight=np.array([1.0]), composition=np.ones((1, S), np.int32),
                 W=np.array(W), T_range=np.tile([200.0, 1000.0, 3500.0], (S, 1)),
                 nasa=np.stack([a, a], axis=1), rtype=[0] * len(reactions),
                 reversible=[1] * len(reactions), arrhenius=arrh,
                 reactants=[r["reac"] for r in reactions],
                 products=[r["prod"] for r in reactions],
                 falloff_low=np.zeros((0, 3)), troe=np.zeros((0, 4)),
                 efficiency=np.zeros((0, S)))


def test_semantic_errors(lib, tmp_path):
    from paper_2503_24286_amd import _lib
    ok = dict(reac=[(0, 1), (1, 1)], prod=[(2, 1)], arrh=(1.0, 0.0, 0.0))
    p = str(tmp_path / "nan.pyromech")
    _write(p, [ok], arrh_nan=True)
    assert _load(lib, p)[0] == _lib.PYRO_E_FORMAT
    p = str(tmp_path / "index.pyromech")
    _write(p, [dict(ok, prod=[(7, 1)])])
    assert _load(lib, p)[0] == _lib.PYRO_E_FORMAT
    p = str(tmp_path / "negW.pyromech")
    _write(p, [ok], W=(0.002, -0.032, 0.034))
    assert _load(lib, p)[0] == _lib.PYRO_E_FORMAT
    p = str(tmp_path / "four.pyromech")
    _write(p, [dict(ok, reac=[(0, 2), (1, 2)])])
    rc, msg = _load(lib, p)
    assert rc == _lib.PYRO_E_UNSUPPORTED and "3 molecules" in msg
    # a well-formed file parses; without a device the upload then fails
    p = str(tmp_path / "good.pyromech")
    _write(p, [ok])
    assert _load(lib, p)[0] in (_lib.PYRO_OK, _lib.PYRO_E_HIP)


def test_call_validation(lib):
    from paper_2503_24286_amd import _lib
    nul = ctypes.c_void_p(0)
    one = ctypes.c_void_p(8)
    # null mechanism
    assert lib.pyro_production_rates(nul, 4, 4, 0, one, one, one, one, nul, nul) == _lib.PYRO_E_ARG
    assert "null mechanism" in lib.pyro_last_error().decode()
    # sizes and dtype are checked first
    assert lib.pyro_production_rates(nul, -1, 4, 0, one, one, one, one, nul, nul) == _lib.PYRO_E_ARG
    assert lib.pyro_production_rates(nul, 8, 4, 0, one, one, one, one, nul, nul) == _lib.PYRO_E_ARG
    assert "ld" in lib.pyro_last_error().decode()
    assert lib.pyro_production_rates(nul, 4, 4, 9, one, one, one, one, nul, nul) == _lib.PYRO_E_ARG
    assert lib.pyro_temperature(nul, 4, 4, one, one, nul, 1200.0, one, one, 0, 1e-12, nul) == _lib.PYRO_E_ARG
    assert lib.pyro_temperature(nul, 4, 4, one, one, nul, -5.0, one, one, 5, 1e-12, nul) == _lib.PYRO_E_ARG
    assert lib.pyro_temperature(nul, 4, 4, one, one, nul, 1200.0, one, one, 5, -1.0, nul) == _lib.PYRO_E_ARG
    for fn in ("pyro_density", "pyro_pressure"):
        assert getattr(lib, fn)(nul, 4, 4, one, one, one, one, nul) == _lib.PYRO_E_ARG
    assert lib.pyro_internal_energy(nul, 4, 4, one, one, one, nul) == _lib.PYRO_E_ARG
    info = _lib.MechInfo()
    assert lib.pyro_mech_get_info(nul, ctypes.byref(info)) == _lib.PYRO_E_ARG
    lib.pyro_mech_free(nul)           # a null handle is ignored
