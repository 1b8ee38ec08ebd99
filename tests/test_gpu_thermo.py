"""Parity of the Newton temperature inversion and the EOS/energy helpers with
the oracle, through the C ABI."""

import numpy as np
import pytest

import mechs
from gpu_util import announce, record, states, to_dev, torch_cuda
from oracle import eos, newton, thermo
from pyro_synth.states import draw_guess_factors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib_mechs():
    torch = torch_cuda()
    import paper_2503_24286_amd as pyro
    out = {c: pyro.Mechanism(mechs.config_path(c)) for c in (0, 1, 3)}
    yield torch, pyro, out
    for m in out.values():
        m.close()


@pytest.mark.parametrize("cfg,n", [(0, 4096), (1, 3000)])
@pytest.mark.parametrize("guess", ["fixed", "per-cell"])
def test_newton_matches_oracle(lib_mechs, cfg, n, guess):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    T, p, Y, rho = states(cfg, n, m.S)
    e = thermo.mixture_internal_energy(m, T, Y)
    Tg = 1200.0 if guess == "fixed" else T * draw_guess_factors(cfg, n)
    T_ref, st_ref = newton.temperature(m, e, Y, Tg)
    announce(f"newton cfg{cfg} n={n} guess={guess}")
    e_d, Y_d = to_dev(torch, e, Y)
    tg = Tg if guess == "fixed" else to_dev(torch, Tg)[0]
    T_gpu, st = pyro.temperature(gms[cfg], e_d, Y_d, T_guess=tg)
    torch.cuda.synchronize()
    T_gpu = T_gpu.cpu().numpy()
    st = st.cpu().numpy()
    assert np.all(st > 0) and np.all(st_ref > 0)
    record(f"newton cfg{cfg} n={n} guess={guess}", "T relative vs oracle",
           np.max(np.abs(T_gpu - T_ref) / T_ref), 1e-12)
    np.testing.assert_allclose(T_gpu, T_ref, rtol=1e-12, atol=0)
    np.testing.assert_allclose(T_gpu, T, rtol=1e-12, atol=0)
    # iteration counts agree up to the last, rounding-decided update
    assert np.all(np.abs(st - st_ref) <= 1)


def test_newton_iteration_limit(lib_mechs):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    T, p, Y, rho = states(1, 300, m.S)
    e = thermo.mixture_internal_energy(m, T, Y)
    T1, st1 = newton.temperature(m, e, Y, 1200.0, max_iter=1)
    announce("newton max_iter=1")
    e_d, Y_d = to_dev(torch, e, Y)
    T_gpu, st = pyro.temperature(gms[1], e_d, Y_d, T_guess=1200.0, max_iter=1)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == st1)
    np.testing.assert_allclose(T_gpu.cpu().numpy(), T1, rtol=1e-12)


@pytest.mark.parametrize("n", [1, 63, 65, 257])
def test_newton_ragged_and_padded(lib_mechs, n):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    T, p, Y, rho = states(1, n, m.S, first=300)
    e = thermo.mixture_internal_energy(m, T, Y)
    announce(f"newton ragged n={n}")
    Yb = torch.full((m.S, n + 5), float("nan"), dtype=torch.float64, device="cuda")
    Yb[:, :n] = torch.from_numpy(Y).cuda()
    (e_d,) = to_dev(torch, e)
    T_gpu, st = pyro.temperature(gms[1], e_d, Yb[:, :n], T_guess=1500.0)
    torch.cuda.synchronize()
    np.testing.assert_allclose(T_gpu.cpu().numpy(), T, rtol=1e-12)


def test_eos_and_energy_helpers(lib_mechs):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    T, p, Y, rho = states(1, 2000, m.S, first=40000)
    announce("eos helpers")
    p_d, T_d, Y_d, rho_d = to_dev(torch, p, T, Y, rho)
    r = pyro.density(gms[1], p_d, T_d, Y_d)
    pp = pyro.pressure(gms[1], rho_d, T_d, Y_d)
    e = pyro.internal_energy(gms[1], T_d, Y_d)
    torch.cuda.synchronize()
    np.testing.assert_allclose(r.cpu().numpy(), eos.density(m, p, T, Y), rtol=1e-14)
    np.testing.assert_allclose(pp.cpu().numpy(), eos.pressure(m, rho, T, Y), rtol=1e-14)
    e_ref = thermo.mixture_internal_energy(m, T, Y)
    # e is a sum of terms of both signs: compare against their magnitude
    scale = np.abs(Y * thermo.species_internal_energy(m, T)).sum(axis=0)
    assert np.all(np.abs(e.cpu().numpy() - e_ref) <= 1e-13 * scale)


@pytest.mark.parametrize("cfg,n", [(0, 4096), (1, 3000 + 7)])
def test_temperature_from_enthalpy_matches_oracle(lib_mechs, cfg, n):
    """The enthalpy-based Newton inversion against the oracle's, fixed and
    per-cell guesses; T round trip T -> h(T, Y) -> T."""
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    T, p, Y, rho = states(cfg, n, m.S, first=600)
    h = thermo.mixture_enthalpy(m, T, Y)
    for guess in ("fixed", "per-cell"):
        Tg = 1200.0 if guess == "fixed" else T * draw_guess_factors(cfg, n)
        T_ref, st_ref = newton.temperature_from_enthalpy(m, h, Y, Tg)
        announce(f"enthalpy newton cfg{cfg} n={n} guess={guess}")
        h_d, Y_d = to_dev(torch, h, Y)
        tg = Tg if guess == "fixed" else to_dev(torch, Tg)[0]
        T_gpu, st = pyro.temperature_from_enthalpy(gms[cfg], h_d, Y_d, T_guess=tg)
        torch.cuda.synchronize()
        T_gpu = T_gpu.cpu().numpy()
        st = st.cpu().numpy()
        assert np.all(st > 0) and np.all(st_ref > 0)
        record(f"enthalpy newton cfg{cfg} n={n} guess={guess}", "T relative vs oracle",
               np.max(np.abs(T_gpu - T_ref) / T_ref), 1e-12)
        np.testing.assert_allclose(T_gpu, T_ref, rtol=1e-12, atol=0)
        np.testing.assert_allclose(T_gpu, T, rtol=1e-12, atol=0)
        assert np.all(np.abs(st - st_ref) <= 1)


@pytest.mark.parametrize("dim", [0, 1, 3])
@pytest.mark.parametrize("cfg,n", [(0, 1000), (1, 2000 + 13), (3, 700)])
def test_primitive_from_conserved_matches_oracle(lib_mechs, cfg, n, dim):
    """rho, Y, u, T, p from (rho_k, rho u, E) against the oracle's routine,
    with padded rows (ld > n) left untouched (configs 0 and 1 hold the
    partial densities in registers, config 3's 160 species are read twice)."""
    from oracle import primitive
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    T, p, Y, rho = states(cfg, n, m.S, first=1700)
    rng = np.random.default_rng(100 + dim)
    u = rng.uniform(-300.0, 300.0, (dim, n))
    e = thermo.mixture_internal_energy(m, T, Y)
    dens = rho * Y
    mom = rho * u
    E = rho * (e + 0.5 * (u ** 2).sum(axis=0))
    ref = primitive.primitive_from_conserved(m, dens, mom, E, 1200.0)
    announce(f"primitive cfg{cfg} n={n} dim={dim}")
    ld = n + 5
    dd = torch.full((m.S, ld), 9.0, dtype=torch.float64, device="cuda")[:, :n]
    dd.copy_(torch.from_numpy(dens))
    md = None
    if dim:
        md = torch.zeros((dim, ld), dtype=torch.float64, device="cuda")[:, :n]
        md.copy_(torch.from_numpy(mom))
    (E_d,) = to_dev(torch, E)
    out = pyro.primitive_from_conserved(gms[cfg], dd, md, E_d, T_guess=1200.0)
    torch.cuda.synchronize()
    rho_g, Y_g, u_g, T_g, p_g, st_g = (x.cpu().numpy() for x in out)
    rho_r, Y_r, u_r, T_r, p_r, st_r = ref
    np.testing.assert_allclose(rho_g, rho_r, rtol=1e-14)
    np.testing.assert_allclose(Y_g, Y_r, rtol=1e-14, atol=0)
    if dim:
        np.testing.assert_allclose(u_g, u_r, rtol=1e-14)
    assert np.all(st_g > 0) and np.all(np.abs(st_g - st_r) <= 1)
    eT = np.max(np.abs(T_g - T_r) / T_r)
    ep = np.max(np.abs(p_g - p_r) / p_r)
    record(f"primitive cfg{cfg} n={n} dim={dim}", "T relative vs oracle", eT, 1e-12)
    record(f"primitive cfg{cfg} n={n} dim={dim}", "p relative vs oracle", ep, 1e-12)
    assert eT <= 1e-12 and ep <= 1e-12
    # the state the conserved variables were built from comes back
    np.testing.assert_allclose(T_g, T, rtol=1e-11)
    np.testing.assert_allclose(p_g, p, rtol=1e-11)


def test_primitive_and_enthalpy_errors(lib_mechs):
    from paper_2503_24286_amd import _lib
    torch, pyro, gms = lib_mechs
    lib = _lib.lib()
    h = gms[0].handle
    one = torch.ones(4, dtype=torch.float64, device="cuda")
    ptr = one.data_ptr()
    assert lib.pyro_primitive_from_conserved(h, 4, 4, 4, ptr, ptr, ptr, None, 1200.0, ptr, ptr,
                                             ptr, ptr, ptr, ptr, 5, 1e-12, None) == _lib.PYRO_E_ARG
    assert lib.pyro_primitive_from_conserved(h, 4, 4, 1, ptr, None, ptr, None, 1200.0, ptr, ptr,
                                             None, ptr, ptr, ptr, 5, 1e-12, None) == _lib.PYRO_E_ARG
    assert lib.pyro_temperature_from_enthalpy(h, 4, 4, ptr, ptr, None, -1.0, ptr, ptr, 5, 1e-12,
                                              None) == _lib.PYRO_E_ARG
    torch.cuda.synchronize()
