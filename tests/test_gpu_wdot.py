"""Parity of the HIP production-rate kernel with the oracle, through the C ABI."""

import numpy as np
import pytest

import mechs
from gpu_util import announce, record, states, to_dev, torch_cuda
from parity import assert_wdot_parity
from oracle import kinetics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib_mechs():
    torch = torch_cuda()
    import paper_2503_24286_amd as pyro
    out = {c: pyro.Mechanism(mechs.config_path(c)) for c in (0, 1)}
    yield torch, pyro, out
    for m in out.values():
        m.close()


def _run(torch, pyro, gm, rho, T, Y, params=None):
    r, t, y = to_dev(torch, rho, T, Y)
    p = None if params is None else to_dev(torch, params)[0]
    w = pyro.production_rates(gm, r, t, y, params=p)
    torch.cuda.synchronize()
    return w.cpu().numpy()


@pytest.mark.parametrize("cfg,n", [(0, 4096), (1, 1000), (1, 4096 + 37)])
def test_wdot_matches_oracle(lib_mechs, cfg, n):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    T, p, Y, rho = states(cfg, n, m.S)
    announce(f"wdot cfg{cfg} n={n}")
    w = _run(torch, pyro, gms[cfg], rho, T, Y)
    r = assert_wdot_parity(m, rho, T, Y, w)
    record(f"wdot cfg{cfg} n={n}", "omega scaled", r["scaled"].max(), 1e-12)
    well = r["kappa"] <= 1e3
    record(f"wdot cfg{cfg} n={n}", "omega normwise (kappa <= 1e3)", r["normwise"][well].max(), 1e-12)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 129, 200])
def test_wdot_ragged_sizes_and_padded_rows(lib_mechs, n):
    """Partial tiles and a row stride ld > n: padding must neither be read
    into results nor written."""
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    T, p, Y, rho = states(1, n, m.S, first=5000)
    ld = n + 29
    announce(f"wdot ragged n={n} ld={ld}")
    Yb = torch.full((m.S, ld), float("nan"), dtype=torch.float64, device="cuda")
    Yb[:, :n] = torch.from_numpy(Y).cuda()
    out = torch.full((m.S, ld), -7.0, dtype=torch.float64, device="cuda")
    r, t = to_dev(torch, rho, T)
    pyro.production_rates(gms[1], r, t, Yb[:, :n], out=out[:, :n])
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.all(o[:, n:] == -7.0)
    assert_wdot_parity(m, rho, T, Y, o[:, :n])


def test_wdot_tiled_states_identical(lib_mechs):
    """The same state repeated over a grid gives the same result in every
    cell (the paper's multi-dimensional input example, Sec. 4.1)."""
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    T, p, Y, rho = states(1, 3, m.S, first=77)
    reps = 300
    announce("wdot tiled states")
    w = _run(torch, pyro, gms[1], np.tile(rho, reps), np.tile(T, reps), np.tile(Y, reps))
    w = w.reshape(m.S, reps, 3)
    assert np.all(w == w[:, :1, :])
    assert_wdot_parity(m, rho, T, Y, w[:, 0, :])


def test_wdot_zero_cells_is_noop(lib_mechs):
    torch, pyro, gms = lib_mechs
    S = gms[1].n_species
    announce("wdot n=0")
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    w = pyro.production_rates(gms[1], e, e, torch.empty((S, 0), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert w.shape == (S, 0)


def test_wdot_degenerate_states(lib_mechs):
    """Zero and negative mass fractions, a single-species mixture, and the
    ends of the NASA7 ranges (T at T_mid exactly and just above)."""
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    T, p, Y, rho = states(1, 256, m.S, first=9000)
    Y[:, :64] = 0.0
    Y[5, :64] = 1.0                       # pure species 5
    Y[3, 64:128] = -1e-3                  # negative mass fraction counts as zero
    Y[:, 128:192] *= 0.5                  # sum(Y) = 1/2
    T[192:200] = m.T_mid[0]
    T[200:208] = np.nextafter(m.T_mid[0], 4000.0)
    announce("wdot degenerate states")
    w = _run(torch, pyro, gms[1], rho, T, Y)
    assert_wdot_parity(m, rho, T, Y, w)
    inert = np.nonzero(np.abs(m.nu).sum(axis=1) == 0)[0]
    assert np.all(w[inert] == 0.0)


def test_wdot_parameter_override(lib_mechs):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    T, p, Y, rho = states(1, 500, m.S, first=123)
    P = m.parameters().copy()
    rng = np.random.default_rng(8)
    P[:, 0] += rng.uniform(-1, 1, P.shape[0])
    P[:, 1] += rng.uniform(-0.2, 0.2, P.shape[0])
    P[:, 2] *= rng.uniform(0.8, 1.2, P.shape[0])
    announce("wdot params override")
    w = _run(torch, pyro, gms[1], rho, T, Y, params=P.reshape(-1))
    assert_wdot_parity(m, rho, T, Y, w, params=P)
    assert np.allclose(gms[1].arrhenius, m.parameters(), rtol=0, atol=0)


def test_wdot_full_size_sampled(lib_mechs):
    """The benchmark's workload: 2^22 cells of config 1 in one launch;
    sampled cells are checked against the oracle one by one."""
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    n = 1 << 22
    T, p, Y, rho = states(1, n, m.S)
    announce(f"wdot full size n={n}")
    r, t, y = to_dev(torch, rho, T, Y)
    w = pyro.production_rates(gms[1], r, t, y)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(w).all())
    rng = np.random.default_rng(99)
    idx = np.unique(np.concatenate([rng.integers(0, n, 2000), np.arange(64),
                                    np.arange(n - 64, n)]))
    ws = w[:, torch.from_numpy(idx).cuda()].cpu().numpy()
    assert_wdot_parity(m, rho[idx], T[idx], Y[:, idx], ws)


@pytest.fixture(scope="module")
def cfg3_mech():
    torch = torch_cuda()
    import paper_2503_24286_amd as pyro
    gm = pyro.Mechanism(mechs.config_path(3))
    yield torch, pyro, gm
    gm.close()


@pytest.mark.parametrize("cfg,n", [(0, 1000), (1, 2000 + 45)])
def test_both_equilibrium_variants_match_oracle(lib_mechs, cfg, n):
    """The species-equilibrium (per-species exp(g/RT) in LDS) and the
    reaction-equilibrium (combined coefficients, one exp per reversible
    reaction) kernels, each with the third-body concentrations and the net
    rates nu q on the FMA units or on the FP64 matrix cores, all pass the
    parity bar."""
    from paper_2503_24286_amd import _lib
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    gm = gms[cfg]
    T, p, Y, rho = states(cfg, n, m.S, first=3333)
    before = gm.wdot_variant
    try:
        for variant in range(8):   # equilibrium form | MFMA [M] | MFMA nu q
            gm.wdot_variant = variant
            assert gm.wdot_variant == variant
            announce(f"wdot variant {variant} cfg{cfg} n={n}")
            w = _run(torch, pyro, gm, rho, T, Y)
            r = assert_wdot_parity(m, rho, T, Y, w)
            record(f"wdot variant {variant} cfg{cfg} n={n}", "omega scaled", r["scaled"].max(), 1e-12)
    finally:
        gm.wdot_variant = before


@pytest.mark.parametrize("n", [300, 64 * 5 + 17])
def test_large_mechanism_net_rates_on_mfma(cfg3_mech, n):
    """The 160-species mechanism with omega = nu q on the FP64 matrix cores:
    ten 16-species blocks spread over the 16 wavefronts (three per wave),
    32-slot chunks (eight K-steps), at the FP64 parity bar."""
    from paper_2503_24286_amd import _lib
    torch, pyro, gm = cfg3_mech
    m = mechs.load_config(3)
    T, p, Y, rho = states(3, n, m.S, first=100000)
    announce(f"wdot cfg3 MFMA net rates n={n}")
    before = gm.wdot_variant
    try:
        gm.wdot_variant = _lib.PYRO_WDOT_REACTION_EQUILIBRIUM | _lib.PYRO_WDOT_MFMA_NET_RATES
        w = _run(torch, pyro, gm, rho, T, Y)
    finally:
        gm.wdot_variant = before
    r = assert_wdot_parity(m, rho, T, Y, w)
    record(f"wdot cfg3 MFMA net rates n={n}", "omega scaled", r["scaled"].max(), 1e-12)


@pytest.mark.parametrize("n", [300, 64 * 5 + 17])
def test_large_mechanism_matches_oracle(cfg3_mech, n):
    """The 160-species, 900-reaction mechanism: its species rows do not fit
    the LDS tile, so the loader selects the reaction-equilibrium kernel (in
    its 16-wavefront form); the [M] block of the MFMA third-body flag no
    longer fits beside it."""
    from paper_2503_24286_amd import _lib
    torch, pyro, gm = cfg3_mech
    m = mechs.load_config(3)
    assert gm.wdot_variant == _lib.PYRO_WDOT_REACTION_EQUILIBRIUM
    T, p, Y, rho = states(3, n, m.S, first=100000)
    announce(f"wdot cfg3 n={n}")
    w = _run(torch, pyro, gm, rho, T, Y)
    r = assert_wdot_parity(m, rho, T, Y, w)
    record(f"wdot cfg3 n={n}", "omega scaled", r["scaled"].max(), 1e-12)
    with pytest.raises(_lib.PyroError) as e:
        gm.wdot_variant = _lib.PYRO_WDOT_REACTION_EQUILIBRIUM | _lib.PYRO_WDOT_MFMA_THIRD_BODY
    assert e.value.code == _lib.PYRO_E_UNSUPPORTED
    assert gm.wdot_variant == _lib.PYRO_WDOT_REACTION_EQUILIBRIUM


def test_variant_selection_errors(cfg3_mech):
    from paper_2503_24286_amd import _lib
    torch, pyro, gm = cfg3_mech
    with pytest.raises(_lib.PyroError) as e:
        gm.wdot_variant = _lib.PYRO_WDOT_SPECIES_EQUILIBRIUM
    assert e.value.code == _lib.PYRO_E_UNSUPPORTED
    with pytest.raises(_lib.PyroError) as e:   # species rows exceed the LDS
        gm.wdot_variant = _lib.PYRO_WDOT_SPECIES_EQUILIBRIUM | _lib.PYRO_WDOT_MFMA_NET_RATES
    assert e.value.code == _lib.PYRO_E_UNSUPPORTED
    with pytest.raises(_lib.PyroError) as e:   # 160 (C, ln C) rows exceed the LDS
        gm.wdot_variant = _lib.PYRO_WDOT_LOG_SPACE
    assert e.value.code == _lib.PYRO_E_UNSUPPORTED
    with pytest.raises(_lib.PyroError) as e:   # a flag of the log-space form only
        gm.wdot_variant = _lib.PYRO_WDOT_MFMA_LOG_PRODUCTS
    assert e.value.code == _lib.PYRO_E_ARG
    with pytest.raises(_lib.PyroError) as e:
        gm.wdot_variant = _lib.PYRO_WDOT_LOG_SPACE | _lib.PYRO_WDOT_MFMA_LOG_PRODUCTS
    assert e.value.code == _lib.PYRO_E_UNSUPPORTED
    with pytest.raises(_lib.PyroError) as e:
        gm.wdot_variant = 32
    assert e.value.code == _lib.PYRO_E_ARG
    with pytest.raises(_lib.PyroError) as e:
        gm.wdot_variant = -1
    assert e.value.code == _lib.PYRO_E_ARG
    assert gm.wdot_variant == _lib.PYRO_WDOT_REACTION_EQUILIBRIUM


@pytest.mark.parametrize("cfg,n", [(0, 1000), (1, 2000 + 45)])
def test_log_space_variant_matches_oracle(lib_mechs, cfg, n):
    """The log-space form (each rate one exponential of ln k plus sums of
    nu ln C) at the FP64 parity bar, with degenerate states: zero and
    negative mass fractions (ln C = -inf), a pure species, T at T_mid."""
    from paper_2503_24286_amd import _lib
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    gm = gms[cfg]
    T, p, Y, rho = states(cfg, n, m.S, first=3333)
    Y[:, :32] = 0.0
    Y[min(5, m.S - 1), :32] = 1.0
    Y[3, 32:64] = -1e-3
    T[64:72] = m.T_mid[0]
    before = gm.wdot_variant
    try:
        gm.wdot_variant = _lib.PYRO_WDOT_LOG_SPACE
        assert gm.wdot_variant == _lib.PYRO_WDOT_LOG_SPACE | _lib.PYRO_WDOT_REACTION_EQUILIBRIUM
        announce(f"wdot log-space cfg{cfg} n={n}")
        w = _run(torch, pyro, gm, rho, T, Y)
        r = assert_wdot_parity(m, rho, T, Y, w)
        record(f"wdot log-space cfg{cfg} n={n}", "omega scaled", r["scaled"].max(), 1e-12)
        for bad in (_lib.PYRO_WDOT_LOG_SPACE | _lib.PYRO_WDOT_MFMA_THIRD_BODY,
                    _lib.PYRO_WDOT_LOG_SPACE | _lib.PYRO_WDOT_MFMA_NET_RATES):
            with pytest.raises(_lib.PyroError):
                gm.wdot_variant = bad
    finally:
        gm.wdot_variant = before


@pytest.mark.parametrize("cfg,n", [(0, 1000), (1, 2000 + 45)])
def test_log_products_on_mfma_match_oracle(lib_mechs, cfg, n):
    """The log-space form with its stoichiometric log sums (sum_k nu'_kj ln C_k,
    sum_k nu''_kj ln C_k) as dense products on the FP64 matrix cores, at the
    FP64 parity bar, with the same degenerate states as the VALU form (ln 0
    floored at -1e30 so that zero coefficients times it stay zero)."""
    from paper_2503_24286_amd import _lib
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    gm = gms[cfg]
    T, p, Y, rho = states(cfg, n, m.S, first=3333)
    Y[:, :32] = 0.0
    Y[min(5, m.S - 1), :32] = 1.0
    Y[3, 32:64] = -1e-3
    T[64:72] = m.T_mid[0]
    before = gm.wdot_variant
    try:
        gm.wdot_variant = _lib.PYRO_WDOT_LOG_SPACE | _lib.PYRO_WDOT_MFMA_LOG_PRODUCTS
        assert gm.wdot_variant == (_lib.PYRO_WDOT_LOG_SPACE | _lib.PYRO_WDOT_REACTION_EQUILIBRIUM
                                   | _lib.PYRO_WDOT_MFMA_LOG_PRODUCTS)
        announce(f"wdot log products on MFMA cfg{cfg} n={n}")
        w = _run(torch, pyro, gm, rho, T, Y)
        r = assert_wdot_parity(m, rho, T, Y, w)
        record(f"wdot log products on MFMA cfg{cfg} n={n}", "omega scaled", r["scaled"].max(),
               1e-12)
    finally:
        gm.wdot_variant = before


# FP32: the stated bar is 1e-4 of the summed terms' magnitudes per species,
# floored at 1e-36 (results below the float normal range keep few digits)
TOL_F32 = 1e-4
F32_FLOOR = 1e-36
F32_MAX = float(np.finfo(np.float32).max)


def fp32_classes(m, rho, T, Y):
    """Per cell, from the oracle's FP64 rates: 'safe' when every partial sum
    of the species gathering stays below half the float range (no result can
    overflow), 'over' when some rate exceeds twice the float range (the
    log-space kernel must return a non-finite omega), else undecided."""
    Rf, Rr, phi, q = kinetics.rates_of_progress(m, rho, T, Y)
    mag = np.abs(m.nu) @ ((np.abs(Rf) + np.abs(Rr)) * np.abs(phi))
    big = np.maximum(np.abs(Rf), np.abs(Rr)) * np.abs(phi)
    safe = mag.max(axis=0) < 0.5 * F32_MAX
    over = big.max(axis=0) > 2.0 * F32_MAX
    return safe, over, mag


@pytest.mark.parametrize("cfg,n", [(0, 4096), (1, 4096 + 37)])
def test_fp32_matches_oracle(lib_mechs, cfg, n):
    """PYRO_F32 against the FP64 oracle on the same (float-rounded) inputs:
    cells whose rates fit the float range are finite and within 1e-4 scaled;
    cells with a rate beyond it come back non-finite (counted)."""
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    T, p, Y, rho = states(cfg, n, m.S, first=2024)
    T32, r32, Y32 = (a.astype(np.float32) for a in (T, rho, Y))
    T, rho, Y = (a.astype(np.float64) for a in (T32, r32, Y32))
    announce(f"wdot fp32 cfg{cfg} n={n}")
    r, t, y = to_dev(torch, r32, T32, Y32)
    w = pyro.production_rates(gms[cfg], r, t, y)
    torch.cuda.synchronize()
    assert w.dtype == torch.float32
    w = w.cpu().numpy().astype(np.float64)
    safe, over, mag = fp32_classes(m, rho, T, Y)
    w_ref = kinetics.net_production_rates(m, rho, T, Y)
    finite = np.isfinite(w).all(axis=0)
    assert np.all(finite[safe]), f"{np.sum(~finite[safe])} in-range cells are not finite"
    assert not np.any(finite[over]), f"{np.sum(finite[over])} overflowing cells came back finite"
    err = (np.abs(w - w_ref) / np.maximum(mag, F32_FLOOR))[:, safe].max(axis=0)
    case = f"wdot fp32 cfg{cfg} n={n}"
    record(case, "omega scaled (in-range cells)", err.max(), TOL_F32)
    record(case, "fraction of cells with a rate beyond the float range", over.mean(), 1.0)
    record(case, "fraction undecided (near the float limit)", (~safe & ~over).mean(), 1.0)
    assert err.max() <= TOL_F32, f"scaled error {err.max():.3e} at cell {np.argmax(err)}"


def test_fp32_ragged_and_padded(lib_mechs):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    n = 129
    T, p, Y, rho = states(1, n, m.S, first=31)
    ld = n + 11
    announce("wdot fp32 ragged/padded")
    Yb = torch.full((m.S, ld), float("nan"), dtype=torch.float32, device="cuda")
    Yb[:, :n] = torch.from_numpy(Y.astype(np.float32)).cuda()
    out = torch.full((m.S, ld), -3.0, dtype=torch.float32, device="cuda")
    r, t = to_dev(torch, rho.astype(np.float32), T.astype(np.float32))
    pyro.production_rates(gms[1], r, t, Yb[:, :n], out=out[:, :n])
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.all(o[:, n:] == -3.0)
    w_ref = _run(torch, pyro, gms[1], rho.astype(np.float32).astype(float),
                 T.astype(np.float32).astype(float), Y.astype(np.float32).astype(float))
    fin = np.isfinite(o[:, :n]).all(axis=0)
    scale = np.abs(w_ref).max(axis=0)
    assert np.all((np.abs(o[:, :n] - w_ref).max(axis=0) <= 1e-3 * scale)[fin])
