"""Reactor steps (pyro_reactor_step): the Runge-Kutta and Crank-Nicolson
steps against the oracle's, and the paper's autoignition comparison of the
implicit scheme at a ten times larger step with the explicit one."""

import numpy as np
import pytest

import mechs
from gpu_util import announce, record, states, to_dev, torch_cuda
from oracle import eos, kinetics, reactor, thermo

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib_mechs():
    torch = torch_cuda()
    import paper_2503_24286_amd as pyro
    out = {c: pyro.Mechanism(mechs.config_path(c)) for c in (0, 1)}
    yield torch, pyro, out
    for m in out.values():
        m.close()


def _setup(m, cfg, n, first, frac):
    T, p, Y, rho = states(cfg, n, m.S, first=first)
    e = thermo.mixture_internal_energy(m, T, Y)
    f, _ = reactor.rhs(m, rho, e, Y, T)
    with np.errstate(divide="ignore"):
        tau = np.min(np.where(np.abs(f) > 0, np.maximum(Y, 1e-3) / np.abs(f), np.inf), axis=0)
    return T, Y, rho, e, frac * tau


def _scale(m, rho, T, Y, dt):
    """|Y| plus dt times the summed magnitudes of the source terms' parts."""
    Rf, Rr, phi, q = kinetics.rates_of_progress(m, rho, T, Y)
    mag = np.abs(m.nu) @ ((np.abs(Rf) + np.abs(Rr)) * np.abs(phi))
    return np.abs(Y) + dt * m.W[:, None] * mag / rho


def _gpu_step(torch, pyro, gm, method, rho, e, Y, T, dt, **kw):
    r, ee, y, t, h = to_dev(torch, rho, e, Y, T, dt)
    st = pyro.reactor_step(gm, method, r, ee, y, t, h, **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy(), t.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("cfg,n", [(0, 200), (1, 70)])
def test_rk4_step_matches_oracle(lib_mechs, cfg, n):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    T, Y, rho, e, dt = _setup(m, cfg, n, 40, 0.05)
    announce(f"reactor rk4 cfg{cfg} n={n}")
    Yg, Tg, st = _gpu_step(torch, pyro, gms[cfg], "rk4", rho, e, Y, T, dt)
    Yr, Tr = reactor.rk4_step(m, rho, e, Y, T, dt)
    assert np.all(st > 0)
    eY = np.max(np.abs(Yg - Yr) / _scale(m, rho, T, Y, dt))
    eT = np.max(np.abs(Tg - Tr) / Tr)
    record(f"reactor rk4 cfg{cfg} n={n}", "Y scaled", eY, 1e-12)
    record(f"reactor rk4 cfg{cfg} n={n}", "T relative", eT, 1e-12)
    assert eY <= 1e-12 and eT <= 1e-12


@pytest.mark.parametrize("cfg,n", [(0, 64), (1, 16)])
def test_cn_step_matches_oracle(lib_mechs, cfg, n):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    T, Y, rho, e, dt = _setup(m, cfg, n, 90, 1.0)
    announce(f"reactor cn cfg{cfg} n={n}")
    Yg, Tg, st = _gpu_step(torch, pyro, gms[cfg], "cn", rho, e, Y, T, dt)
    Yr, Tr, st_r = reactor.cn_step(m, rho, e, Y, T, dt)
    assert np.all(st > 0) and np.all(st_r > 0)
    assert np.all(np.abs(st - st_r) <= 1)
    eY = np.max(np.abs(Yg - Yr) / _scale(m, rho, T, Y, dt))
    eT = np.max(np.abs(Tg - Tr) / Tr)
    record(f"reactor cn cfg{cfg} n={n}", "Y scaled", eY, 1e-12)
    record(f"reactor cn cfg{cfg} n={n}", "T relative", eT, 1e-12)
    np.testing.assert_allclose(Yg.sum(axis=0), Y.sum(axis=0), rtol=1e-13)
    assert eY <= 1e-12 and eT <= 1e-12


def test_cn_step_sampled_at_scale(lib_mechs):
    """2^14 config-1 cells, a step of one chemical time scale per cell: the
    cells converge at different updates, so the later updates run on the
    gathered remaining cells (a compaction over 16 workgroups).  Sampled
    cells of every Newton count against the oracle's step of those cells
    (cells are independent: a subset steps as it does in the whole).  Both
    sides iterate to |dY| <= 1e-14: where Newton stops at 1e-12 the step is
    only determined to about 1e-13 scaled (the oracle against itself at
    1e-12 and 1e-15), which would leave the 1e-12 bar little room."""
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    n = 1 << 14
    tol = 1e-14
    T, Y, rho, e, dt = _setup(m, 1, n, 300, 1.0)
    announce(f"reactor cn cfg1 n={n} sampled")
    Yg, Tg, st = _gpu_step(torch, pyro, gms[1], "cn", rho, e, Y, T, dt, tol=tol)
    counts = np.unique(st[st > 0])
    assert np.mean(st > 0) >= 0.99 and len(counts) >= 3
    rng = np.random.default_rng(14)
    idx = np.sort(np.concatenate([rng.choice(np.nonzero(st == c)[0], min(4, int((st == c).sum())),
                                             replace=False) for c in counts]))
    Yr, Tr, st_r = reactor.cn_step(m, rho[idx], e[idx], Y[:, idx], T[idx], dt[idx], tol=tol)
    assert np.all(np.abs(st[idx] - st_r) <= 1)
    eY = np.max(np.abs(Yg[:, idx] - Yr) / _scale(m, rho[idx], T[idx], Y[:, idx], dt[idx]))
    eT = np.max(np.abs(Tg[idx] - Tr) / Tr)
    record(f"reactor cn cfg1 n={n} sampled", "Y scaled", eY, 1e-12)
    record(f"reactor cn cfg1 n={n} sampled", "T relative", eT, 1e-12)
    np.testing.assert_allclose(Yg.sum(axis=0), Y.sum(axis=0), rtol=1e-13)
    assert eY <= 1e-12 and eT <= 1e-12


def test_cn_step_padded_rows(lib_mechs):
    """Species rows of stride ld > n (the Newton updates gather from and
    write back to the padded layout): 40 config-1 cells in rows of 64; the
    padding is left untouched."""
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    n, ld = 40, 64
    T, Y, rho, e, dt = _setup(m, 1, n, 500, 1.0)
    announce(f"reactor cn cfg1 n={n} ld={ld}")
    Yp = torch.full((m.S, ld), 7.0, dtype=torch.float64, device="cuda")
    Yp[:, :n] = torch.from_numpy(Y).cuda()
    r, ee, t, h = to_dev(torch, rho, e, T, dt)
    st = pyro.reactor_step(gms[1], "cn", r, ee, Yp[:, :n], t, h).cpu().numpy()
    Yg, Tg = Yp.cpu().numpy(), t.cpu().numpy()
    Yr, Tr, st_r = reactor.cn_step(m, rho, e, Y, T, dt)
    assert np.all(Yg[:, n:] == 7.0)
    assert np.all(st > 0) and np.all(np.abs(st - st_r) <= 1)
    eY = np.max(np.abs(Yg[:, :n] - Yr) / _scale(m, rho, T, Y, dt))
    eT = np.max(np.abs(Tg - Tr) / Tr)
    record(f"reactor cn cfg1 n={n} ld={ld}", "Y scaled", eY, 1e-12)
    record(f"reactor cn cfg1 n={n} ld={ld}", "T relative", eT, 1e-12)
    assert eY <= 1e-12 and eT <= 1e-12


def test_cn_step_past_64_species(tmp_path):
    """66 species (the solve's one-cell-per-lane form, past the 64 of the
    one-cell-per-wavefront form): 33 isomer pairs A_i <-> B_i and the
    bimolecular exchanges A_i + A_i+1 <-> B_i + B_i+1, constant heat
    capacities, a Crank-Nicolson step of one chemical time scale against the
    oracle's; the cells converge at different updates, so the later updates
    run on the gathered remaining cells."""
    torch = torch_cuda()
    import paper_2503_24286_amd as pyro
    rng = np.random.default_rng(66)
    H, S = 33, 66
    Wh = rng.uniform(0.002, 0.05, H)
    a1 = rng.uniform(2.5, 4.5, S)
    a6 = rng.uniform(-3e4, 3e4, S)
    rx = []
    for i in range(H):
        rx.append(dict(reac=[(i, 1)], prod=[(H + i, 1)],
                       arrh=(np.log(rng.uniform(1e6, 1e8)), rng.uniform(-0.5, 0.5),
                             rng.uniform(1e5, 2e5))))
    for i in range(H - 1):
        rx.append(dict(reac=[(i, 1), (i + 1, 1)], prod=[(H + i, 1), (H + i + 1, 1)],
                       arrh=(np.log(rng.uniform(1e6, 1e8)), rng.uniform(-0.5, 0.5),
                             rng.uniform(1e5, 2e5))))
    path = str(tmp_path / "pairs.pyromech")
    m = mechs.make(path, W=np.concatenate([Wh, Wh]), nasa_low=mechs.constant_cp(S, a1, a6, 10.0),
                   reactions=rx)
    n = 96
    T = rng.uniform(1000.0, 1800.0, n)
    Y = rng.uniform(0.0, 1.0, (S, n)) ** 4
    Y /= Y.sum(axis=0)
    rho = eos.density(m, np.full(n, 101325.0), T, Y)
    e = thermo.mixture_internal_energy(m, T, Y)
    f, _ = reactor.rhs(m, rho, e, Y, T)
    with np.errstate(divide="ignore"):
        dt = np.min(np.where(np.abs(f) > 0, np.maximum(Y, 1e-3) / np.abs(f), np.inf), axis=0)
    gm = pyro.Mechanism(path)
    try:
        announce(f"reactor cn 66 species n={n}")
        Yg, Tg, st = _gpu_step(torch, pyro, gm, "cn", rho, e, Y, T, dt)
    finally:
        gm.close()
    Yr, Tr, st_r = reactor.cn_step(m, rho, e, Y, T, dt)
    assert np.all(st > 0) and np.all(st_r > 0)
    assert np.all(np.abs(st - st_r) <= 1)
    assert len(np.unique(st_r)) > 1
    eY = np.max(np.abs(Yg - Yr) / _scale(m, rho, T, Y, dt))
    eT = np.max(np.abs(Tg - Tr) / Tr)
    record(f"reactor cn 66 species n={n}", "Y scaled", eY, 1e-12)
    record(f"reactor cn 66 species n={n}", "T relative", eT, 1e-12)
    assert eY <= 1e-12 and eT <= 1e-12


def test_autoignition_implicit_at_ten_times_the_step(lib_mechs):
    """The paper's reactor demonstration on the 9-species mechanism: 200
    explicit steps (matching the oracle's trajectory) and 20 Crank-Nicolson
    steps ten times larger reach the same state."""
    torch, pyro, gms = lib_mechs
    gm = gms[0]
    m = mechs.load_config(0)
    n = 4
    T, Y, rho, e, tau = _setup(m, 0, n, 40, 1.0)
    dt = np.full(n, 0.05 * tau.min())
    announce("reactor autoignition rk4 x200 vs cn x20")
    r, ee, h, h10 = to_dev(torch, rho, e, dt, 10 * dt)
    y1, t1 = to_dev(torch, Y, T)
    y2, t2 = to_dev(torch, Y, T)
    for _ in range(200):
        pyro.reactor_step(gm, "rk4", r, ee, y1, t1, h)
    for _ in range(20):
        st = pyro.reactor_step(gm, "cn", r, ee, y2, t2, h10)
    torch.cuda.synchronize()
    Y1, T1, Y2, T2 = (x.cpu().numpy() for x in (y1, t1, y2, t2))
    assert bool((st > 0).all())
    Yr, Tr = Y.copy(), T.copy()
    for _ in range(200):
        Yr, Tr = reactor.rk4_step(m, rho, e, Yr, Tr, dt)
    record("reactor autoignition", "rk4 trajectory T relative vs oracle",
           np.max(np.abs(T1 - Tr) / Tr), 1e-10)
    record("reactor autoignition", "cn (10 dt) vs rk4 (dt) T relative",
           np.max(np.abs(T2 - T1) / T1), 1e-4)
    assert np.max(np.abs(T1 - Tr) / Tr) <= 1e-10
    assert np.max(np.abs(Y1 - Yr)) <= 1e-10
    assert np.max(np.abs(T2 - T1) / T1) <= 1e-4
    assert np.max(np.abs(Y2 - Y1)) <= 1e-4
    assert np.max(np.abs(T1 - T)) > 1.0          # the mixture did react


def test_reactor_errors(lib_mechs):
    from paper_2503_24286_amd import _lib
    torch, pyro, gms = lib_mechs
    lib = _lib.lib()
    gm = gms[0]
    one = torch.ones(8, dtype=torch.float64, device="cuda")
    p = one.data_ptr()
    assert lib.pyro_reactor_workspace_size(gm.handle, 4, 4, 7) == 0
    assert lib.pyro_reactor_step(gm.handle, 7, 4, 4, p, p, p, p, None, 1e-9, 1e-12, 5, p, p,
                                 1 << 20, None) == _lib.PYRO_E_ARG
    # a workspace that is too small
    assert lib.pyro_reactor_step(gm.handle, 0, 4, 4, p, p, p, p, None, 1e-9, 1e-12, 5, p, p,
                                 16, None) == _lib.PYRO_E_ARG
    assert lib.pyro_reactor_step(gm.handle, 1, 4, 4, p, p, p, p, None, 1e-9, 1e-12, 0, p, p,
                                 1 << 20, None) == _lib.PYRO_E_ARG
