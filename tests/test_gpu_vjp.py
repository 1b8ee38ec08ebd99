"""The HIP reverse-mode kernel (pyro_production_rates_vjp) against the
oracle's complex-step gradients, central differences of the HIP forward
kernel, conservation invariants and the autograd wrapper."""

import numpy as np
import pytest

import mechs
from gpu_util import announce, record, states, to_dev, torch_cuda
from oracle import gradients
from parity import vjp_scales
from pyro_synth.states import draw_cotangent

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def lib_mechs():
    torch = torch_cuda()
    import paper_2503_24286_amd as pyro
    out = {c: pyro.Mechanism(mechs.config_path(c)) for c in (0, 1)}
    yield torch, pyro, out
    for m in out.values():
        m.close()


def _gpu_vjp(torch, pyro, gm, rho, T, Y, wbar, params=None):
    r, t, y, wb = to_dev(torch, rho, T, Y, wbar)
    p = None if params is None else to_dev(torch, params.reshape(-1))[0]
    Yb, Tb, pb = pyro.production_rates_vjp(gm, r, t, y, wb, params=p)
    torch.cuda.synchronize()
    return Yb.cpu().numpy(), Tb.cpu().numpy(), pb.cpu().numpy()


def _check_vs_oracle(m, rho, T, Y, wbar, Yb, Tb, pb, tol=TOL, case="vjp"):
    Yr, Tr, pr = gradients.vjp(m, rho, T, Y, wbar)
    sY, sT, sP = vjp_scales(m, rho, T, Y, wbar)
    assert np.array_equal(Yb[sY == 0], Yr[sY == 0])
    eY = np.where(sY > 0, np.abs(Yb - Yr) / np.where(sY > 0, sY, 1.0), 0.0)
    eT = np.abs(Tb - Tr) / np.maximum(sT, 1e-300)
    eP = np.abs(pb - pr) / np.maximum(sP, 1e-300)
    record(case, "Ybar scaled", eY.max(), tol)
    record(case, "Tbar scaled", eT.max(), tol)
    record(case, "params_bar scaled", eP.max(), tol)
    assert eY.max() <= tol, f"Ybar error {eY.max():.3e} at {np.unravel_index(eY.argmax(), eY.shape)}"
    assert eT.max() <= tol, f"Tbar error {eT.max():.3e}"
    assert eP.max() <= tol, f"params_bar error {eP.max():.3e} at {np.unravel_index(eP.argmax(), eP.shape)}"
    assert np.all(Yb[Y <= 0] == 0.0)


@pytest.mark.parametrize("cfg,n", [(0, 130), (1, 70)])
def test_vjp_matches_complex_step_oracle(lib_mechs, cfg, n):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    T, p, Y, rho = states(cfg, n, m.S, first=11)
    wbar = draw_cotangent(2, n, m.S)
    announce(f"vjp cfg{cfg} n={n}")
    Yb, Tb, pb = _gpu_vjp(torch, pyro, gms[cfg], rho, T, Y, wbar)
    _check_vs_oracle(m, rho, T, Y, wbar, Yb, Tb, pb, case=f"vjp cfg{cfg} n={n}")


def test_vjp_degenerate_states(lib_mechs):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    n = 70
    T, p, Y, rho = states(1, n, m.S, first=700)
    Y[4, :10] = 0.0
    Y[9, 10:20] = -1e-4
    T[20:25] = m.T_mid[0]
    wbar = draw_cotangent(2, n, m.S, seed=5)
    announce("vjp degenerate states")
    Yb, Tb, pb = _gpu_vjp(torch, pyro, gms[1], rho, T, Y, wbar)
    _check_vs_oracle(m, rho, T, Y, wbar, Yb, Tb, pb, case="vjp degenerate states")


def test_vjp_conserved_combinations_have_zero_gradient(lib_mechs):
    """sum_k W_k omega_k = 0 for every state, so its gradient vanishes."""
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    n = 200
    T, p, Y, rho = states(1, n, m.S, first=300)
    announce("vjp invariants")
    for wbar in (np.repeat(m.W[:, None], n, axis=1),
                 np.repeat(m.composition[2][:, None].astype(float), n, axis=1)):
        Yb, Tb, pb = _gpu_vjp(torch, pyro, gms[1], rho, T, Y, wbar)
        sY, sT, sP = vjp_scales(m, rho, T, Y, wbar, abs_qbar=True)
        assert np.all(Yb[sY == 0] == 0.0)
        eY = np.max(np.abs(Yb) / np.where(sY > 0, sY, 1.0))
        eT = np.max(np.abs(Tb) / sT)
        eP = np.max(np.abs(pb) / np.maximum(sP, 1e-300))
        for q, v in (("Ybar", eY), ("Tbar", eT), ("params_bar", eP)):
            record("vjp conserved combination", f"{q} scaled (exact value 0)", v, TOL)
        assert eY <= TOL and eT <= TOL and eP <= TOL


def test_vjp_matches_central_differences_of_the_forward_kernel(lib_mechs):
    """64 random cells of the 53-species workload; h = 1e-6 relative (floors
    ln A 1, b 1, Ea 1e4 J/mol, Y 1e-20); |fd - g| <= 1e-5 |g| + rounding floor
    30 eps |L|_abs / h."""
    torch, pyro, gms = lib_mechs
    gm = gms[1]
    m = mechs.load_config(1)
    n = 64
    rng = np.random.default_rng(64)
    first = int(rng.integers(0, (1 << 20) - n))
    T, p, Y, rho = states(2, n, m.S, first=first)
    wbar = draw_cotangent(2, n, m.S, seed=77)
    announce("vjp vs central differences")
    Yb, Tb, pb = _gpu_vjp(torch, pyro, gm, rho, T, Y, wbar)
    r_d, w_d = to_dev(torch, rho, wbar)
    P = m.parameters()

    def cellL(Tc, Yc, Pc=None):
        t, y = to_dev(torch, Tc, Yc)
        pp = None if Pc is None else to_dev(torch, Pc.reshape(-1))[0]
        w = pyro.production_rates(gm, r_d, t, y, params=pp)
        return (w_d * w).sum(dim=0).cpu().numpy(), (w_d * w).abs().sum(dim=0).cpu().numpy()

    eps = np.finfo(float).eps
    checked = resolved = 0
    L0, Labs = cellL(T, Y)
    for k in range(m.S):
        h = 1e-6 * np.maximum(Y[k], 1e-20)
        Yp, Ym = Y.copy(), Y.copy()
        Yp[k] += h
        Ym[k] -= h
        fd = (cellL(T, Yp)[0] - cellL(T, Ym)[0]) / (2 * h)
        floor = 30 * eps * Labs / h
        ok = (Y[k] > 2 * h)                      # stay on one side of max(Y, 0)
        assert np.all((np.abs(fd - Yb[k]) <= 1e-5 * np.abs(Yb[k]) + floor)[ok])
        checked += ok.sum()
        resolved += (ok & (np.abs(Yb[k]) > 1e3 * floor)).sum()
    h = 1e-6 * T
    fd = (cellL(T + h, Y)[0] - cellL(T - h, Y)[0]) / (2 * h)
    floor = 30 * eps * Labs / h
    assert np.all(np.abs(fd - Tb) <= 1e-5 * np.abs(Tb) + floor)
    checked += n
    resolved += (np.abs(Tb) > 1e3 * floor).sum()
    floors = (1.0, 1.0, 1e4)
    rows = list(range(0, m.R, 7)) + list(range(m.R, m.R + m.n_falloff))
    for j in rows:
        for c in range(3):
            hh = 1e-6 * max(abs(P[j, c]), floors[c])
            Pp, Pm = P.copy(), P.copy()
            Pp[j, c] += hh
            Pm[j, c] -= hh
            fd = (cellL(T, Y, Pp)[0].sum() - cellL(T, Y, Pm)[0].sum()) / (2 * hh)
            floor = 30 * eps * Labs.sum() / hh
            assert abs(fd - pb[j, c]) <= 1e-5 * abs(pb[j, c]) + floor, (j, c, fd, pb[j, c])
            checked += 1
            resolved += abs(pb[j, c]) > 1e3 * floor
    # the synthetic rates span ~60 decades, so most single entries sit below
    # the differences' rounding floor; hundreds are still resolved sharply
    announce(f"  resolved {resolved}/{checked}")
    assert resolved >= 300 and resolved >= 0.1 * checked


def test_vjp_is_deterministic_and_linear(lib_mechs):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    n = 5000
    T, p, Y, rho = states(1, n, m.S, first=900)
    w1 = draw_cotangent(2, n, m.S, seed=1)
    w2 = draw_cotangent(2, n, m.S, seed=2)
    announce("vjp determinism and linearity")
    a = _gpu_vjp(torch, pyro, gms[1], rho, T, Y, w1)
    b = _gpu_vjp(torch, pyro, gms[1], rho, T, Y, w1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    c = _gpu_vjp(torch, pyro, gms[1], rho, T, Y, w2)
    d = _gpu_vjp(torch, pyro, gms[1], rho, T, Y, w1 + w2)
    sP = vjp_scales(m, rho, T, Y, np.abs(w1) + np.abs(w2))[2]
    assert np.max(np.abs(d[2] - a[2] - c[2]) / np.maximum(sP, 1e-300)) <= 1e-12


def test_autograd_function(lib_mechs):
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(0)
    n = 300
    T, p, Y, rho = states(0, n, m.S)
    wbar = draw_cotangent(0, n, m.S)
    announce("autograd")
    r, t, y, wb = to_dev(torch, rho, T, Y, wbar)
    params = torch.from_numpy(m.parameters()).cuda().requires_grad_(True)
    t.requires_grad_(True)
    y.requires_grad_(True)
    w = pyro.production_rates_autograd(gms[0], r, t, y, params)
    (w * wb).sum().backward()
    Yb, Tb, pb = _gpu_vjp(torch, pyro, gms[0], rho, T, Y, wbar)
    assert np.array_equal(y.grad.cpu().numpy(), Yb)
    assert np.array_equal(t.grad.cpu().numpy(), Tb)
    assert np.array_equal(params.grad.cpu().numpy(), pb)


def test_vjp_zero_cells_zeroes_parameter_gradients(lib_mechs):
    torch, pyro, gms = lib_mechs
    gm = gms[1]
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    Z = torch.empty((gm.n_species, 0), dtype=torch.float64, device="cuda")
    pb = torch.full((gm.n_params, 3), 7.0, dtype=torch.float64, device="cuda")
    pyro.production_rates_vjp(gm, e, e, Z, Z, params_bar=pb)
    torch.cuda.synchronize()
    assert bool((pb == 0).all())


def test_vjp_full_size(lib_mechs):
    """2^20 cells (the differentiation workload) in the launch configuration
    of a full call (one persistent workgroup per compute unit, then the
    workgroup-order reduction of the parameter sums).  The cotangent is zero
    except on 2048 cells spread over the whole range, so the parameter
    gradients of the full launch are sums over those cells only and can be
    compared with the oracle's; every other cell's Ybar and Tbar must be
    exactly zero.  Additivity over a split of the cells is checked too."""
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(1)
    n = 1 << 20
    T, p, Y, rho = states(2, n, m.S)
    wbar = draw_cotangent(2, n, m.S)
    rng = np.random.default_rng(2048)
    idx = np.unique(np.concatenate([[0, 1, 63, 64, n // 2, n - 2, n - 1],
                                    rng.choice(n, 2048 - 7, replace=False)]))
    keep = np.zeros(n, bool)
    keep[idx] = True
    wbar[:, ~keep] = 0.0
    announce(f"vjp full size n={n}, {len(idx)} cells with a nonzero cotangent")
    r, t, y, wb = to_dev(torch, rho, T, Y, wbar)
    Yb, Tb, pb = pyro.production_rates_vjp(gms[1], r, t, y, wb)
    h = n // 2 + 37
    _, _, p1 = pyro.production_rates_vjp(gms[1], r[:h], t[:h], y[:, :h], wb[:, :h])
    _, _, p2 = pyro.production_rates_vjp(gms[1], r[h:], t[h:], y[:, h:].contiguous(),
                                         wb[:, h:].contiguous())
    torch.cuda.synchronize()
    Yb_all = Yb.cpu().numpy()
    Tb_all = Tb.cpu().numpy()
    pb = pb.cpu().numpy()
    assert np.all(Yb_all[:, ~keep] == 0.0) and np.all(Tb_all[~keep] == 0.0)
    _check_vs_oracle(m, rho[idx], T[idx], Y[:, idx], wbar[:, idx], Yb_all[:, idx],
                     Tb_all[idx], pb, case=f"vjp full launch n={n} ({len(idx)} cells)")
    sP = vjp_scales(m, rho[idx], T[idx], Y[:, idx], wbar[:, idx])[2]
    eadd = np.max(np.abs(p1.cpu().numpy() + p2.cpu().numpy() - pb) / np.maximum(sP, 1e-300))
    record(f"vjp full launch n={n}", "params_bar additivity over a split", eadd, TOL)
    assert eadd <= TOL


@pytest.mark.parametrize("cfg,n", [(0, 200), (1, 1000 + 29)])
def test_vjp_also_returns_the_production_rates(lib_mechs, cfg, n):
    """The optional omega output of the reverse sweep passes the forward
    kernel's parity bar against the oracle, and requesting it leaves every
    gradient bitwise unchanged."""
    from parity import assert_wdot_parity
    torch, pyro, gms = lib_mechs
    m = mechs.load_config(cfg)
    T, p, Y, rho = states(2 if cfg == 1 else 0, n, m.S, first=777)
    wbar = draw_cotangent(2, n, m.S)
    ld = n + 3
    announce(f"vjp with omega cfg{cfg} n={n}")
    r, t, wb = to_dev(torch, rho, T, wbar)
    y = torch.zeros((m.S, ld), dtype=torch.float64, device="cuda")[:, :n]
    y.copy_(torch.from_numpy(Y))
    wbl = torch.zeros((m.S, ld), dtype=torch.float64, device="cuda")[:, :n]
    wbl.copy_(wb)
    w = torch.full((m.S, ld), 7.0, dtype=torch.float64, device="cuda")[:, :n]
    Yb1, Tb1, pb1 = pyro.production_rates_vjp(gms[cfg], r, t, y, wbl, wdot=w)
    Yb0, Tb0, pb0 = pyro.production_rates_vjp(gms[cfg], r, t, y, wbl)
    torch.cuda.synchronize()
    assert_wdot_parity(m, rho, T, Y, w.cpu().numpy())
    for a, b in ((Yb1, Yb0), (Tb1, Tb0), (pb1, pb0)):
        assert torch.equal(a, b)
    # padding columns of the strided output are untouched
    full = w.as_strided((m.S, ld), (ld, 1)).cpu().numpy()
    assert np.all(full[:, n:] == 7.0)
