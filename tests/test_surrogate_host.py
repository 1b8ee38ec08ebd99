"""Host-side logic of the surrogate: threshold calibration, error summaries,
initialisation and the learning-rate schedule (no GPU needed)."""

import math

import numpy as np

from paper_2503_24286_amd import surrogate as sur


def _brute_force(spread, resid, err, d2, r2, target, gs, gr):
    n = err.shape[0]
    best = None
    for a in gs:
        for b in gr:
            kept = (spread < a) & (resid < b)
            bad = (kept & (err > target)).sum()
            frob = math.sqrt(d2[kept].sum() / r2.sum())
            if bad <= math.floor(1e-3 * n) and frob <= target:
                if best is None or kept.sum() > best[0]:
                    best = (kept.sum(), a, b)
    return best


def _grid(x, q):
    return np.unique(np.concatenate([[0.0], np.quantile(x, np.linspace(0, 1, q)), [np.inf]]))


def test_calibration_matches_brute_force_over_its_grid():
    rng = np.random.default_rng(1)
    n = 4000
    spread = rng.lognormal(-4, 1, n)
    resid = rng.lognormal(-6, 1, n)
    # errors grow with both indicators, plus noise
    err = 0.05 * spread + 2.0 * resid + rng.lognormal(-9, 1, n)
    r2 = rng.uniform(0.5, 2.0, n)
    d2 = (err ** 2) * r2
    for target in (1e-3, 3e-3, 1e-2):
        ts, tr, frac = sur.calibrate(spread, resid, err, d2, r2, target=target, quantiles=24)
        kept = (spread < ts) & (resid < tr)
        assert abs(frac - (1 - kept.mean())) < 1e-12
        assert (kept & (err > target)).sum() <= math.floor(1e-3 * n)
        assert math.sqrt(d2[kept].sum() / r2.sum()) <= target
        best = _brute_force(spread, resid, err, d2, r2, target, _grid(spread, 24), _grid(resid, 24))
        assert best is not None and kept.sum() == best[0]


def test_calibration_falls_back_everywhere_when_nothing_is_accurate():
    rng = np.random.default_rng(2)
    n = 1000
    spread = rng.random(n)
    resid = rng.random(n)
    err = np.full(n, 0.5)
    ts, tr, frac = sur.calibrate(spread, resid, err, err ** 2, np.ones(n), target=1e-3)
    assert frac == 1.0
    assert not ((spread < ts) & (resid < tr)).any()


def test_calibration_keeps_everything_when_all_cells_are_accurate():
    rng = np.random.default_rng(3)
    n = 1000
    err = np.full(n, 1e-5)
    ts, tr, frac = sur.calibrate(rng.random(n), rng.random(n), err, err ** 2, np.ones(n))
    assert frac == 0.0 and ts == math.inf and tr == math.inf


def test_calibration_treats_non_finite_indicators_as_fallback():
    n = 100
    spread = np.full(n, 1e-3)
    spread[:7] = np.nan
    resid = np.full(n, 1e-6)
    err = np.full(n, 1e-6)
    err[:7] = 1.0
    ts, tr, frac = sur.calibrate(spread, resid, err, err ** 2, np.ones(n), target=1e-3)
    assert math.isclose(frac, 0.07)


def test_error_summary_definitions():
    w = np.array([[3.0, 1.0], [4.0, 0.0]])
    ws = np.array([[3.0, 1.1], [4.5, 0.0]])
    s = sur.error_summary(ws, w)
    assert math.isclose(s["max"], 0.1)
    assert math.isclose(s["p50"], 0.1)        # median of {0.1, 0.1}
    assert math.isclose(s["frobenius"], math.sqrt((0.25 + 0.01) / 26.0))


def test_init_member_layout_and_scale():
    H = 128
    w, b = sur.init_member(H, 56, 53, seed=0)
    assert w.dtype == np.float32 and b.dtype == np.float32
    dims = [(64, H), (H, H), (H, H), (H, 64)]
    assert w.size == sum(k * n for k, n in dims) and b.size == sum(n for _, n in dims)
    assert not b.any()
    W1 = w[:64 * H].reshape(64, H)
    assert not W1[56:].any()
    assert abs(W1[:56].std() - math.sqrt(2 / 56)) < 0.02
    W4 = w[-H * 64:].reshape(H, 64)
    assert not W4[:, 53:].any()
    assert abs(W4[:, :53].std() - math.sqrt(1 / H)) < 0.01


def test_learning_rate_schedule():
    assert math.isclose(sur.lr_at(0, 1000, 1e-3, 10), 1e-4)
    assert math.isclose(sur.lr_at(9, 1000, 1e-3, 10), 1e-3)
    assert math.isclose(sur.lr_at(10, 1000, 1e-3, 10), 1e-3)
    assert math.isclose(sur.lr_at(1000, 1000, 1e-3, 10), 1e-5)
    lrs = [sur.lr_at(s, 1000, 1e-3, 10) for s in range(10, 1001)]
    assert all(a >= b for a, b in zip(lrs, lrs[1:]))


def test_bf16_decoding():
    bits = np.array([0x3F80, 0xC000, 0x0000, 0x7F80], dtype=np.uint16)
    assert np.array_equal(sur.bf16_to_float(bits), np.array([1.0, -2.0, 0.0, np.inf], np.float32))
