"""Pins of the surrogate's NumPy reference: BF16 rounding against brute
force, backpropagation against central differences, AdamW against its first-
step closed form, and the target transform round trip."""

import numpy as np

from oracle import mlp


def _brute_bf16(x):
    """Nearest BF16 value by enumerating the two neighbours (ties to even)."""
    f = np.float32(x)
    u = int(np.array(f).view(np.uint32))
    lo = (u >> 16) << 16
    hi = lo + (1 << 16)
    vlo = np.array(lo, dtype=np.uint32).view(np.float32)
    vhi = np.array(hi & 0xFFFFFFFF, dtype=np.uint32).view(np.float32)
    dlo, dhi = abs(float(f) - float(vlo)), abs(float(vhi) - float(f))
    if dlo < dhi or (dlo == dhi and ((lo >> 16) & 1) == 0):
        return float(vlo)
    return float(vhi)


def test_bf16_rounding_matches_brute_force():
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-30, 30, 2000),
                         [1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, -2.5, 0.0, 65504.0]])
    got = mlp.bf16_round(xs)
    for x, g in zip(xs, got):
        assert g == _brute_bf16(x), x
    assert mlp.bf16_round(1.0 + 2**-8) == 1.0           # tie goes to even
    assert mlp.bf16_round(1.0 + 3 * 2**-8) == 1.0 + 2**-6
    assert np.array_equal(mlp.from_bf16_bits(mlp.bf16_bits(got)), got)


def test_backprop_matches_central_differences():
    """In exact arithmetic (no rounding) the backward pass is the gradient of
    the summed squared error over the batch, divided by batch * n_out."""
    rng = np.random.default_rng(1)
    H = 64
    Ws = [rng.standard_normal((k, n)) * 0.2 for k, n in mlp.layer_dims(H)]
    bs = [rng.standard_normal(n) * 0.1 for _, n in mlp.layer_dims(H)]
    B, n_out = 5, 7
    X = rng.standard_normal((B, mlp.FEAT_PAD))
    Zt = rng.standard_normal((B, mlp.OUT_PAD))
    ident = lambda x: np.asarray(x, dtype=float)  # noqa: E731

    def loss(Ws_, bs_):
        _, _, Z = mlp.forward(X, Ws_, bs_, rnd=ident)
        return mlp.mse_grad(Z, Zt, n_out, rnd=ident)[0] / (B * n_out)

    P, Hs, Z = mlp.forward(X, Ws, bs, rnd=ident)
    _, dZ = mlp.mse_grad(Z, Zt, n_out, rnd=ident)
    gW, gb, _ = mlp.backward(X, Ws, P, Hs, dZ, rnd=ident)
    for l in range(4):
        for (i, j) in [(0, 0), (3, 5), (Ws[l].shape[0] - 1, Ws[l].shape[1] - 1), (7, 2)]:
            h = 1e-6
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][i, j] += h
            Wm[l][i, j] -= h
            fd = (loss(Wp, bs) - loss(Wm, bs)) / (2 * h)
            assert abs(fd - gW[l][i, j]) <= 1e-6 * abs(fd) + 1e-9, (l, i, j)
        j = 3
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][j] += 1e-6
        bm[l][j] -= 1e-6
        fd = (loss(Ws, bp) - loss(Ws, bm)) / 2e-6
        assert abs(fd - gb[l][j]) <= 1e-6 * abs(fd) + 1e-9


def test_adamw_first_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2, so the update is
    -lr g/(|g| + eps) after the decay."""
    rng = np.random.default_rng(2)
    w = rng.standard_normal(100)
    g = rng.standard_normal(100)
    lr, wd, eps = 1e-3, 1e-2, 1e-8
    w1, m1, m2 = mlp.adamw(w, g, np.zeros(100), np.zeros(100), lr, 0.9, 0.999, eps, wd, 1)
    np.testing.assert_allclose(w1, w * (1 - lr * wd) - lr * g / (np.abs(g) + eps), rtol=1e-12)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(m2, 0.001 * g * g)


def test_target_transform_round_trip():
    rng = np.random.default_rng(3)
    S, n = 9, 50
    w = rng.standard_normal((S, n)) * 10.0 ** rng.integers(-20, 40, (S, n))
    s = 10.0 ** rng.uniform(-5, 5, S)
    mu = rng.uniform(-2, 2, S)
    sig = rng.uniform(1, 20, S)
    Z = mlp.targets(w, s, mu, sig)
    # relative accuracy for |omega| >> s; absolute ~ s eps (1 + |mu|) below,
    # where the affine normalisation cancels
    back = mlp.inverse_targets(Z, s, mu, sig)
    bound = 1e-12 * (np.abs(w) + s[:, None] * (1 + np.abs(mu[:, None])))
    assert np.all(np.abs(back - w) <= bound)
    assert np.all(Z[:, S:] == 0)
