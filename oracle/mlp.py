"""Reference of the learned surrogate (not part of the paper's method): the
BF16 multilayer perceptron, its gradients, AdamW, and the feature and target
transforms, in plain NumPy FP64 with BF16 rounding applied where the GPU
stores BF16 values.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Network: 64 -> H -> H -> H -> 64 with SiLU after the hidden layers; weights
W_l are [in][out] (row-major, input index first).  The backward pass of the
mean squared error rounds the output cotangent and every hidden-layer
cotangent to BF16, as the GPU stores them.
"""

import numpy as np

FEAT_PAD = 64
OUT_PAD = 64


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def bf16_bits(x):
    """BF16 bit patterns (uint16) of the rounded values."""
    f = bf16_round(x).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b):
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def silu(x):
    return x / (1.0 + np.exp(-x))


def dsilu(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def layer_dims(hidden):
    return [(FEAT_PAD, hidden), (hidden, hidden), (hidden, hidden), (hidden, OUT_PAD)]


def unpack(hidden, w_flat, b_flat):
    """Split one member's packed parameters into per-layer arrays."""
    Ws, bs = [], []
    ow = ob = 0
    for k, n in layer_dims(hidden):
        Ws.append(np.asarray(w_flat[ow:ow + k * n], dtype=np.float64).reshape(k, n))
        bs.append(np.asarray(b_flat[ob:ob + n], dtype=np.float64))
        ow += k * n
        ob += n
    return Ws, bs


def forward(X, Ws, bs, rnd=bf16_round):
    """Returns (P, H, Z): BF16-rounded pre-activations and activations of the
    hidden layers and the FP64 output.  X, Ws hold BF16-representable values.
    ``rnd`` is the rounding applied where the GPU stores BF16 (identity for
    an exact-arithmetic reference)."""
    P, H = [], []
    a = X
    for l in range(3):
        p = a @ Ws[l] + bs[l]
        P.append(rnd(p))
        h = rnd(silu(p))
        H.append(h)
        a = h
    Z = a @ Ws[3] + bs[3]
    return P, H, Z


def mse_grad(Z, Zt, n_out, rnd=bf16_round):
    """Sum of squared errors and the BF16 cotangent of their mean over
    batch x n_out."""
    B = Z.shape[0]
    d = np.zeros_like(Z)
    d[:, :n_out] = Z[:, :n_out] - Zt[:, :n_out]
    loss = (d[:, :n_out] ** 2).sum()
    return loss, rnd(2.0 * d / (B * n_out))


def backward(X, Ws, P, H, dZ, rnd=bf16_round):
    """Gradients (gW, gb) per layer and the hidden cotangents dP (BF16)."""
    gW = [None] * 4
    gb = [None] * 4
    dPs = [None] * 3
    dY = dZ
    for l in range(3, -1, -1):
        a = X if l == 0 else H[l - 1]
        gW[l] = a.T @ dY
        gb[l] = dY.sum(axis=0)
        if l == 0:
            break
        dP = rnd((dY @ Ws[l].T) * dsilu(P[l - 1]))
        dPs[l - 1] = dP
        dY = dP
    return gW, gb, dPs


def adamw(w, g, m1, m2, lr, b1, b2, eps, wd, step):
    """One AdamW step (decoupled weight decay); returns new (w, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    w = w * (1 - lr * wd) - lr * mh / (np.sqrt(vh) + eps)
    return w, m1, m2


def features(mech, rho, T, Y, shift, scale):
    """Feature rows [n][64] before BF16 rounding: T/1000, log10 p (p from the
    equation of state), ln(max(Y_k, 0) + 1e-12), shifted and scaled; then a
    constant 1 and zeros."""
    from . import eos
    n = T.shape[0]
    S = mech.S
    X = np.zeros((n, FEAT_PAD))
    p = eos.pressure(mech, rho, T, Y)
    X[:, 0] = (T * 1e-3 - shift[0]) * scale[0]
    X[:, 1] = (np.log10(p) - shift[1]) * scale[1]
    for k in range(S):
        X[:, 2 + k] = (np.log(np.maximum(Y[k], 0.0) + 1e-12) - shift[2 + k]) * scale[2 + k]
    X[:, 2 + S] = 1.0
    return X


def targets(wdot, s, mu, sigma):
    """z_k = (asinh(omega_k / s_k) - mu_k) / sigma_k, rows [n][64]."""
    S, n = wdot.shape
    Z = np.zeros((n, OUT_PAD))
    Z[:, :S] = ((np.arcsinh(wdot / s[:, None]) - mu[:, None]) / sigma[:, None]).T
    return Z


def inverse_targets(Z, s, mu, sigma):
    """omega_k = s_k sinh(mu_k + sigma_k z_k), shape (S, n)."""
    S = s.shape[0]
    return (s[:, None] * np.sinh(mu[:, None] + sigma[:, None] * Z[:, :S].T))
