"""Learned surrogate of the net production rates.

An ensemble of BF16 multilayer perceptrons maps per-cell features to the
transformed rates z_k = (asinh(omega_k / s_k) - mu_k) / sigma_k.  Everything
that touches cell data runs in libpyro: the labels come from the exact
production-rate kernel, the features and targets from their kernels, and each
training step is the library's forward GEMMs, MSE, backward GEMMs and AdamW.
The host only draws the seeded states, computes normalisation statistics on a
sample, schedules the steps and picks the fallback thresholds.

Evaluation (``Surrogate.eval``) is one ``pyro_surrogate_eval`` call: a fused
kernel computes the features, every member's network, the ensemble mean, the
inverse transform and the two error indicators (ensemble spread of omega and
element residual), then the exact kernel runs on every cell whose indicators
are not below the thresholds.
"""

import ctypes
import math
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import _lib, api
from ._lib import check, lib

FEAT_PAD = 64
OUT_PAD = 64
INIT_SEED = 4100          # member e is initialised and shuffled from INIT_SEED + e


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def param_counts(hidden):
    nw, nb = ctypes.c_int64(), ctypes.c_int64()
    if lib().pyro_mlp_param_counts(int(hidden), ctypes.byref(nw), ctypes.byref(nb)) == 0:
        raise ValueError("hidden width must be a multiple of 64 in [64, 4096]")
    return nw.value, nb.value


def layer_dims(hidden):
    return [(FEAT_PAD, hidden), (hidden, hidden), (hidden, hidden), (hidden, OUT_PAD)]


def init_member(hidden, n_in, n_out, seed):
    """He-normal hidden layers, variance-1/fan-in output layer, zero biases.
    Rows of W1 beyond the ``n_in`` used features and columns of W4 beyond
    the ``n_out`` outputs are zero."""
    rng = np.random.default_rng(seed)
    ws, bs = [], []
    for l, (k, n) in enumerate(layer_dims(hidden)):
        fan_in = n_in if l == 0 else k
        gain = 1.0 if l == 3 else 2.0
        w = rng.standard_normal((k, n)) * math.sqrt(gain / fan_in)
        if l == 0:
            w[n_in:, :] = 0.0
        if l == 3:
            w[:, n_out:] = 0.0
        ws.append(w.astype(np.float32).ravel())
        bs.append(np.zeros(n, dtype=np.float32))
    return np.concatenate(ws), np.concatenate(bs)


# ---------------------------------------------------------------------------
# Data: seeded states labelled by the exact kernel


def draw_chunks(cfg, n, S, seed, chunk=1 << 20, threads=16):
    """Yields (first, T, p, Y) host chunks of the seeded states, drawn in
    parallel threads (the generator's chunks are independent)."""
    from pyro_synth.states import draw_states
    starts = list(range(0, n, chunk))
    with ThreadPoolExecutor(max(1, threads)) as ex:
        futs = [ex.submit(draw_states, cfg, min(chunk, n - a), S, seed, a) for a in starts]
        for a, f in zip(starts, futs):
            T, p, Y = f.result()
            yield a, T, p, Y


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.cuda() if dtype is None else t.to(dtype).cuda()


def label(mech, T, p, Y):
    """rho from the equation of state and omega from the exact kernel, on
    device tensors."""
    rho = api.density(mech, p, T, Y)
    w = api.production_rates(mech, rho, T, Y)
    return rho, w


class Normalisation:
    """Feature shift/scale (FP32, 64) and target s, mu, sigma (FP64, S)."""

    def __init__(self, feat_shift, feat_scale, target_scale, target_mean, target_std):
        self.feat_shift = np.asarray(feat_shift, dtype=np.float32)
        self.feat_scale = np.asarray(feat_scale, dtype=np.float32)
        self.target_scale = np.asarray(target_scale, dtype=np.float64)
        self.target_mean = np.asarray(target_mean, dtype=np.float64)
        self.target_std = np.asarray(target_std, dtype=np.float64)

    def device(self):
        return (_dev(self.feat_shift), _dev(self.feat_scale), _dev(self.target_scale),
                _dev(self.target_mean), _dev(self.target_std))


def features(mech, rho, T, Y, shift, scale, out=None):
    S, n = Y.shape
    ld = Y.stride(0) if S > 1 else n
    if out is None:
        out = torch.empty((n, FEAT_PAD), dtype=torch.int16, device=Y.device)
    check(lib().pyro_surrogate_features(mech.handle, n, ld, _p(rho), _p(T), _p(Y), _p(shift),
                                        _p(scale), _p(out), _stream()))
    return out


def targets(mech, w, s, mu, sig, out=None):
    S, n = w.shape
    ld = w.stride(0) if S > 1 else n
    if out is None:
        out = torch.empty((n, OUT_PAD), dtype=torch.float32, device=w.device)
    check(lib().pyro_surrogate_targets(mech.handle, n, ld, _p(w), _p(s), _p(mu), _p(sig),
                                       _p(out), _stream()))
    return out


def bf16_to_float(bits):
    """Host decoding of BF16 bit patterns (int16/uint16 numpy) to float32."""
    u = np.asarray(bits).astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32)


def fit_normalisation(mech, rho, T, Y, w):
    """Statistics of a sample of labelled states (device tensors): feature
    mean and standard deviation, s_k = median |omega_k| (1 where it is 0),
    and the mean and standard deviation of asinh(omega_k / s_k)."""
    S = mech.n_species
    zeros = torch.zeros(FEAT_PAD, dtype=torch.float32, device=Y.device)
    ones = torch.ones(FEAT_PAD, dtype=torch.float32, device=Y.device)
    raw = bf16_to_float(features(mech, rho, T, Y, zeros, ones).cpu().numpy()).astype(np.float64)
    shift = np.zeros(FEAT_PAD, dtype=np.float32)
    scale = np.ones(FEAT_PAD, dtype=np.float32)
    used = S + 2
    mu = raw[:, :used].mean(axis=0)
    sd = raw[:, :used].std(axis=0)
    shift[:used] = mu
    scale[:used] = np.where(sd > 0, 1.0 / np.where(sd > 0, sd, 1.0), 1.0)
    wh = w.cpu().numpy()
    s = np.median(np.abs(wh), axis=1)
    s = np.where(s > 0, s, 1.0)
    a = np.arcsinh(wh / s[:, None])
    tmu = a.mean(axis=1)
    tsd = a.std(axis=1)
    tsd = np.where(tsd > 0, tsd, 1.0)
    return Normalisation(shift, scale, s, tmu, tsd)


class Dataset:
    """Features X [N][64] (BF16 bits in int16) and targets Zt [N][64] (FP32)
    of N seeded states, resident on the device."""

    def __init__(self, X, Zt, n_out):
        self.X = X
        self.Zt = Zt
        self.n = X.shape[0]
        self.n_out = n_out


def build_dataset(mech, n, seed, norm=None, cfg=4, sample=1 << 20, threads=16, log=None):
    """Draws n states (workload ``cfg``, generator seed ``seed``), labels
    them with the exact kernel and converts them to features and targets.
    Without ``norm``, the statistics are fitted on the first ``sample``
    states.  Returns (Dataset, Normalisation)."""
    S = mech.n_species
    X = torch.empty((n, FEAT_PAD), dtype=torch.int16, device="cuda")
    Zt = torch.empty((n, OUT_PAD), dtype=torch.float32, device="cuda")
    dev_norm = None
    t0 = time.time()
    for a, T, p, Y in draw_chunks(cfg, n, S, seed, chunk=min(sample, n), threads=threads):
        Td, pd, Yd = _dev(T), _dev(p), _dev(Y)
        rho, w = label(mech, Td, pd, Yd)
        if norm is None:
            norm = fit_normalisation(mech, rho, Td, Yd, w)
        if dev_norm is None:
            dev_norm = norm.device()
        fs, fc, ts, tm, tsd = dev_norm
        m = Td.shape[0]
        features(mech, rho, Td, Yd, fs, fc, out=X[a:a + m])
        targets(mech, w, ts, tm, tsd, out=Zt[a:a + m])
        if log:
            log(f"dataset: {a + m}/{n} states labelled ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return Dataset(X, Zt, S), norm


# ---------------------------------------------------------------------------
# Training


class Trainer:
    """One member's training state: FP32 master weights and biases, their
    BF16 copy, AdamW moments, and the step buffers for a fixed batch."""

    def __init__(self, hidden, batch, w0, b0, splits=None):
        self.hidden = hidden
        self.batch = batch
        self.nw, self.nb = param_counts(hidden)
        f32 = dict(dtype=torch.float32, device="cuda")
        self.w = _dev(w0)
        self.b = _dev(b0)
        self.w16 = torch.empty(self.nw, dtype=torch.int16, device="cuda")
        check(lib().pyro_to_bf16(self.nw, _p(self.w), _p(self.w16), _stream()))
        self.mw = torch.zeros(self.nw, **f32)
        self.vw = torch.zeros(self.nw, **f32)
        self.mb = torch.zeros(self.nb, **f32)
        self.vb = torch.zeros(self.nb, **f32)
        self.gw = torch.empty(self.nw, **f32)
        self.gb = torch.empty(self.nb, **f32)
        H = hidden
        self.acts = torch.empty(6 * batch * H, dtype=torch.int16, device="cuda")
        self.Z = torch.empty((batch, OUT_PAD), **f32)
        self.dZ = torch.empty((batch, OUT_PAD), dtype=torch.int16, device="cuda")
        self.work = torch.empty(2 * batch * H, dtype=torch.int16, device="cuda")
        if splits is None:
            splits = max(1, min(64, batch // 256))
        self.splits = splits
        self.split_work = torch.empty(splits * H * H, **f32)
        self.n_partials = lib().pyro_mlp_loss_partials(batch)
        self.t = 0

    def step(self, X, Zt, n_out, lr, loss_out, beta1=0.9, beta2=0.999, eps=1e-8,
             weight_decay=0.0):
        """One AdamW step on the batch X [B][64], Zt [B][64]; the per-block
        squared-error partials go to loss_out."""
        s = _stream()
        L = lib()
        B, H = self.batch, self.hidden
        check(L.pyro_mlp_forward(H, B, _p(X), _p(self.w16), _p(self.b), _p(self.acts),
                                 _p(self.Z), s))
        check(L.pyro_mlp_mse(B, n_out, _p(self.Z), _p(Zt), _p(self.dZ), _p(loss_out), s))
        check(L.pyro_mlp_backward(H, B, _p(X), _p(self.w16), _p(self.acts), _p(self.dZ),
                                  _p(self.gw), _p(self.gb), _p(self.work), _p(self.split_work),
                                  self.splits, s))
        self.t += 1
        check(L.pyro_adamw_step(self.nw, _p(self.w), _p(self.w16), _p(self.gw), _p(self.mw),
                                _p(self.vw), lr, beta1, beta2, eps, weight_decay, self.t, s))
        check(L.pyro_adamw_step(self.nb, _p(self.b), None, _p(self.gb), _p(self.mb),
                                _p(self.vb), lr, beta1, beta2, eps, 0.0, self.t, s))

    def forward(self, X, Z=None):
        """Outputs Z [n][64] (FP32) of the current weights on features X."""
        n = X.shape[0]
        if Z is None:
            Z = torch.empty((n, OUT_PAD), dtype=torch.float32, device="cuda")
        acts = torch.empty(6 * n * self.hidden, dtype=torch.int16, device="cuda")
        check(lib().pyro_mlp_forward(self.hidden, n, _p(X), _p(self.w16), _p(self.b), _p(acts),
                                     _p(Z), _stream()))
        return Z


def lr_at(step, total, lr_max, warmup):
    """Linear warm-up, then cosine decay to 1% of the peak."""
    if step < warmup:
        return lr_max * (step + 1) / warmup
    u = (step - warmup) / max(1, total - warmup)
    return lr_max * (0.01 + 0.99 * 0.5 * (1.0 + math.cos(math.pi * u)))


def train_member(data, hidden, seed, epochs, batch, lr=2e-3, weight_decay=1e-5,
                 warmup=200, log=None):
    """Trains one member on the device dataset; batches are contiguous
    ranges of the (independent, identically drawn) states, visited in a
    seeded random order each epoch.  Returns (Trainer, per-epoch mean
    squared error)."""
    S = data.n_out
    w0, b0 = init_member(hidden, S + 3, S, seed)
    tr = Trainer(hidden, batch, w0, b0)
    nbat = data.n // batch
    if nbat < 1:
        raise ValueError("dataset smaller than one batch")
    total = epochs * nbat
    rng = np.random.default_rng(seed)
    partials = torch.empty((nbat, tr.n_partials), dtype=torch.float32, device="cuda")
    history = []
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        for j, bi in enumerate(rng.permutation(nbat)):
            a = int(bi) * batch
            tr.step(data.X[a:a + batch], data.Zt[a:a + batch], S,
                    lr_at(step, total, lr, warmup), partials[j], weight_decay=weight_decay)
            step += 1
        mse = float(partials.double().sum().item()) / (nbat * batch * S)
        history.append(mse)
        if log:
            log(f"member seed {seed}: epoch {ep + 1}/{epochs} mse {mse:.4e} "
                f"({time.time() - t0:.1f} s)")
    return tr, history


# ---------------------------------------------------------------------------
# Evaluation


class Surrogate:
    """A trained ensemble with its normalisation and fallback thresholds."""

    def __init__(self, hidden, weights, biases, norm, thr_spread=math.inf, thr_resid=math.inf):
        self.hidden = int(hidden)
        self.nw, self.nb = param_counts(hidden)
        self.weights = np.asarray(weights, dtype=np.uint16).reshape(-1, self.nw)
        self.biases = np.asarray(biases, dtype=np.float32).reshape(-1, self.nb)
        self.members = self.weights.shape[0]
        self.norm = norm
        self.thr_spread = float(thr_spread)
        self.thr_resid = float(thr_resid)
        self._dev = None
        self._ws = None

    @classmethod
    def from_trainers(cls, trainers, norm, **kw):
        w = np.stack([t.w16.cpu().numpy().view(np.uint16) for t in trainers])
        b = np.stack([t.b.cpu().numpy() for t in trainers])
        return cls(trainers[0].hidden, w, b, norm, **kw)

    def save(self, path):
        n = self.norm
        np.savez(path, hidden=self.hidden, weights=self.weights, biases=self.biases,
                 feat_shift=n.feat_shift, feat_scale=n.feat_scale, target_scale=n.target_scale,
                 target_mean=n.target_mean, target_std=n.target_std,
                 thr=np.array([self.thr_spread, self.thr_resid]))

    @classmethod
    def load(cls, path):
        z = np.load(path)
        norm = Normalisation(z["feat_shift"], z["feat_scale"], z["target_scale"],
                             z["target_mean"], z["target_std"])
        return cls(int(z["hidden"]), z["weights"], z["biases"], norm, *z["thr"])

    def _device(self):
        if self._dev is None:
            w = _dev(self.weights.view(np.int16).ravel())
            b = _dev(self.biases.ravel())
            fs, fc, ts, tm, tsd = self.norm.device()
            st = _lib.Surrogate(self.members, self.hidden, w.data_ptr(), b.data_ptr(),
                                fs.data_ptr(), fc.data_ptr(), ts.data_ptr(), tm.data_ptr(),
                                tsd.data_ptr())
            self._dev = (st, (w, b, fs, fc, ts, tm, tsd))
        return self._dev[0]

    def workspace(self, mech, n):
        need = lib().pyro_surrogate_workspace_size(mech.handle, n, self.hidden, self.members)
        if need == 0 and n > 0:
            raise ValueError("invalid surrogate workspace request")
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
        return self._ws, need

    def outputs(self, mech, rho, T, Y):
        """Raw member outputs Z (members, n, 64) of the fused kernel."""
        S, n = Y.shape
        ld = api._species_major(Y, S, torch.float64, "Y")
        api._cells(rho, n, torch.float64, "rho")
        api._cells(T, n, torch.float64, "T")
        Z = torch.empty((self.members, n, OUT_PAD), dtype=torch.float32, device=Y.device)
        ws, need = self.workspace(mech, n)
        st = self._device()
        check(lib().pyro_surrogate_outputs(mech.handle, ctypes.byref(st), n, ld, _p(rho), _p(T),
                                           _p(Y), _p(Z), _p(ws), need, _stream()))
        return Z

    def eval(self, mech, rho, T, Y, thr_spread=None, thr_resid=None, out=None,
             indicators=False):
        """omega (S, n) with exact fallback; returns (omega, fell_back u8 (n,),
        n_fallback int64 (1,), indicators (2, n) or None)."""
        S, n = Y.shape
        ld = api._species_major(Y, S, torch.float64, "Y")
        api._cells(rho, n, torch.float64, "rho")
        api._cells(T, n, torch.float64, "T")
        if out is None:
            out = torch.empty((S, ld), dtype=torch.float64, device=Y.device)[:, :n]
        if api._species_major(out, S, torch.float64, "out") != ld:
            raise ValueError("out must have the row stride of Y")
        flags = torch.empty(n, dtype=torch.uint8, device=Y.device)
        count = torch.zeros(1, dtype=torch.int64, device=Y.device)
        ind = torch.empty((2, n), dtype=torch.float64, device=Y.device) if indicators else None
        ws, need = self.workspace(mech, n)
        st = self._device()
        ts = self.thr_spread if thr_spread is None else float(thr_spread)
        tr = self.thr_resid if thr_resid is None else float(thr_resid)
        check(lib().pyro_surrogate_eval(mech.handle, ctypes.byref(st), n, ld, _p(rho), _p(T),
                                        _p(Y), ts, tr, _p(out), _p(flags), _p(count), _p(ind),
                                        _p(ws), need, _stream()))
        return out, flags, count, ind


# ---------------------------------------------------------------------------
# Errors and threshold calibration (host statistics of device results)


def cell_errors(w_sur, w_exact):
    """Per-cell normwise relative error ||w_sur - w_exact|| / ||w_exact||
    (host arrays (S, n)) and the pieces of the global Frobenius error."""
    d = np.sqrt(((w_sur - w_exact) ** 2).sum(axis=0))
    r = np.sqrt((w_exact ** 2).sum(axis=0))
    return d / np.maximum(r, 1e-300), d ** 2, r ** 2


def error_summary(w_sur, w_exact):
    e, d2, r2 = cell_errors(w_sur, w_exact)
    return {"p50": float(np.percentile(e, 50)), "p99": float(np.percentile(e, 99)),
            "p99.9": float(np.percentile(e, 99.9)), "max": float(e.max()),
            "frobenius": float(math.sqrt(d2.sum() / r2.sum()))}


def calibrate(spread, resid, err, d2, r2, target=1e-3, quantiles=64):
    """Thresholds (thr_spread, thr_resid) with the smallest fallback fraction
    such that, on these held-out cells, the 99.9th percentile of the per-cell
    error and the Frobenius error after fallback are both at most ``target``
    (cells that fall back have zero error).  Candidates are quantiles of each
    indicator plus +inf and 0 (everything falls back), so a solution always
    exists.  Returns (thr_spread, thr_resid, fallback_fraction)."""
    n = err.shape[0]

    def grid(x):
        q = np.quantile(x[np.isfinite(x)], np.linspace(0.0, 1.0, quantiles)) if np.isfinite(
            x).any() else np.array([])
        return np.unique(np.concatenate([[0.0], q, [np.inf]]))

    gs, gr = grid(spread), grid(resid)
    # a cell is kept at thresholds (gs[j], gr[k]) iff spread < gs[j] and
    # resid < gr[k], i.e. iff bs <= j and br <= k with b = #grid <= x
    bs = np.searchsorted(gs, np.nan_to_num(spread, nan=np.inf), side="right")
    br = np.searchsorted(gr, np.nan_to_num(resid, nan=np.inf), side="right")
    ok = (bs < len(gs)) & (br < len(gr))
    shape = (len(gs), len(gr))
    bad = err > target

    def cum(weights):
        h = np.zeros(shape)
        np.add.at(h, (bs[ok], br[ok]), weights[ok])
        return h.cumsum(axis=0).cumsum(axis=1)

    kept = cum(np.ones(n))
    kept_bad = cum(bad.astype(np.float64))
    kept_d2 = cum(d2)
    frob = np.sqrt(kept_d2 / max(r2.sum(), 1e-300))
    feasible = (kept_bad <= math.floor(1e-3 * n)) & (frob <= target)
    kept_f = np.where(feasible, kept, -1.0)
    j, k = np.unravel_index(np.argmax(kept_f), shape)
    return float(gs[j]), float(gr[k]), 1.0 - float(kept[j, k]) / n
