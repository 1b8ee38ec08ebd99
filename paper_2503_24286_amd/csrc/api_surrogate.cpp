// C ABI of the learned surrogate: MLP training steps (forward, backward,
// loss, AdamW), feature and target preparation, and the evaluation pipeline
// with per-cell fallback to the exact production-rate kernel.
#include <string>

#include "mlp_internal.h"
#include "pyro_internal.h"
#include "surrogate_internal.h"

namespace pyro {
namespace {

// BF16 operands are read 16 bytes at a time
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_hidden(int hidden) {
    if (hidden < 64 || hidden > 4096 || hidden % 64 != 0)
        return fail(PYRO_E_ARG, "hidden width must be a multiple of 64 in [64, 4096]");
    return PYRO_OK;
}

// offsets of the four layers inside one member's packed parameters
struct Layout {
    int64_t w[4], b[4], w_total, b_total;
    int64_t kin[4], nout[4];
    explicit Layout(int H) {
        const int64_t K[4] = {kFeatPad, H, H, H}, N[4] = {H, H, H, kOutPad};
        int64_t ow = 0, ob = 0;
        for (int l = 0; l < 4; ++l) {
            kin[l] = K[l];
            nout[l] = N[l];
            w[l] = ow;
            b[l] = ob;
            ow += K[l] * N[l];
            ob += N[l];
        }
        w_total = ow;
        b_total = ob;
    }
};

GemmArgs nn(const uint16_t* A, int64_t lda, const uint16_t* B, int64_t M, int64_t N, int64_t K) {
    // C = A [M x K] (row-major, ld lda) * B [K x N] (row-major)
    GemmArgs g{};
    g.A = A;
    g.B = B;
    g.M = M;
    g.N = N;
    g.K = K;
    g.sam = lda;
    g.sak = 1;
    g.sbk = N;
    g.sbn = 1;
    g.ldc = N;
    return g;
}

hipError_t forward(const Layout& L, int64_t B, const uint16_t* X, const uint16_t* W,
                   const float* b, uint16_t* P[3], uint16_t* H[3], float* Z, hipStream_t s) {
    const uint16_t* in = X;
    int64_t ldin = kFeatPad;
    for (int l = 0; l < 4; ++l) {
        GemmArgs g = nn(in, ldin, W + L.w[l], B, L.nout[l], L.kin[l]);
        g.bias = b + L.b[l];
        hipError_t e;
        if (l < 3) {
            g.C_bf16 = H[l];
            g.P_bf16 = P[l];
            e = launch_gemm(g, kEpiBiasSilu, 1, s);
            in = H[l];
            ldin = L.nout[l];
        } else {
            g.C_f32 = Z;
            e = launch_gemm(g, kEpiBiasF32, 1, s);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int check_surrogate(const pyro_mech* m, const pyro_surrogate* sur, int64_t n, int64_t ld) {
    if (!m || !sur) return fail(PYRO_E_ARG, "null mechanism or surrogate");
    if (n < 0 || ld < n) return fail(PYRO_E_ARG, "bad n or ld");
    if (int rc = check_hidden(sur->hidden)) return rc;
    if (!fused_supported(sur->hidden))
        return fail(PYRO_E_UNSUPPORTED, "surrogate evaluation supports hidden widths 64, 128, 256");
    if (sur->n_members < 1 || sur->n_members > kMaxMembers)
        return fail(PYRO_E_ARG, "n_members must be in [1, 4]");
    if (m->S + 3 > kFeatPad) return fail(PYRO_E_UNSUPPORTED, "surrogate supports at most 61 species");
    if (!sur->weights || !sur->biases || !sur->feat_shift || !sur->feat_scale ||
        !sur->target_scale || !sur->target_mean || !sur->target_std)
        return fail(PYRO_E_ARG, "null pointer in the surrogate description");
    return PYRO_OK;
}

struct Packed {
    uint16_t* wp;
    float* bp;
    int64_t w_stride, b_stride;
    unsigned char* rest;
};

// packs every member's weights into the fragment order of the fused kernel
Packed pack(const pyro_surrogate* sur, void* workspace, hipStream_t s, hipError_t* e) {
    const Layout L(sur->hidden);
    Packed p;
    p.w_stride = packed_weight_elems(sur->hidden);
    p.b_stride = L.b_total;
    unsigned char* q = static_cast<unsigned char*>(workspace);
    p.wp = reinterpret_cast<uint16_t*>(q);
    q += (size_t(sur->n_members) * p.w_stride * 2 + 255) / 256 * 256;
    p.bp = reinterpret_cast<float*>(q);
    q += (size_t(sur->n_members) * p.b_stride * 4 + 255) / 256 * 256;
    p.rest = q;
    *e = launch_pack(sur->hidden, sur->n_members, L.w_total, L.b_total, sur->weights,
                     sur->biases, p.wp, p.bp, s);
    return p;
}

}  // namespace
}  // namespace pyro

using namespace pyro;

extern "C" {

size_t pyro_mlp_param_counts(int hidden, int64_t* n_weights, int64_t* n_biases) {
    if (check_hidden(hidden)) return 0;
    const Layout L(hidden);
    if (n_weights) *n_weights = L.w_total;
    if (n_biases) *n_biases = L.b_total;
    return size_t(L.w_total);
}

int pyro_mlp_forward(int hidden, int64_t batch, const uint16_t* X, const uint16_t* W,
                     const float* b, uint16_t* acts, float* Z, void* stream) {
    clear_error();
    if (int rc = check_hidden(hidden)) return rc;
    if (batch < 0) return fail(PYRO_E_ARG, "batch must be >= 0");
    if (batch == 0) return PYRO_OK;
    if (!X || !W || !b || !acts || !Z) return fail(PYRO_E_ARG, "null pointer argument");
    if (!aligned16(X) || !aligned16(W) || !aligned16(acts))
        return fail(PYRO_E_ARG, "BF16 arrays must be 16-byte aligned");
    const Layout L(hidden);
    uint16_t* P[3];
    uint16_t* H[3];
    for (int l = 0; l < 3; ++l) {
        P[l] = acts + (2 * l) * batch * hidden;
        H[l] = acts + (2 * l + 1) * batch * hidden;
    }
    hipError_t e = forward(L, batch, X, W, b, P, H, Z, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PYRO_OK : hip_fail(e, "MLP forward launch");
}

int pyro_mlp_backward(int hidden, int64_t batch, const uint16_t* X, const uint16_t* W,
                      const uint16_t* acts, const uint16_t* dZ, float* gW, float* gb,
                      uint16_t* work, float* split_work, int splits, void* stream) {
    clear_error();
    if (int rc = check_hidden(hidden)) return rc;
    if (batch <= 0) return fail(PYRO_E_ARG, "batch must be > 0");
    if (splits < 1 || splits > 1024) return fail(PYRO_E_ARG, "splits must be in [1, 1024]");
    if (!X || !W || !acts || !dZ || !gW || !gb || !work || !split_work)
        return fail(PYRO_E_ARG, "null pointer argument");
    if (!aligned16(X) || !aligned16(W) || !aligned16(acts) || !aligned16(dZ) || !aligned16(work))
        return fail(PYRO_E_ARG, "BF16 arrays must be 16-byte aligned");
    const Layout L(hidden);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint16_t* P[3];
    const uint16_t* H[3];
    for (int l = 0; l < 3; ++l) {
        P[l] = acts + (2 * l) * batch * hidden;
        H[l] = acts + (2 * l + 1) * batch * hidden;
    }
    // dY of layer l (bf16 [batch][nout]); two ping-pong buffers
    uint16_t* buf[2] = {work, work + batch * hidden};
    const uint16_t* dY = dZ;
    int64_t lddy = kOutPad;
    hipError_t e = hipSuccess;
    for (int l = 3; l >= 0 && e == hipSuccess; --l) {
        const uint16_t* in = l == 0 ? X : H[l - 1];
        const int64_t ldin = l == 0 ? kFeatPad : hidden;
        // weight gradient: gW[l](i, o) = sum_b in(b, i) dY(b, o), split over the batch
        GemmArgs g{};
        g.A = in;
        g.sam = 1;
        g.sak = ldin;
        g.B = dY;
        g.sbk = lddy;
        g.sbn = 1;
        g.M = L.kin[l];
        g.N = L.nout[l];
        g.K = batch;
        g.ldc = L.nout[l];
        g.C_f32 = split_work;
        e = launch_gemm(g, kEpiPartial, splits, s);
        if (e == hipSuccess)
            e = launch_sum_splits(split_work, splits, L.kin[l] * L.nout[l], gW + L.w[l], s);
        if (e == hipSuccess) e = launch_colsum_bf16(dY, batch, lddy, int(L.nout[l]), gb + L.b[l], s);
        if (l == 0 || e != hipSuccess) break;
        // input gradient through SiLU: dP(b, i) = silu'(P(b, i)) sum_o dY(b, o) W(i, o)
        GemmArgs h{};
        h.A = dY;
        h.sam = lddy;
        h.sak = 1;
        h.B = W + L.w[l];
        h.sbk = 1;
        h.sbn = L.nout[l];
        h.M = batch;
        h.N = L.kin[l];
        h.K = L.nout[l];
        h.ldc = hidden;
        uint16_t* out = buf[l & 1];
        h.C_bf16 = out;
        h.P_bf16 = const_cast<uint16_t*>(P[l - 1]);
        e = launch_gemm(h, kEpiDsilu, 1, s);
        dY = out;
        lddy = hidden;
    }
    return e == hipSuccess ? PYRO_OK : hip_fail(e, "MLP backward launch");
}

int64_t pyro_mlp_loss_partials(int64_t batch) { return mse_partials(batch, kOutPad); }

int pyro_mlp_mse(int64_t batch, int n_out, const float* Z, const float* Zt, uint16_t* dZ,
                 float* loss_partials, void* stream) {
    clear_error();
    if (batch <= 0 || n_out < 1 || n_out > kOutPad) return fail(PYRO_E_ARG, "bad batch or n_out");
    if (!Z || !Zt || !dZ || !loss_partials) return fail(PYRO_E_ARG, "null pointer argument");
    hipError_t e = launch_mse(Z, Zt, batch, kOutPad, n_out, dZ, loss_partials,
                              static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PYRO_OK : hip_fail(e, "MSE launch");
}

int pyro_adamw_step(int64_t n, float* w, uint16_t* w_bf16, const float* grad, float* m1,
                    float* m2, float lr, float beta1, float beta2, float eps, float weight_decay,
                    int step, void* stream) {
    clear_error();
    if (n < 0 || step < 1) return fail(PYRO_E_ARG, "n must be >= 0 and step >= 1");
    if (n == 0) return PYRO_OK;
    if (!w || !grad || !m1 || !m2) return fail(PYRO_E_ARG, "null pointer argument");
    hipError_t e = launch_adamw(n, w, w_bf16, grad, m1, m2, lr, beta1, beta2, eps, weight_decay,
                                step, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PYRO_OK : hip_fail(e, "AdamW launch");
}

int pyro_to_bf16(int64_t n, const float* x, uint16_t* y, void* stream) {
    clear_error();
    if (n < 0) return fail(PYRO_E_ARG, "n must be >= 0");
    if (n == 0) return PYRO_OK;
    if (!x || !y) return fail(PYRO_E_ARG, "null pointer argument");
    hipError_t e = launch_to_bf16(n, x, y, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PYRO_OK : hip_fail(e, "conversion launch");
}

int pyro_surrogate_features(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                            const double* T, const double* Y, const float* shift,
                            const float* scale, uint16_t* X, void* stream) {
    clear_error();
    if (!m) return fail(PYRO_E_ARG, "null mechanism handle");
    if (n < 0 || ld < n) return fail(PYRO_E_ARG, "bad n or ld");
    if (m->S + 3 > kFeatPad) return fail(PYRO_E_UNSUPPORTED, "surrogate supports at most 61 species");
    if (n == 0) return PYRO_OK;
    if (!rho || !T || !Y || !shift || !scale || !X) return fail(PYRO_E_ARG, "null pointer argument");
    if (!aligned16(X)) return fail(PYRO_E_ARG, "X must be 16-byte aligned");
    hipError_t e = launch_features(m, n, ld, rho, T, Y, shift, scale, X,
                                   static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PYRO_OK : hip_fail(e, "feature launch");
}

int pyro_surrogate_targets(const pyro_mech* m, int64_t n, int64_t ld, const double* wdot,
                           const double* scale, const double* mean, const double* std_dev,
                           float* Zt, void* stream) {
    clear_error();
    if (!m) return fail(PYRO_E_ARG, "null mechanism handle");
    if (n < 0 || ld < n) return fail(PYRO_E_ARG, "bad n or ld");
    if (m->S > kOutPad) return fail(PYRO_E_UNSUPPORTED, "surrogate supports at most 64 species");
    if (n == 0) return PYRO_OK;
    if (!wdot || !scale || !mean || !std_dev || !Zt) return fail(PYRO_E_ARG, "null pointer argument");
    hipError_t e = launch_targets(m, n, ld, wdot, scale, mean, std_dev, Zt,
                                  static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PYRO_OK : hip_fail(e, "target launch");
}

size_t pyro_surrogate_workspace_size(const pyro_mech* m, int64_t n, int hidden, int members) {
    if (!m || n < 0 || check_hidden(hidden) || !fused_supported(hidden) || members < 1 ||
        members > kMaxMembers)
        return 0;
    const Layout L(hidden);
    const int64_t nb = compaction_blocks(n);
    size_t b = 0;
    auto add = [&](size_t bytes) { b += (bytes + 255) / 256 * 256; };
    add(size_t(members) * packed_weight_elems(hidden) * 2);  // packed weights
    add(size_t(members) * L.b_total * 4);                    // packed biases
    add(size_t(nb + 1) * 8);                                 // block counts
    add(size_t(n) * 8);                                      // indices
    add(size_t(n) * 8 * 2);                                  // compact rho, T
    add(size_t(n) * m->S * 8 * 2);                           // compact Y, omega
    return b;
}

int pyro_surrogate_outputs(const pyro_mech* m, const pyro_surrogate* sur, int64_t n, int64_t ld,
                           const double* rho, const double* T, const double* Y, float* Z,
                           void* workspace, size_t workspace_bytes, void* stream) {
    clear_error();
    if (int rc = check_surrogate(m, sur, n, ld)) return rc;
    if (n == 0) return PYRO_OK;
    if (!rho || !T || !Y || !Z || !workspace) return fail(PYRO_E_ARG, "null pointer argument");
    if (!aligned16(sur->weights) || (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return fail(PYRO_E_ARG, "weights must be 16-byte and the workspace 256-byte aligned");
    const size_t need = pyro_surrogate_workspace_size(m, n, sur->hidden, sur->n_members);
    if (workspace_bytes < need)
        return fail(PYRO_E_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    const Packed p = pack(sur, workspace, s, &e);
    if (e == hipSuccess)
        e = launch_fused(m, sur->hidden, sur->n_members, n, ld, rho, T, Y, p.wp, p.bp, p.w_stride,
                         p.b_stride, sur->feat_shift, sur->feat_scale, sur->target_scale,
                         sur->target_mean, sur->target_std, 0.0, 0.0, nullptr, nullptr, nullptr, Z,
                         nullptr, s);
    return e == hipSuccess ? PYRO_OK : hip_fail(e, "surrogate output launch");
}

int pyro_surrogate_eval(const pyro_mech* m, const pyro_surrogate* sur, int64_t n, int64_t ld,
                        const double* rho, const double* T, const double* Y, double thr_spread,
                        double thr_resid, double* wdot, uint8_t* fell_back,
                        int64_t* n_fallback, double* indicators, void* workspace,
                        size_t workspace_bytes, void* stream) {
    clear_error();
    if (int rc = check_surrogate(m, sur, n, ld)) return rc;
    if (m->E > kMaxElements) return fail(PYRO_E_UNSUPPORTED, "surrogate supports at most 16 elements");
    if (n == 0) return PYRO_OK;
    if (!rho || !T || !Y || !wdot || !fell_back || !n_fallback || !workspace)
        return fail(PYRO_E_ARG, "null pointer argument");
    if (!aligned16(sur->weights) || (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return fail(PYRO_E_ARG, "weights must be 16-byte and the workspace 256-byte aligned");
    const size_t need = pyro_surrogate_workspace_size(m, n, sur->hidden, sur->n_members);
    if (workspace_bytes < need)
        return fail(PYRO_E_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (!indicators && !(thr_spread > 0.0 && thr_resid > 0.0)) {
        // no cell can be kept (spread and residual are never negative): the
        // call is the exact kernel on every cell, the network is not run
        e = launch_fallback_all(n, fell_back, n_fallback, s);
        if (e == hipSuccess)
            e = launch_production_rates(m, n, ld, PYRO_F64, rho, T, Y, wdot, nullptr, s, nullptr);
        return e == hipSuccess ? PYRO_OK : hip_fail(e, "surrogate launch");
    }
    const Packed p = pack(sur, workspace, s, &e);
    const int64_t nb = compaction_blocks(n);
    unsigned char* q = p.rest;
    auto take = [&](size_t bytes) {
        unsigned char* r = q;
        q += (bytes + 255) / 256 * 256;
        return r;
    };
    int64_t* counts = reinterpret_cast<int64_t*>(take(size_t(nb + 1) * 8));
    int64_t* idx = reinterpret_cast<int64_t*>(take(size_t(n) * 8));
    double* rc = reinterpret_cast<double*>(take(size_t(n) * 8 * 2));
    double* tc = rc + n;
    double* yc = reinterpret_cast<double*>(take(size_t(n) * m->S * 8 * 2));
    double* wc = yc + size_t(n) * m->S;

    // the network (member outputs staged in the compacted-state region, free
    // until the compaction), then prediction, indicators and flags; then the
    // flagged cells, compacted in ascending order, through the exact kernel.
    // The staged outputs, members x S x n floats, fit that region (2 S n
    // doubles) for up to four members.
    static_assert(kMaxMembers <= 4, "staged member outputs must fit the compacted-state region");
    if (e == hipSuccess)
        e = launch_fused(m, sur->hidden, sur->n_members, n, ld, rho, T, Y, p.wp, p.bp, p.w_stride,
                         p.b_stride, sur->feat_shift, sur->feat_scale, sur->target_scale,
                         sur->target_mean, sur->target_std, thr_spread, thr_resid, wdot,
                         fell_back, indicators, nullptr, reinterpret_cast<float*>(yc), s);
    if (e == hipSuccess) e = launch_compaction(n, fell_back, counts, n_fallback, idx, s);
    if (e == hipSuccess) e = launch_gather(m->S, n, ld, n_fallback, idx, rho, T, Y, rc, tc, yc, s);
    if (e == hipSuccess)
        e = launch_production_rates(m, n, n, PYRO_F64, rc, tc, yc, wc, nullptr, s, n_fallback);
    if (e == hipSuccess) e = launch_scatter(m->S, n, ld, n_fallback, idx, wc, wdot, s);
    return e == hipSuccess ? PYRO_OK : hip_fail(e, "surrogate launch");
}

}  // extern "C"
