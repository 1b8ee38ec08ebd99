// Mixture-averaged transport properties per cell (appendix "Extensions to
// Flow & Transport": eq. mixavg_viscosity, eq. mixavg_conductivity,
// eq. species_cond, eq. diff_mix_rule and the binary-diffusivity fit).
//
// With L = ln T and the species fits P_k(L) = sum_m b_km L^m,
//   mu_k = sqrt(T) P_k^2,   sqrt(mu_k/mu_j) = |P_k|/|P_j|,
// so Phi_kj = (1 + (|P_k|/|P_j|) w_kj)^2 v_kj with the per-pair constants
// w_kj = (W_j/W_k)^(1/4) and v_kj = (8 (1 + W_k/W_j))^(-1/2) formed once on
// the host: no square root per pair.  The O(S^2) sums over pairs run with one
// cell per lane; the species k are taken in blocks of KB whose accumulators
// (sum_j Phi_kj X_j and sum_{j != k} X_j/D_kj) stay in registers while j
// streams through every species, its mole fraction and |P_j| formed on the
// fly.  Pair records (w, v, the five D_kj coefficients) are 64 bytes, read as
// wave-uniform scalar loads.
#include "pyro_internal.h"

namespace pyro {
namespace {

constexpr int kTBlock = 256;   // lanes per workgroup

__device__ inline double poly5(cptr<double> a, double L) {
    return fma(L, fma(L, fma(L, fma(L, a[4], a[3]), a[2]), a[1]), a[0]);
}

// 1/x from the hardware estimate refined by two Newton steps
__device__ inline double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

template <int KB>
__global__ __launch_bounds__(kTBlock) void transport_kernel(
    DevMech m, TransportTables tt, int64_t n, int64_t ld, const double* __restrict__ T,
    const double* __restrict__ Y, double* __restrict__ mu_out, double* __restrict__ kappa_out,
    double* __restrict__ D_out) {
    const int64_t i = int64_t(blockIdx.x) * kTBlock + threadIdx.x;
    const bool valid = i < n;
    const int64_t c = valid ? i : n - 1;
    const int S = m.S;
    const cptr<double> inv_w = cst(tt.inv_w);
    const cptr<double> visc = cst(tt.visc);
    const cptr<double> cond = cst(tt.cond);
    const cptr<double> pair = cst(tt.pair);
    const double Tc = T[c];
    const double L = log(Tc);
    const double sT = sqrt(Tc);
    // mixture molar mass and the conductivity sums (X_k = W Y_k/W_k)
    double xs = 0.0, ka = 0.0, kb = 0.0;
    for (int k = 0; k < S; ++k) {
        const double x = Y[size_t(k) * ld + c] * inv_w[k];
        const double kap = sT * poly5(cond + 5 * k, L);
        xs += x;
        ka = fma(x, kap, ka);
        kb = fma(x, recip(kap), kb);
    }
    const double Wm = 1.0 / xs;
    // kappa = (sum X k + (sum X/k)^-1)/2 with X = x W
    const double kappa = 0.5 * (Wm * ka + 1.0 / (Wm * kb));
    double mu = 0.0;
    for (int k0 = 0; k0 < S; k0 += KB) {
        double ap[KB], ad[KB], rk[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            ap[u] = ad[u] = 0.0;
            rk[u] = k0 + u < S ? fabs(poly5(visc + 5 * (k0 + u), L)) : 1.0;
        }
        for (int j = 0; j < S; ++j) {
            const double xj = Y[size_t(j) * ld + c] * inv_w[j] * Wm;
            const double irj = recip(fabs(poly5(visc + 5 * j, L)));
            const cptr<double> pj = pair + size_t(j) * S * 8;
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                const int k = k0 + u;
                if (k < S) {
                    const cptr<double> pr = pj + size_t(k) * 8;   // pair (k, j)
                    const double q = fma(rk[u], pr[0] * irj, 1.0);
                    ap[u] = fma(q * q * pr[1], xj, ap[u]);
                    if (j != k) ad[u] = fma(xj, recip(poly5(pr + 2, L)), ad[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int k = k0 + u;
            if (k < S) {
                const double xk = Y[size_t(k) * ld + c] * inv_w[k] * Wm;
                mu = fma(xk * sT * rk[u] * rk[u], 1.0 / ap[u], mu);
                // D_km = (W - X_k W_k)/W (sum_{j != k} X_j/D_kj)^-1, D_kj = sqrt(T) P_kj
                const double num = (Wm - xk / inv_w[k]) / Wm;
                if (valid) D_out[size_t(k) * ld + i] = num * sT / ad[u];
            }
        }
    }
    if (valid) {
        mu_out[i] = mu;
        kappa_out[i] = kappa;
    }
}

}  // namespace

hipError_t launch_transport(const pyro_mech* m, const TransportTables& tt, int64_t n,
                            int64_t ld, const double* T, const double* Y, double* mu,
                            double* kappa, double* D, hipStream_t stream) {
    const unsigned blocks = unsigned((n + kTBlock - 1) / kTBlock);
    // blocks of four species: 58 VGPRs, eight waves per SIMD to cover the
    // scalar loads of the pair records (2^20 config-1 cells: 3.78 ms, against
    // 3.85 with 128-lane workgroups, 4.0 with blocks of 6, 4.25 of 8, 4.55
    // of 2 and 5.49 of 16 at three waves per SIMD)
    hipLaunchKernelGGL(transport_kernel<4>, dim3(blocks), dim3(kTBlock), 0, stream, m->dev, tt,
                       n, ld, T, Y, mu, kappa, D);
    return hipGetLastError();
}

}  // namespace pyro
