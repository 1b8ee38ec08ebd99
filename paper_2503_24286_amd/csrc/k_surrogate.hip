// The learned surrogate's per-cell helpers: training features and targets,
// and the deterministic compaction, gather and scatter around the
// exact-kernel fallback.
//
// Features (S + 3 used of 64, BF16, one row per cell): T/1000, log10 p (p
// from the equation of state, eq. eos), ln(max(Y_k, 0) + 1e-12), each shifted
// and scaled by the training-set statistics, a constant 1, and zero padding.
// Targets: z_k = (asinh(omega_k / s_k) - mu_k) / sigma_k with s_k the median
// |omega_k| of the training set, inverted as omega_k = s_k sinh(mu_k +
// sigma_k z_k).
#include "pyro_internal.h"
#include "mlp_internal.h"
#include "surrogate_internal.h"

namespace pyro {
namespace {

constexpr int kBlock = 256;
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kBlock) void features_kernel(DevMech m, int64_t n, int64_t ld,
                                                          const double* __restrict__ rho,
                                                          const double* __restrict__ T,
                                                          const double* __restrict__ Y,
                                                          const float* __restrict__ shift,
                                                          const float* __restrict__ scale,
                                                          uint16_t* __restrict__ X) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    uint16_t row[kFeatPad];
#pragma unroll
    for (int f = 0; f < kFeatPad; ++f) row[f] = 0;
    const double Tc = T[i];
    double x = 0.0;  // 1/W
    for (int k = 0; k < m.S; ++k) {
        const double y = Y[size_t(k) * ld + i];
        x += y * m.newton[k].inv_w;
        row[k + 2] = f2bf(float((log(fmax(y, 0.0) + 1e-12) - shift[k + 2]) * scale[k + 2]));
    }
    const double p = rho[i] * kGasConstant * Tc * x;
    row[0] = f2bf(float((Tc * 1e-3 - shift[0]) * scale[0]));
    row[1] = f2bf(float((log10(p) - shift[1]) * scale[1]));
    row[m.S + 2] = f2bf(1.0f);
    uint4* dst = reinterpret_cast<uint4*>(X + i * kFeatPad);
#pragma unroll
    for (int q = 0; q < kFeatPad / 8; ++q) dst[q] = reinterpret_cast<const uint4*>(row)[q];
}

__global__ __launch_bounds__(kBlock) void targets_kernel(int S, int64_t n, int64_t ld,
                                                         const double* __restrict__ wdot,
                                                         const double* __restrict__ ts,
                                                         const double* __restrict__ tmu,
                                                         const double* __restrict__ tsig,
                                                         float* __restrict__ Zt) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < kOutPad; ++k)
        Zt[i * kOutPad + k] =
            k < S ? float((asinh(wdot[size_t(k) * ld + i] / ts[k]) - tmu[k]) / tsig[k]) : 0.0f;
}

// Compaction of the flagged cells in ascending order: per-block counts, one
// exclusive scan of the counts, per-block prefix sums.
__global__ __launch_bounds__(kScanBlock) void count_kernel(int64_t n, const uint8_t* __restrict__ flag,
                                                           int64_t* __restrict__ counts) {
    __shared__ int red[kScanBlock];
    const int64_t i = int64_t(blockIdx.x) * kScanBlock + threadIdx.x;
    red[threadIdx.x] = (i < n && flag[i]) ? 1 : 0;
    __syncthreads();
    for (int h = kScanBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

// exclusive scan of nb block counts by one block; total to *total
__global__ __launch_bounds__(kScanBlock) void scan_counts_kernel(int64_t nb, int64_t* __restrict__ counts,
                                                                int64_t* __restrict__ total) {
    __shared__ int64_t part[kScanBlock];
    const int64_t per = (nb + kScanBlock - 1) / kScanBlock;
    const int64_t b0 = threadIdx.x * per, b1 = b0 + per < nb ? b0 + per : nb;
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += counts[b];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int t = 0; t < kScanBlock; ++t) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
        *total = run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t v = counts[b];
        counts[b] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kScanBlock) void compact_kernel(int64_t n, const uint8_t* __restrict__ flag,
                                                             const int64_t* __restrict__ offsets,
                                                             int64_t* __restrict__ idx) {
    __shared__ int sc[kScanBlock];
    const int64_t i = int64_t(blockIdx.x) * kScanBlock + threadIdx.x;
    const int f = (i < n && flag[i]) ? 1 : 0;
    sc[threadIdx.x] = f;
    __syncthreads();
    // Hillis-Steele inclusive scan
    for (int h = 1; h < kScanBlock; h <<= 1) {
        const int v = threadIdx.x >= h ? sc[threadIdx.x - h] : 0;
        __syncthreads();
        sc[threadIdx.x] += v;
        __syncthreads();
    }
    if (f) idx[offsets[blockIdx.x] + sc[threadIdx.x] - 1] = i;
}

__global__ __launch_bounds__(kBlock) void gather_kernel(int S, int64_t n, int64_t ld,
                                                        const int64_t* __restrict__ count,
                                                        const int64_t* __restrict__ idx,
                                                        const double* __restrict__ rho,
                                                        const double* __restrict__ T,
                                                        const double* __restrict__ Y,
                                                        double* __restrict__ rc,
                                                        double* __restrict__ Tcc,
                                                        double* __restrict__ Yc) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= *count) return;
    const int64_t c = idx[i];
    rc[i] = rho[c];
    Tcc[i] = T[c];
    for (int k = 0; k < S; ++k) Yc[size_t(k) * n + i] = Y[size_t(k) * ld + c];
}

__global__ __launch_bounds__(kBlock) void scatter_kernel(int S, int64_t n, int64_t ld,
                                                         const int64_t* __restrict__ count,
                                                         const int64_t* __restrict__ idx,
                                                         const double* __restrict__ wc,
                                                         double* __restrict__ wdot) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= *count) return;
    const int64_t c = idx[i];
    for (int k = 0; k < S; ++k) wdot[size_t(k) * ld + c] = wc[size_t(k) * n + i];
}

// every cell sent to the exact kernel: flags set, the count is n
__global__ __launch_bounds__(kBlock) void fallback_all_kernel(int64_t n, uint8_t* __restrict__ flag,
                                                              int64_t* __restrict__ total) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) flag[i] = 1;
    if (i == 0) *total = n;
}

unsigned grid(int64_t n, int b) { return unsigned((n + b - 1) / b); }

}  // namespace

hipError_t launch_features(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                           const double* T, const double* Y, const float* shift,
                           const float* scale, uint16_t* X, hipStream_t stream) {
    hipLaunchKernelGGL(features_kernel, dim3(grid(n, kBlock)), dim3(kBlock), 0, stream, m->dev, n,
                       ld, rho, T, Y, shift, scale, X);
    return hipGetLastError();
}

hipError_t launch_targets(const pyro_mech* m, int64_t n, int64_t ld, const double* wdot,
                          const double* ts, const double* tmu, const double* tsig, float* Zt,
                          hipStream_t stream) {
    hipLaunchKernelGGL(targets_kernel, dim3(grid(n, kBlock)), dim3(kBlock), 0, stream, m->S, n, ld,
                       wdot, ts, tmu, tsig, Zt);
    return hipGetLastError();
}

int64_t compaction_blocks(int64_t n) { return (n + kScanBlock - 1) / kScanBlock; }

hipError_t launch_compaction(int64_t n, const uint8_t* flag, int64_t* counts, int64_t* total,
                             int64_t* idx, hipStream_t stream) {
    const int64_t nb = compaction_blocks(n);
    hipLaunchKernelGGL(count_kernel, dim3(unsigned(nb)), dim3(kScanBlock), 0, stream, n, flag,
                       counts);
    hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(kScanBlock), 0, stream, nb, counts, total);
    hipLaunchKernelGGL(compact_kernel, dim3(unsigned(nb)), dim3(kScanBlock), 0, stream, n, flag,
                       counts, idx);
    return hipGetLastError();
}

hipError_t launch_fallback_all(int64_t n, uint8_t* flag, int64_t* total, hipStream_t stream) {
    hipLaunchKernelGGL(fallback_all_kernel, dim3(grid(n, kBlock)), dim3(kBlock), 0, stream, n, flag,
                       total);
    return hipGetLastError();
}

hipError_t launch_gather(int S, int64_t n, int64_t ld, const int64_t* count, const int64_t* idx,
                         const double* rho, const double* T, const double* Y, double* rc,
                         double* Tc, double* Yc, hipStream_t stream) {
    hipLaunchKernelGGL(gather_kernel, dim3(grid(n, kBlock)), dim3(kBlock), 0, stream, S, n, ld,
                       count, idx, rho, T, Y, rc, Tc, Yc);
    return hipGetLastError();
}

hipError_t launch_scatter(int S, int64_t n, int64_t ld, const int64_t* count, const int64_t* idx,
                          const double* wc, double* wdot, hipStream_t stream) {
    hipLaunchKernelGGL(scatter_kernel, dim3(grid(n, kBlock)), dim3(kBlock), 0, stream, S, n, ld,
                       count, idx, wc, wdot);
    return hipGetLastError();
}

}  // namespace pyro
