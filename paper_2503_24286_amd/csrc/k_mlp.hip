// BF16 multilayer-perceptron kernels of the learned surrogate: a tiled GEMM
// on the gfx950 matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation)
// with fused epilogues, and the small element-wise kernels of training
// (loss, bias gradients, AdamW).
//
// GEMM: C(m, n) = sum_k A(m, k) B(k, n) with A(m, k) = A[m*sam + k*sak] and
// B(k, n) = B[k*sbk + n*sbn], so one kernel serves X W (forward),
// dY W^T (input gradients) and X^T dY (weight gradients, split over the
// batch).  A workgroup of four wavefronts owns a 64 x 64 output tile, each
// wavefront a 32 x 32 block; the K loop stages 64 x 32 slices of A and B in
// LDS (rows padded against bank conflicts) and issues two 32x32x16 MFMAs per
// wavefront per slice.
#include "mlp_internal.h"

namespace pyro {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBM = 64, kBN = 64, kBK = 32;
constexpr int kLdsK = kBK + 8;  // padded row of a staged slice (bf16 elements)


// Stage a 64 x 32 slice: rows r0.., k k0.. of X(r, k) = X[r*sr + k*sk]
// (zero outside rows < R, k < K) into S[row][k].
__device__ inline void stage(uint16_t* S, const uint16_t* __restrict__ X, int64_t sr, int64_t sk,
                             int64_t R, int64_t K, int64_t r0, int64_t k0, int tid) {
    if (sk == 1) {
        // k contiguous: each thread copies 8 consecutive k of one row
        const int row = tid >> 2, kc = (tid & 3) * 8;
        const int64_t r = r0 + row, k = k0 + kc;
        uint16_t v[8];
        if (r < R && k + 8 <= K && ((sr & 7) == 0)) {
            const uint4 q = *reinterpret_cast<const uint4*>(X + r * sr + k);
            *reinterpret_cast<uint4*>(v) = q;
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (r < R && k + j < K) ? X[r * sr + k + j] : uint16_t(0);
        }
        *reinterpret_cast<uint4*>(S + row * kLdsK + kc) = *reinterpret_cast<uint4*>(v);
    } else {
        // rows contiguous: each thread copies 8 consecutive rows of one k
        const int kk = tid >> 3, rc = (tid & 7) * 8;
        const int64_t k = k0 + kk, r = r0 + rc;
        uint16_t v[8];
        if (k < K && r + 8 <= R && sr == 1 && ((sk & 7) == 0)) {
            const uint4 q = *reinterpret_cast<const uint4*>(X + k * sk + r);
            *reinterpret_cast<uint4*>(v) = q;
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (k < K && r + j < R) ? X[(r + j) * sr + k * sk] : uint16_t(0);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) S[(rc + j) * kLdsK + kk] = v[j];
    }
}

template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kBM * kLdsK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN * kLdsK];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int64_t m0 = int64_t(blockIdx.x) * kBM;
    const int64_t n0 = int64_t(blockIdx.y) * kBN;
    // split of the K range (weight gradients): blockIdx.z
    const int64_t kper = ((g.K + gridDim.z - 1) / gridDim.z + kBK - 1) / kBK * kBK;
    const int64_t kb = int64_t(blockIdx.z) * kper;
    const int64_t ke = kb + kper < g.K ? kb + kper : g.K;
    f32x16 acc = {};
    for (int64_t k0 = kb; k0 < ke; k0 += kBK) {
        stage(As, g.A, g.sam, g.sak, g.M, ke, m0, k0, tid);
        // B(k, n): staged as Bs[n][k]
        stage(Bs, g.B, g.sbn, g.sbk, g.N, ke, n0, k0, tid);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kBK / 16; ++s) {
            const int kk = s * 16 + 8 * (lane >> 5);
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(As + (32 * wr + (lane & 31)) * kLdsK + kk);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(Bs + (32 * wc + (lane & 31)) * kLdsK + kk);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // result element i of the lane: row 8(i/4) + 4(lane/32) + i%4, column lane%32
    const int64_t col = n0 + 32 * wc + (lane & 31);
    if (col >= g.N) return;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t row = m0 + 32 * wr + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        if (row >= g.M) continue;
        const float v = acc[i];
        const int64_t o = row * g.ldc + col;
        if constexpr (EPI == kEpiBiasSilu) {
            const float p = v + g.bias[col];
            g.C_bf16[o] = f2bf(silu(p));
            if (g.P_bf16) g.P_bf16[o] = f2bf(p);
        } else if constexpr (EPI == kEpiBiasF32) {
            g.C_f32[o] = v + g.bias[col];
        } else if constexpr (EPI == kEpiDsilu) {
            g.C_bf16[o] = f2bf(v * dsilu(bf2f(g.P_bf16[o])));
        } else {  // kEpiPartial: [split][M][N]
            g.C_f32[int64_t(blockIdx.z) * g.M * g.ldc + o] = v;
        }
    }
}

// dW = sum of the split partials, in split order; db[n] = sum_m dY(m, n).
__global__ void sum_splits_kernel(const float* __restrict__ part, int splits, int64_t count,
                                  float* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += part[int64_t(z) * count + i];
    out[i] = s;
}

// column sums of a [M][ld] bf16 matrix: one block per column group, fixed
// order (deterministic)
__global__ void colsum_bf16_kernel(const uint16_t* __restrict__ X, int64_t M, int64_t ld, int N,
                                   float* __restrict__ out) {
    __shared__ float red[256];
    const int col = blockIdx.x;
    float s = 0.0f;
    for (int64_t m = threadIdx.x; m < M; m += blockDim.x) s += bf2f(X[m * ld + col]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && col < N) out[col] = red[0];
}

// MSE in the normalised target space over the first n_out columns:
// dZ = 2 (Z - Zt) / (M n_out) as bf16 (zero in padded columns) and the
// per-block partial loss sums.
__global__ void mse_kernel(const float* __restrict__ Z, const float* __restrict__ Zt, int64_t M,
                           int ld, int n_out, uint16_t* __restrict__ dZ,
                           float* __restrict__ loss_part) {
    __shared__ float red[256];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (i < M * ld) {
        const int col = int(i % ld);
        float d = 0.0f;
        if (col < n_out) {
            d = Z[i] - Zt[i];
            l = d * d;
        }
        dZ[i] = f2bf(2.0f * d / float(M * n_out));
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// AdamW (decoupled weight decay) on FP32 master weights; writes the BF16 copy.
__global__ void adamw_kernel(int64_t n, float* __restrict__ w, uint16_t* __restrict__ w_bf16,
                             const float* __restrict__ grad, float* __restrict__ m1,
                             float* __restrict__ m2, float lr, float b1, float b2, float eps,
                             float wd, float c1, float c2) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float a = b1 * m1[i] + (1.0f - b1) * g;
    const float b = b2 * m2[i] + (1.0f - b2) * g * g;
    m1[i] = a;
    m2[i] = b;
    const float mh = a / c1, vh = b / c2;
    const float x = w[i] * (1.0f - lr * wd) - lr * mh / (sqrtf(vh) + eps);
    w[i] = x;
    if (w_bf16) w_bf16[i] = f2bf(x);
}

__global__ void to_bf16_kernel(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

}  // namespace

hipError_t launch_gemm(const GemmArgs& g, int epi, int splits, hipStream_t stream) {
    const dim3 grid(unsigned((g.M + kBM - 1) / kBM), unsigned((g.N + kBN - 1) / kBN),
                    unsigned(splits));
    switch (epi) {
        case kEpiBiasSilu:
            hipLaunchKernelGGL(gemm_bf16_kernel<kEpiBiasSilu>, grid, dim3(256), 0, stream, g);
            break;
        case kEpiBiasF32:
            hipLaunchKernelGGL(gemm_bf16_kernel<kEpiBiasF32>, grid, dim3(256), 0, stream, g);
            break;
        case kEpiDsilu:
            hipLaunchKernelGGL(gemm_bf16_kernel<kEpiDsilu>, grid, dim3(256), 0, stream, g);
            break;
        default:
            hipLaunchKernelGGL(gemm_bf16_kernel<kEpiPartial>, grid, dim3(256), 0, stream, g);
    }
    return hipGetLastError();
}

hipError_t launch_sum_splits(const float* part, int splits, int64_t count, float* out,
                             hipStream_t stream) {
    hipLaunchKernelGGL(sum_splits_kernel, dim3(unsigned((count + 255) / 256)), dim3(256), 0,
                       stream, part, splits, count, out);
    return hipGetLastError();
}

hipError_t launch_colsum_bf16(const uint16_t* X, int64_t M, int64_t ld, int N, float* out,
                              hipStream_t stream) {
    hipLaunchKernelGGL(colsum_bf16_kernel, dim3(unsigned(N)), dim3(256), 0, stream, X, M, ld, N,
                       out);
    return hipGetLastError();
}

hipError_t launch_mse(const float* Z, const float* Zt, int64_t M, int ld, int n_out, uint16_t* dZ,
                      float* loss_part, hipStream_t stream) {
    const int64_t total = M * ld;
    hipLaunchKernelGGL(mse_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, stream, Z,
                       Zt, M, ld, n_out, dZ, loss_part);
    return hipGetLastError();
}

int64_t mse_partials(int64_t M, int ld) { return (M * ld + 255) / 256; }

hipError_t launch_adamw(int64_t n, float* w, uint16_t* w_bf16, const float* grad, float* m1,
                        float* m2, float lr, float b1, float b2, float eps, float wd, int step,
                        hipStream_t stream) {
    // bias corrections in FP64: 1 - b2^t cancels badly in FP32 for b2 near 1
    const float c1 = float(1.0 - pow(double(b1), double(step)));
    const float c2 = float(1.0 - pow(double(b2), double(step)));
    hipLaunchKernelGGL(adamw_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, n, w,
                       w_bf16, grad, m1, m2, lr, b1, b2, eps, wd, c1, c2);
    return hipGetLastError();
}

hipError_t launch_to_bf16(int64_t n, const float* x, uint16_t* y, hipStream_t stream) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, n, x,
                       y);
    return hipGetLastError();
}

}  // namespace pyro
