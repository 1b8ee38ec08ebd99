// Internal declarations of the surrogate's MLP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pyro {

enum : int { kEpiBiasSilu = 0, kEpiBiasF32 = 1, kEpiDsilu = 2, kEpiPartial = 3 };

// BF16 <-> FP32.  The narrowing rounds to nearest even with gfx950's
// v_cvt_pk_bf16_f32 (NaN stays NaN).
__device__ inline float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, __bf16(f)); }
__device__ inline uint32_t f2bf2(float lo, float hi) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 v = {__bf16(lo), __bf16(hi)};
    return __builtin_bit_cast(uint32_t, v);
}

// SiLU x sigma(x) and its derivative, sigma(x) = 1/(1 + e^-x) from the
// hardware exponential and reciprocal (a few FP32 ulps; the results are
// rounded to BF16).  e^-x = inf gives sigma = 0.
__device__ inline float sigmoid(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }
__device__ inline float silu(float x) { return x * sigmoid(x); }
__device__ inline float dsilu(float x) {
    const float s = sigmoid(x);
    return s * (1.0f + x * (1.0f - s));
}

// C(m, n) = sum_k A(m, k) B(k, n), A(m, k) = A[m*sam + k*sak],
// B(k, n) = B[k*sbk + n*sbn]; BF16 operands (raw 16-bit patterns), FP32
// accumulation; the epilogue decides what is written at C[m*ldc + n].
struct GemmArgs {
    const uint16_t* A;
    const uint16_t* B;
    int64_t M, N, K;
    int64_t sam, sak, sbk, sbn;
    int64_t ldc;
    const float* bias;      // kEpiBiasSilu, kEpiBiasF32
    uint16_t* C_bf16;       // kEpiBiasSilu (activation), kEpiDsilu
    uint16_t* P_bf16;       // kEpiBiasSilu (pre-activation out), kEpiDsilu (in)
    float* C_f32;           // kEpiBiasF32, kEpiPartial ([split][M][ldc])
};

hipError_t launch_gemm(const GemmArgs& g, int epi, int splits, hipStream_t stream);
hipError_t launch_sum_splits(const float* part, int splits, int64_t count, float* out,
                             hipStream_t stream);
hipError_t launch_colsum_bf16(const uint16_t* X, int64_t M, int64_t ld, int N, float* out,
                              hipStream_t stream);
hipError_t launch_mse(const float* Z, const float* Zt, int64_t M, int ld, int n_out,
                      uint16_t* dZ, float* loss_part, hipStream_t stream);
int64_t mse_partials(int64_t M, int ld);
hipError_t launch_adamw(int64_t n, float* w, uint16_t* w_bf16, const float* grad, float* m1,
                        float* m2, float lr, float b1, float b2, float eps, float wd, int step,
                        hipStream_t stream);
hipError_t launch_to_bf16(int64_t n, const float* x, uint16_t* y, hipStream_t stream);

}  // namespace pyro
