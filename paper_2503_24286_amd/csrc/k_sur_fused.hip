// Surrogate inference in two kernels.  The network kernel forms the features
// and runs every ensemble member's four layers; activations never leave
// registers and each member's outputs go straight from registers to global
// memory (species-major for the evaluation, cell-major for the raw-output
// call).  The post kernel, one thread per cell at full occupancy, forms the
// ensemble mean, the inverse target transform and the error indicators in
// FP64 (they ran at the network's one wavefront per SIMD when fused, where
// their latencies had nothing to hide behind).
//
// One wavefront owns 32 cells.  Each layer is computed transposed,
// out^T [N x 32 cells] = W^T [N x K] in^T [K x 32 cells], with
// v_mfma_f32_32x32x16_bf16: the A operand (weights) is a pre-packed 16-byte
// fragment per lane, the B operand is the previous layer's output.  The
// workgroup's wavefronts share the weights: each two-K-step slice of a layer
// is copied once into LDS (double-buffered, the next slice's global loads in
// flight while the current one multiplies) and read from there by every
// wavefront.  Lane l holds, for cell l%32, the outputs 8(i/4) + 4(l/32) + i%4
// of each 32-row block (register i).  Reading registers 8t..8t+7 of block
// ob as the B operand of K-step 2 ob + t therefore sums over the inputs
// 32 ob + 16 t + 8(j/4) + 4(l/32) + j%4 (j = 0..7) of the next layer; the
// packed weights of layers 2..4 follow that order, so no data moves
// between layers.
//
// Weight fragments: [ks][ob][lane][8] per layer, ks = K-step of 16, ob =
// output block of 32 (a slice of K-steps is contiguous); biases
// [ob][l/32][16] in the register order above.
#include "pyro_internal.h"
#include "mlp_internal.h"
#include "surrogate_internal.h"

namespace pyro {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kCells = 32;                 // cells per wavefront
constexpr int kFeatRow = kFeatPad + 8;     // padded LDS feature row (bf16)
// wavefronts per workgroup (they share the weights)
__host__ __device__ constexpr int waves_per_block(int) { return 4; }

// LDS: feature rows, two weight slices of the widest layer
__host__ __device__ constexpr size_t fused_lds_bytes_ks(int H, int members, int slice_ks) {
    return size_t(waves_per_block(members)) * kCells * kFeatRow * 2 +
           2 * size_t(slice_ks) * (H / 32) * 64 * 16;
}
// K-steps per staged weight slice: as many as let two slices fit (one
// barrier per slice)
__host__ __device__ constexpr int slice_ks(int H, int members) {
    return fused_lds_bytes_ks(H, members, 8) <= 160 * 1024 ? 8
         : fused_lds_bytes_ks(H, members, 4) <= 160 * 1024 ? 4 : 2;
}
__host__ __device__ constexpr size_t fused_lds_bytes(int H, int members) {
    return fused_lds_bytes_ks(H, members, slice_ks(H, members));
}

// sinh in FP64 from one exponential: (e - 1/e)/2 with e = exp(|x|) for
// |x| >= 1/2 (the subtraction loses at most coth(1/2) < 2.2 in relative
// terms), the odd Taylor series through x^17 below (truncation < 1e-22
// relative); 1/e is the hardware reciprocal refined by two Newton steps, and
// zero once e has overflowed.  A few ulps, where the library sinh also works
// in extended precision.
__device__ inline double sinh_d(double x) {
    const double ax = fabs(x);
    const double e = exp(ax);
    double r = __builtin_amdgcn_rcp(e);
    r = fma(r, fma(-e, r, 1.0), r);
    r = fma(r, fma(-e, r, 1.0), r);
    const double big = 0.5 * (e - (e < 0x1p1020 ? r : 0.0));
    const double x2 = x * x;
    double t = 1.0 / 355687428096000.0;                  // 1/17!
    t = fma(t, x2, 1.0 / 1307674368000.0);               // 1/15!
    t = fma(t, x2, 1.0 / 6227020800.0);                  // 1/13!
    t = fma(t, x2, 1.0 / 39916800.0);                    // 1/11!
    t = fma(t, x2, 1.0 / 362880.0);                      // 1/9!
    t = fma(t, x2, 1.0 / 5040.0);                        // 1/7!
    t = fma(t, x2, 1.0 / 120.0);                         // 1/5!
    t = fma(t, x2, 1.0 / 6.0);                           // 1/3!
    const double small = fma(ax * x2, t, ax);
    return copysign(ax < 0.5 ? small : big, x);
}

// packed-fragment sizes (elements) of one member for hidden width H
__host__ __device__ constexpr int64_t frag_elems(int nb, int ks) { return int64_t(nb) * ks * 64 * 8; }

struct PackLayout {
    int64_t w_off[4], b_off[4];
    int nb[4], ks[4];
    __host__ __device__ explicit PackLayout(int H) {
        const int K[4] = {kFeatPad, H, H, H}, N[4] = {H, H, H, kOutPad};
        int64_t ow = 0, ob = 0;
        for (int l = 0; l < 4; ++l) {
            nb[l] = N[l] / 32;
            ks[l] = K[l] / 16;
            w_off[l] = ow;
            b_off[l] = ob;
            ow += frag_elems(nb[l], ks[l]);
            ob += N[l];
        }
    }
};

// input index of K-slot (8 h + j) of K-step ks: natural for the feature
// layer, the register order of the previous layer's outputs otherwise
__host__ __device__ inline int input_index(int layer, int ks, int h, int j) {
    if (layer == 0) return 16 * ks + 8 * h + j;
    return 32 * (ks >> 1) + 16 * (ks & 1) + 8 * (j >> 2) + 4 * h + (j & 3);
}

// output index of register i in block ob for lane half h
__host__ __device__ inline int output_index(int ob, int h, int i) {
    return 32 * ob + 8 * (i >> 2) + 4 * h + (i & 3);
}

__global__ void pack_kernel(int H, int members, int64_t w_total, int64_t b_total,
                            const uint16_t* __restrict__ W, const float* __restrict__ b,
                            uint16_t* __restrict__ wp, float* __restrict__ bp) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const PackLayout P(H);
    const int K[4] = {kFeatPad, H, H, H}, N[4] = {H, H, H, kOutPad};
    if (t < w_total * members) {
        const int e = int(t / w_total);
        const int64_t p = t % w_total;
        int l = 3;
        while (l > 0 && p < P.w_off[l]) --l;
        const int64_t q = p - P.w_off[l];
        const int j = int(q & 7), lane = int((q >> 3) & 63);
        const int64_t frag = q >> 9;
        const int ob = int(frag % P.nb[l]), ks = int(frag / P.nb[l]);
        // natural weights of layer l: [K][N] row-major after the previous layers
        int64_t nat = 0;
        for (int i = 0; i < l; ++i) nat += int64_t(K[i]) * N[i];
        const int in = input_index(l, ks, lane >> 5, j), out = 32 * ob + (lane & 31);
        wp[t] = W[e * w_total + nat + int64_t(in) * N[l] + out];
    }
    if (t < b_total * members) {
        const int e = int(t / b_total);
        const int64_t p = t % b_total;
        int l = 3;
        while (l > 0 && p < P.b_off[l]) --l;
        const int q = int(p - P.b_off[l]);
        const int ob = q >> 5, h = (q >> 4) & 1, i = q & 15;
        bp[t] = b[e * b_total + P.b_off[l] + output_index(ob, h, i)];
    }
}

struct FusedArgs {
    const uint16_t* wp;    // packed weights, members after one another
    const float* bp;       // packed biases
    int64_t w_stride, b_stride;
    const float* shift;
    const float* scale;
    float* zout;           // raw mode: [members][n][64]; else [members][S][n]
};

// One layer for the wavefront's 32 cells: acc = bias + W^T in, with the
// weight slices staged through LDS by the whole workgroup (NT threads).
// Every call ends with a barrier, so the next call may refill both buffers.
template <int NB, int KS, int NT, int SKS>
__device__ inline void layer(f32x16 (&acc)[NB], const bf16x8 (&in)[KS],
                             const uint16_t* __restrict__ wp, const float* __restrict__ bp,
                             u32x4* wbuf, int lane, int tid) {
    constexpr int kSliceKs = SKS < KS ? SKS : KS;       // a slice never spans layers
    constexpr int kUnits = kSliceKs * NB * 64;          // 16-byte fragments per slice
    constexpr int kPer = kUnits / NT;                   // per thread
    constexpr int kSlices = KS / kSliceKs;
    static_assert(KS % kSliceKs == 0, "K-steps come in whole slices");
    // every thread copies the same number of fragments: no per-lane
    // conditions (the compiler cannot prove tid < NT, and a guarded copy
    // becomes an exec-masked load waited on at once)
    static_assert(kUnits % NT == 0, "a slice is a whole number of fragments per thread");
    const int h = lane >> 5;
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) {
        const float4* bq = reinterpret_cast<const float4*>(bp + ob * 32 + h * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v = bq[q];
            acc[ob][4 * q] = v.x;
            acc[ob][4 * q + 1] = v.y;
            acc[ob][4 * q + 2] = v.z;
            acc[ob][4 * q + 3] = v.w;
        }
    }
    const u32x4* src = reinterpret_cast<const u32x4*>(wp);
#pragma unroll
    for (int j = 0; j < kPer; ++j) wbuf[tid + j * NT] = src[tid + j * NT];
    __syncthreads();
#pragma unroll
    for (int sl = 0; sl < kSlices; ++sl) {
        const u32x4* cur = wbuf + (sl & 1) * kUnits;
        u32x4* nxt = wbuf + ((sl + 1) & 1) * kUnits;
        u32x4 pre[kPer];
        if (sl + 1 < kSlices) {
#pragma unroll
            for (int j = 0; j < kPer; ++j) pre[j] = src[(sl + 1) * kUnits + tid + j * NT];
        }
        // the fragments of K-step kk + 1 are read while those of kk multiply
        // (one LDS latency per slice instead of one per MFMA)
        u32x4 f[2][NB];
#pragma unroll
        for (int ob = 0; ob < NB; ++ob) f[0][ob] = cur[ob * 64 + lane];
#pragma unroll
        for (int kk = 0; kk < kSliceKs; ++kk) {
            if (kk + 1 < kSliceKs) {
#pragma unroll
                for (int ob = 0; ob < NB; ++ob)
                    f[(kk + 1) & 1][ob] = cur[((kk + 1) * NB + ob) * 64 + lane];
            }
#pragma unroll
            for (int ob = 0; ob < NB; ++ob)
                acc[ob] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    __builtin_bit_cast(bf16x8, f[kk & 1][ob]), in[sl * kSliceKs + kk], acc[ob],
                    0, 0, 0);
        }
        // pin that order for the scheduler (it otherwise sinks every read to
        // its MFMA and waits on it there): K-step 0's reads, then per K-step
        // the next one's reads followed by this one's MFMAs
        __builtin_amdgcn_sched_group_barrier(0x100, NB, 0);
#pragma unroll
        for (int kk = 0; kk < kSliceKs; ++kk) {
            if (kk + 1 < kSliceKs) __builtin_amdgcn_sched_group_barrier(0x100, NB, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, NB, 0);
        }
        if (sl + 1 < kSlices) {
#pragma unroll
            for (int j = 0; j < kPer; ++j) nxt[tid + j * NT] = pre[j];
        }
        __syncthreads();
    }
}

// bias-added outputs -> SiLU -> BF16 inputs of the next layer
template <int NB>
__device__ inline void activate(const f32x16 (&acc)[NB], bf16x8 (&out)[2 * NB]) {
#pragma unroll
    for (int ob = 0; ob < NB; ++ob)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            u32x4 packed;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                packed[q] = f2bf2(silu(acc[ob][8 * t + 2 * q]), silu(acc[ob][8 * t + 2 * q + 1]));
            out[2 * ob + t] = __builtin_bit_cast(bf16x8, packed);
        }
}

template <int H, int E, bool RAW>
__global__ __launch_bounds__(waves_per_block(E) * 64) void fused_kernel(
    DevMech m, int64_t n, int64_t ld, const double* __restrict__ rho,
    const double* __restrict__ T, const double* __restrict__ Y, FusedArgs a) {
    constexpr int NBH = H / 32, KSH = H / 16;
    constexpr int WPB = waves_per_block(E), NT = WPB * 64, SKS = slice_ks(H, E);
    // LDS: feature rows [wave][cell][kFeatRow] (BF16), then two weight
    // slices
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    uint16_t* feat = reinterpret_cast<uint16_t*>(lds) + wv * kCells * kFeatRow;
    u32x4* wbuf = reinterpret_cast<u32x4*>(lds + WPB * kCells * kFeatRow * 2);
    // every wavefront takes part in the weight staging and its barriers;
    // cells past n compute on cell n - 1 and write nothing
    const int64_t c0 = (int64_t(blockIdx.x) * WPB + wv) * kCells;
    const int cl = lane & 31, h = lane >> 5;
    const int64_t cell = c0 + cl;
    const bool valid = cell < n;
    const int64_t c = valid ? cell : n - 1;

    // ---- features of the 32 cells, staged in this wave's LDS rows; lane
    // half h converts the species k = h, h + 2, ...  All of the lane's mass
    // fractions are loaded before any is used (one memory latency per wave
    // instead of one per species: this phase runs at the MLP's occupancy).
    constexpr int kHalfSpecies = (kFeatPad - 2) / 2;   // species per lane half
    uint16_t* fr = feat + cl * kFeatRow;
    const double Tc = T[c];
    double yv[kHalfSpecies];
#pragma unroll
    for (int i = 0; i < kHalfSpecies; ++i) {
        const int k = h + 2 * i;
        yv[i] = k < m.S ? Y[size_t(k) * ld + c] : 0.0;
    }
    double x = 0.0;  // partial 1/W
#pragma unroll
    for (int i = 0; i < kHalfSpecies; ++i) {
        const int k = h + 2 * i;
        if (k < m.S) {
            x = fma(yv[i], m.newton[k].inv_w, x);
            fr[k + 2] = f2bf(float((log(fmax(yv[i], 0.0) + 1e-12) - a.shift[k + 2]) * a.scale[k + 2]));
        }
    }
    x += __shfl_xor(x, 32);
    if (h == 0) {
        const double p = rho[c] * kGasConstant * Tc * x;
        fr[0] = f2bf(float((Tc * 1e-3 - a.shift[0]) * a.scale[0]));
        fr[1] = f2bf(float((log10(p) - a.shift[1]) * a.scale[1]));
    } else {
        for (int f = m.S + 2; f < kFeatPad; ++f) fr[f] = f == m.S + 2 ? uint16_t(0x3f80) : uint16_t(0);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    bf16x8 xb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) xb[s] = *reinterpret_cast<const bf16x8*>(fr + 16 * s + 8 * h);

    // ---- ensemble members (the loop stays rolled: one member's code is
    // already 320 MFMAs)
#pragma nounroll
    for (int e = 0; e < E; ++e) {
        const PackLayout P(H);
        const uint16_t* wp = a.wp + e * a.w_stride;
        const float* bp = a.bp + e * a.b_stride;
        f32x16 acc[NBH];
        bf16x8 act[KSH];
        layer<NBH, 4, NT, SKS>(acc, xb, wp + P.w_off[0], bp + P.b_off[0], wbuf, lane, tid);
        activate<NBH>(acc, act);
        layer<NBH, KSH, NT, SKS>(acc, act, wp + P.w_off[1], bp + P.b_off[1], wbuf, lane, tid);
        activate<NBH>(acc, act);
        layer<NBH, KSH, NT, SKS>(acc, act, wp + P.w_off[2], bp + P.b_off[2], wbuf, lane, tid);
        activate<NBH>(acc, act);
        f32x16 z[2];
        layer<2, KSH, NT, SKS>(z, act, wp + P.w_off[3], bp + P.b_off[3], wbuf, lane, tid);
        // register i of block ob holds output k = output_index(ob, h, i):
        // species-major stores are two 128-byte runs of cells per register
        if (valid) {
#pragma unroll
            for (int ob = 0; ob < 2; ++ob)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int k = output_index(ob, h, i);
                    if constexpr (RAW) {
                        a.zout[(int64_t(e) * n + cell) * kOutPad + k] = z[ob][i];
                    } else if (k < m.S) {
                        a.zout[(int64_t(e) * m.S + k) * n + cell] = z[ob][i];
                    }
                }
        }
    }
}

// Ensemble mean, inverse target transform and indicators of one cell per
// thread from the staged member outputs z [E][S][n]: omega_k = s_k
// sinh(sigma_k zbar_k + mu_k) with zbar the FP32 mean of the members;
// spread = sqrt(sum_e sum_k (omega_ek - omega_k)^2 / E) / ||omega||;
// residual = ||A omega|| / || |A| |omega| ||; flag = 0 only where all are
// finite and both indicators are under their thresholds.
template <int E>
__global__ __launch_bounds__(256) void post_kernel(DevMech m, int64_t n, int64_t ld,
                                                   const float* __restrict__ z,
                                                   const double* __restrict__ ts,
                                                   const double* __restrict__ tmu,
                                                   const double* __restrict__ tsig,
                                                   double thr_spread, double thr_resid,
                                                   double* __restrict__ wdot,
                                                   uint8_t* __restrict__ flag,
                                                   double* __restrict__ ind) {
    const int64_t cell = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (cell >= n) return;
    const float inv_e = 1.0f / float(E);
    const cptr<double> cs = cst(ts), cm = cst(tmu), cg = cst(tsig);
    double r[kMaxElements], q[kMaxElements];
#pragma unroll
    for (int el = 0; el < kMaxElements; ++el) r[el] = q[el] = 0.0;
    double mean2 = 0.0, dev2 = 0.0;
    bool finite = true;
    for (int k = 0; k < m.S; ++k) {
        float ze[E];
        float zs = 0.0f;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            ze[e] = z[(int64_t(e) * m.S + k) * n + cell];
            zs += ze[e];
        }
        const double s = cs[k], mu = cm[k], sg = cg[k];
        const double w = s * sinh_d(fma(sg, double(zs * inv_e), mu));
        finite = finite && isfinite(w);
        mean2 = fma(w, w, mean2);
        if (E > 1) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double d = s * sinh_d(fma(sg, double(ze[e]), mu)) - w;
                dev2 = fma(d, d, dev2);
            }
        }
        wdot[size_t(k) * ld + cell] = w;
        const cptr<double> ce = cst(m.comp) + k;
#pragma unroll
        for (int el = 0; el < kMaxElements; ++el)
            if (el < m.E) {
                const double ak = ce[size_t(el) * m.S];
                r[el] = fma(ak, w, r[el]);
                q[el] = fma(fabs(ak), fabs(w), q[el]);
            }
    }
    double r2 = 0.0, q2 = 0.0;
#pragma unroll
    for (int el = 0; el < kMaxElements; ++el)
        if (el < m.E) {
            r2 = fma(r[el], r[el], r2);
            q2 = fma(q[el], q[el], q2);
        }
    const double spread = sqrt(dev2 / E) / fmax(sqrt(mean2), 1e-300);
    const double resid = q2 > 0.0 ? sqrt(r2 / q2) : 0.0;
    flag[cell] = (finite && spread < thr_spread && resid < thr_resid) ? 0 : 1;
    if (ind) {
        ind[cell] = spread;
        ind[n + cell] = resid;
    }
}

template <int H, int E>
hipError_t launch_fused_he(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                           const double* T, const double* Y, const FusedArgs& a, bool raw,
                           hipStream_t stream) {
    constexpr int WPB = waves_per_block(E);
    const int64_t waves = (n + kCells - 1) / kCells;
    const dim3 grid(unsigned((waves + WPB - 1) / WPB));
    const size_t lds = fused_lds_bytes(H, E);
    const void* fn = raw ? reinterpret_cast<const void*>(&fused_kernel<H, E, true>)
                         : reinterpret_cast<const void*>(&fused_kernel<H, E, false>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    if (raw)
        hipLaunchKernelGGL((fused_kernel<H, E, true>), grid, dim3(WPB * 64), lds,
                           stream, m->dev, n, ld, rho, T, Y, a);
    else
        hipLaunchKernelGGL((fused_kernel<H, E, false>), grid, dim3(WPB * 64), lds,
                           stream, m->dev, n, ld, rho, T, Y, a);
    return hipGetLastError();
}

template <int E>
hipError_t launch_post_e(const pyro_mech* m, int64_t n, int64_t ld, const float* z,
                         const double* ts, const double* tmu, const double* tsig,
                         double thr_spread, double thr_resid, double* wdot, uint8_t* flag,
                         double* ind, hipStream_t stream) {
    hipLaunchKernelGGL(post_kernel<E>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream,
                       m->dev, n, ld, z, ts, tmu, tsig, thr_spread, thr_resid, wdot, flag, ind);
    return hipGetLastError();
}

template <int H>
hipError_t launch_fused_h(const pyro_mech* m, int members, int64_t n, int64_t ld,
                          const double* rho, const double* T, const double* Y, const FusedArgs& a,
                          bool raw, hipStream_t stream) {
    switch (members) {
        case 1: return launch_fused_he<H, 1>(m, n, ld, rho, T, Y, a, raw, stream);
        case 2: return launch_fused_he<H, 2>(m, n, ld, rho, T, Y, a, raw, stream);
        case 3: return launch_fused_he<H, 3>(m, n, ld, rho, T, Y, a, raw, stream);
        default: return launch_fused_he<H, 4>(m, n, ld, rho, T, Y, a, raw, stream);
    }
}

}  // namespace

bool fused_supported(int hidden) { return hidden == 64 || hidden == 128 || hidden == 256; }

int64_t packed_weight_elems(int hidden) {
    const PackLayout P(hidden);
    return P.w_off[3] + frag_elems(P.nb[3], P.ks[3]);
}

hipError_t launch_pack(int hidden, int members, int64_t w_total, int64_t b_total,
                       const uint16_t* W, const float* b, uint16_t* wp, float* bp,
                       hipStream_t stream) {
    const int64_t count = (w_total > b_total ? w_total : b_total) * members;
    hipLaunchKernelGGL(pack_kernel, dim3(unsigned((count + 255) / 256)), dim3(256), 0, stream,
                       hidden, members, w_total, b_total, W, b, wp, bp);
    return hipGetLastError();
}

hipError_t launch_fused(const pyro_mech* m, int hidden, int members, int64_t n, int64_t ld,
                        const double* rho, const double* T, const double* Y,
                        const uint16_t* wp, const float* bp, int64_t w_stride, int64_t b_stride,
                        const float* shift, const float* scale, const double* ts,
                        const double* tmu, const double* tsig, double thr_spread,
                        double thr_resid, double* wdot, uint8_t* flag, double* ind, float* zout,
                        float* zstage, hipStream_t stream) {
    const bool raw = zout != nullptr;
    FusedArgs a{wp, bp, w_stride, b_stride, shift, scale, raw ? zout : zstage};
    hipError_t e;
    switch (hidden) {
        case 64: e = launch_fused_h<64>(m, members, n, ld, rho, T, Y, a, raw, stream); break;
        case 128: e = launch_fused_h<128>(m, members, n, ld, rho, T, Y, a, raw, stream); break;
        default: e = launch_fused_h<256>(m, members, n, ld, rho, T, Y, a, raw, stream);
    }
    if (e != hipSuccess || raw) return e;
    switch (members) {
        case 1: return launch_post_e<1>(m, n, ld, zstage, ts, tmu, tsig, thr_spread, thr_resid, wdot, flag, ind, stream);
        case 2: return launch_post_e<2>(m, n, ld, zstage, ts, tmu, tsig, thr_spread, thr_resid, wdot, flag, ind, stream);
        case 3: return launch_post_e<3>(m, n, ld, zstage, ts, tmu, tsig, thr_spread, thr_resid, wdot, flag, ind, stream);
        default: return launch_post_e<4>(m, n, ld, zstage, ts, tmu, tsig, thr_spread, thr_resid, wdot, flag, ind, stream);
    }
}

}  // namespace pyro
