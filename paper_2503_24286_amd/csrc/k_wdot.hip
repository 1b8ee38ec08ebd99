// Net production rates omega(rho, T, Y) for a tile of 64 cells per
// workgroup (Appendix A.1: eq. concentrations, eq. nasa_poly, eq. gibbs,
// eq. rate_coeff, eq. equil_constants, eq. reaction_rates,
// eq. production_rates).
//
// Mapping on CDNA4: one cell per lane, eight wavefronts per workgroup, all
// lanes of a wave on the same species or reaction at the same time, so every
// mechanism-table read is wave-uniform and goes through the scalar cache.
//
//  1. species phase: each wave computes, for the species it owns,
//     C_k = rho max(Y_k, 0)/W_k and G_k = exp(g0_k/(R T)) and parks them in
//     LDS row k (C in the first 512 bytes, G in the second, so that both load
//     with one ds_read2 and neither access has bank conflicts);
//  2. third-body concentrations: each wave forms [M]_j = sum_k eps_jk C_k for
//     the third-body and falloff reactions it evaluates, in one pass over the
//     species, and keeps them in registers;
//  3. reaction phase, in chunks of 16 reactions (2 per wave): the forward
//     coefficient k = exp(ln A + b ln T - Ea/(R T)), falloff corrections, and
//     the rate of progress
//         q = k prod_r C_r - k (R T/p0)^dnu prod_p (C_p G_p) / prod_r G_r,
//     which is eq. reaction_rates with 1/K = (R T/p0)^dnu prod G^nu; q goes to
//     an LDS slot of the chunk (double buffered);
//  4. after the chunk barrier, each wave adds nu_kj q_j into register
//     accumulators of the species it owns, in a fixed order (deterministic);
//  5. the owners write omega_k for the 64 cells (coalesced 512-byte rows).
//
// The equilibrium constant of every reaction thus costs products of S
// per-species exponentials instead of one exponential per reaction.
//
// Reaction-equilibrium variant (RKC): g0/(R T) is linear in the NASA7
// coefficients, so for a reaction whose species share one T_mid,
// sum_k nu_kj g0_k/(R T) is a single polynomial with the combined
// coefficients sum_k nu_kj a_k (prepared by the loader).  The reverse rate is
// then k exp(dg_j) (R T/p0)^dnu prod_p C_p with one exponential per
// reversible reaction, and LDS holds C only (half the bytes per species),
// which lets large mechanisms fit and raises occupancy.
//
// MFMA third-body variant (MM): [M]_j = sum_k eps_jk C_k is a dense
// contraction (every species has an efficiency), computed for the whole tile
// as M[64 cells x n_pd] = C[64 x S] eps^T[S x n_pd] with v_mfma_f64_16x16x4f64
// (A = C from the LDS rows, B = pre-packed eps^T fragments), written to LDS
// once per tile; the waves then read [M] of their reactions from there.
#include "pyro_internal.h"

namespace pyro {
namespace {

constexpr int kRow = kTile * 16;          // bytes per species row: C[64] then G[64]
constexpr int kRowC = kTile * 8;          // RKC variant: C[64]

struct CG {
    double c, g;
};

__device__ inline CG lds_cg(const unsigned char* lds, int off, int lane) {
    const double* p = reinterpret_cast<const double*>(lds + off) + lane;
    return CG{p[0], p[kTile]};
}

// 1/x from the hardware estimate refined by two Newton steps
// r <- r + r (1 - x r); each step squares the relative error.
__device__ inline double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// g0/(R T) = c0 (1 - ln T) + c1 T + c2 T^2 + c3 T^3 + c4 T^4 + c5/T + c6.
__device__ inline double gibbs_poly(const double* c, double T, double omlnT, double invT) {
    return fma(c[0], omlnT, fma(c[5], invT, c[6])) +
           T * fma(T, fma(T, fma(T, c[4], c[3]), c[2]), c[1]);
}

// ln k of the Arrhenius triple in row ``row`` of ``params``.
__device__ inline double log_arrhenius(const double* __restrict__ params, int row, double lnT,
                                       double invRT) {
    const double* p = params + 3 * row;
    return fma(-p[2], invRT, fma(p[1], lnT, p[0]));
}

// Head of the wave's queue of third-body concentrations; the queue is
// popped by shifting, so the values stay in registers with static indices.
template <int N>
__device__ inline double pop_front(double (&v)[N]) {
    const double head = v[0];
#pragma unroll
    for (int i = 0; i + 1 < N; ++i) v[i] = v[i + 1];
    return head;
}

// C of the species at byte offset ``off`` of a species row (RKC rows are
// half as long as the C/G rows the offsets are given for)
__device__ inline double lds_c(const unsigned char* lds, int off, int lane) {
    return reinterpret_cast<const double*>(lds + (off >> 1))[lane];
}

// Rate of progress of one reaction for the calling lane's cell, given its
// Arrhenius coefficient kf and, for third-body and falloff reactions, [M].
// RKC: ``kc`` holds the reaction's combined Gibbs coefficients (low range,
// high range, T_mid).
template <bool RKC>
__device__ inline double rate_of_progress(const DevMech& m, const RxnRec& r,
                                          const double* __restrict__ params,
                                          const unsigned char* lds, int lane, double kf,
                                          double M, double Tc, double lnT, double invT,
                                          double invRT, double rtp, double irtp,
                                          cptr<double> kc) {
    if (r.cls >= kLindemann) {
        const double k0 = exp(log_arrhenius(params, m.R + r.fo, lnT, invRT));
        const double Pr = k0 * M / kf;
        double F = 1.0;
        if (r.cls == kTroe) {
            const FalloffRec f = m.falloff[r.fo];
            double Fcent = (1.0 - f.alpha) * exp(Tc * f.a3) + f.alpha * exp(Tc * f.a1) +
                           exp(f.a2 * invT);
            Fcent = fmax(Fcent, 1e-300);
            const double lfc = log10(Fcent);
            const double c = -0.4 - 0.67 * lfc;
            const double nn = 0.75 - 1.27 * lfc;
            const double x = log10(fmax(Pr, 1e-300)) + c;
            const double f1 = x / (nn - 0.14 * x);
            F = exp10(lfc / (1.0 + f1 * f1));
        }
        kf = kf * (Pr / (1.0 + Pr)) * F;
    }
    if constexpr (RKC) {
        double cr = lds_c(lds, r.r[0], lane);
        if (r.nr > 1) {
            cr *= lds_c(lds, r.r[1], lane);
            if (r.nr > 2) cr *= lds_c(lds, r.r[2], lane);
        }
        double q = kf * cr;
        if (r.rev) {
            double cp = lds_c(lds, r.p[0], lane);
            if (r.np > 1) {
                cp *= lds_c(lds, r.p[1], lane);
                if (r.np > 2) cp *= lds_c(lds, r.p[2], lane);
            }
            double pw = 1.0;
            if (r.dnu > 0)
                for (int i = 0; i < r.dnu; ++i) pw *= rtp;
            else
                for (int i = 0; i < -r.dnu; ++i) pw *= irtp;
            const double lo[7] = {kc[0], kc[1], kc[2], kc[3], kc[4], kc[5], kc[6]};
            const double hi[7] = {kc[7], kc[8], kc[9], kc[10], kc[11], kc[12], kc[13]};
            const double omlnT = 1.0 - lnT;
            const double d_lo = gibbs_poly(lo, Tc, omlnT, invT);
            const double d_hi = gibbs_poly(hi, Tc, omlnT, invT);
            q -= kf * pw * exp(Tc <= kc[14] ? d_lo : d_hi) * cp;
        }
        if (r.cls == kThirdBody) q *= M;
        return q;
    }
    // forward term k prod_r C_r
    CG a = lds_cg(lds, r.r[0], lane);
    double cr = a.c, gr = a.g;
    if (r.nr > 1) {
        const CG b = lds_cg(lds, r.r[1], lane);
        cr *= b.c;
        gr *= b.g;
        if (r.nr > 2) {
            const CG c = lds_cg(lds, r.r[2], lane);
            cr *= c.c;
            gr *= c.g;
        }
    }
    double q = kf * cr;
    if (r.rev) {
        const CG p = lds_cg(lds, r.p[0], lane);
        double cgp = p.c * p.g;
        if (r.np > 1) {
            const CG b = lds_cg(lds, r.p[1], lane);
            cgp *= b.c * b.g;
            if (r.np > 2) {
                const CG c = lds_cg(lds, r.p[2], lane);
                cgp *= c.c * c.g;
            }
        }
        double pw = 1.0;
        if (r.dnu > 0)
            for (int i = 0; i < r.dnu; ++i) pw *= rtp;
        else
            for (int i = 0; i < -r.dnu; ++i) pw *= irtp;
        q -= kf * pw * cgp * recip(gr);
    }
    if (r.cls == kThirdBody) q *= M;
    return q;
}

typedef double d4 __attribute__((ext_vector_type(4)));

template <int WAVES, int MAXOWN, int MAXPD, bool RKC, bool MM, bool NQ>
__global__ __launch_bounds__(WAVES * 64) void wdot_f64_kernel(
    DevMech m, int64_t n, int64_t ld, const double* __restrict__ rho,
    const double* __restrict__ T, const double* __restrict__ Y,
    double* __restrict__ wdot, const double* __restrict__ params,
    const int64_t* __restrict__ n_dev) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    if (n_dev) {
        n = *n_dev;  // cells counted on the device (the whole workgroup agrees)
        if (int64_t(blockIdx.x) * kTile >= n) return;
    }
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t cell = int64_t(blockIdx.x) * kTile + lane;
    const bool valid = cell < n;
    const int64_t c = valid ? cell : n - 1;

    const double Tc = T[c];
    const double rc = rho[c];
    const double lnT = log(Tc);
    const double invT = 1.0 / Tc;
    const double invRT = invT * (1.0 / kGasConstant);
    const double rtp = kGasConstant * Tc / kOneAtm;
    const double irtp = 1.0 / rtp;
    const double omlnT = 1.0 - lnT;

    // ---- species phase: all of this wave's mass-fraction loads first
    const int nown = m.n_own[w];
    const int32_t* own = m.own + w * kMaxOwn;
    double y[MAXOWN];
#pragma unroll
    for (int i = 0; i < MAXOWN; ++i)
        if (i < nown) y[i] = Y[size_t(own[i]) * ld + c];
#pragma unroll
    for (int i = 0; i < MAXOWN; ++i) {
        if (i < nown) {
            const int k = own[i];
            const SpeciesRec& s = m.species[k];
            const double Ck = rc * fmax(y[i], 0.0) * s.inv_w;
            if constexpr (RKC) {
                reinterpret_cast<double*>(lds + k * kRowC)[lane] = Ck;
            } else {
                // both ranges from scalar loads, then a per-lane select of the
                // value (selecting the coefficient address would turn the
                // uniform table reads into per-lane vector loads)
                const double g_lo = gibbs_poly(s.lo, Tc, omlnT, invT);
                const double g_hi = gibbs_poly(s.hi, Tc, omlnT, invT);
                const double gRT = Tc <= s.t_mid ? g_lo : g_hi;
                double* row = reinterpret_cast<double*>(lds + k * kRow) + lane;
                row[0] = Ck;
                row[kTile] = exp(gRT);
            }
        }
    }
    __syncthreads();

    constexpr int rowb = RKC ? kRowC : kRow;
    unsigned char* qbase = lds + size_t(m.S) * rowb;
    constexpr int qbuf = WAVES * kRxnPerWave * kTile * 8;     // bytes per chunk buffer
    static_assert(!NQ || WAVES == kWaves, "the MFMA net rates assume kWaves wavefronts");
    double* Ml = reinterpret_cast<double*>(qbase + 2 * qbuf);  // MM: [n_pd16][64]
    if constexpr (MM) {
        // ---- the tile's third-body concentrations on the matrix cores: wave w
        // takes the 16-cell x 16-reaction output blocks w, w + 8, ...
        const int n_pb = (m.n_pd + 15) / 16, n_ks = (m.S + 3) / 4;
        for (int t = w; t < 4 * n_pb; t += WAVES) {
            const int cb = t & 3, pb = t >> 2;
            const double* eb = m.eps_frag + size_t(pb) * n_ks * 64 + lane;
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int kk = 0; kk < n_ks; ++kk) {
                const int k = 4 * kk + (lane >> 4);
                const double a = k < m.S
                    ? reinterpret_cast<const double*>(lds + k * rowb)[16 * cb + (lane & 15)] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, eb[size_t(kk) * 64], acc, 0, 0, 0);
            }
            // D: register i of lane l is cell 4 i + l/16, reaction l % 16 of the block
#pragma unroll
            for (int i = 0; i < 4; ++i)
                Ml[(16 * pb + (lane & 15)) * kTile + 16 * cb + 4 * i + (lane >> 4)] = acc[i];
        }
        __syncthreads();
    }

    // ---- third-body concentrations of this wave's reactions
    double Mr[MAXPD];
#pragma unroll
    for (int i = 0; i < MAXPD; ++i) Mr[i] = 0.0;
    if (!MM && m.n_pdw[w] > 0) {
        const double* ew = m.effw + size_t(w) * m.S * MAXPD;
        for (int k = 0; k < m.S; ++k) {
            const double ck = reinterpret_cast<const double*>(lds + k * rowb)[lane];
#pragma unroll
            for (int i = 0; i < MAXPD; ++i) Mr[i] = fma(ew[k * MAXPD + i], ck, Mr[i]);
        }
    }

    // ---- reaction chunks and gathering
    double acc[NQ ? 1 : MAXOWN];
#pragma unroll
    for (int i = 0; i < (NQ ? 1 : MAXOWN); ++i) acc[i] = 0.0;
    // NQ: omega[64 cells x S] accumulated on the matrix cores over the chunks,
    // omega += q[cells x 16 slots] nu[16 slots x S]; wave w holds the
    // 16-cell x 16-species output blocks (cell block w & 3, species blocks
    // (w >> 2) and (w >> 2) + 2)
    const int nq_cb = w & 3, nq_sb = w >> 2;
    d4 wacc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    static_assert(kRxnPerWave == 2, "the reaction phase handles reactions in pairs");
    for (int ch = 0; ch < m.n_chunks; ++ch) {
        unsigned char* qb = qbase + (ch & 1) * qbuf;
        // NQ: this chunk's B fragments of nu, loaded before the rates are evaluated
        double nub[2][4];
        if constexpr (NQ) {
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    nub[b][kk] = m.nu_frag[((size_t(ch) * 4 + nq_sb + 2 * b) * 4 + kk) * 64 + lane];
        }
        const RxnRec* rb = m.rxn + (size_t(ch) * WAVES + w) * kRxnPerWave;
        const RxnRec r0 = rb[0];
        const RxnRec r1 = rb[1];
        // both Arrhenius exponentials in one block, so they interleave
        const double kf0 = exp(log_arrhenius(params, r0.prow, lnT, invRT));
        const double kf1 = exp(log_arrhenius(params, r1.prow, lnT, invRT));
        // the wave meets its third-body/falloff reactions in queue order
        double M0 = 1.0, M1 = 1.0;
        if constexpr (MM) {
            if (r0.cls >= kThirdBody) M0 = Ml[r0.pd * kTile + lane];
            if (r1.cls >= kThirdBody) M1 = Ml[r1.pd * kTile + lane];
        } else {
            M0 = r0.cls >= kThirdBody ? pop_front(Mr) : 1.0;
            M1 = r1.cls >= kThirdBody ? pop_front(Mr) : 1.0;
        }
        const cptr<double> kc = cst(m.rxn_kc) + (size_t(ch) * WAVES + w) * kRxnPerWave * 16;
        if (r0.cls != kNoReaction)
            *reinterpret_cast<double*>(qb + r0.qoff + lane * 8) = rate_of_progress<RKC>(
                m, r0, params, lds, lane, kf0, M0, Tc, lnT, invT, invRT, rtp, irtp, kc);
        else if (NQ)   // empty slots enter the dense product: zero, not stale LDS
            *reinterpret_cast<double*>(qb + (2 * w) * kTile * 8 + lane * 8) = 0.0;
        if (r1.cls != kNoReaction)
            *reinterpret_cast<double*>(qb + r1.qoff + lane * 8) = rate_of_progress<RKC>(
                m, r1, params, lds, lane, kf1, M1, Tc, lnT, invT, invRT, rtp, irtp, kc + 16);
        else if (NQ)
            *reinterpret_cast<double*>(qb + (2 * w + 1) * kTile * 8 + lane * 8) = 0.0;
        __syncthreads();
        if constexpr (NQ) {
            // A[cell][slot]: slot 4 kk + l/16, cell 16 cb + l%16 of the chunk buffer
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const double a = reinterpret_cast<const double*>(
                    qb + (4 * kk + (lane >> 4)) * kTile * 8)[16 * nq_cb + (lane & 15)];
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    wacc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, nub[b][kk], wacc[b], 0, 0, 0);
            }
            continue;
        }
        // gather: the boundaries of all owned species in one scalar load,
        // then each species' entries in pairs
        const int32_t* gp = m.gptr + (size_t(ch) * WAVES + w) * (kMaxOwn + 1);
        int32_t bound[MAXOWN + 1];
#pragma unroll
        for (int i = 0; i <= MAXOWN; ++i) bound[i] = gp[i];
#pragma unroll
        for (int i = 0; i < MAXOWN; ++i) {
            if (i < nown) {
                double a = acc[i], b = 0.0;
                int e = bound[i];
                const int e1 = bound[i + 1];
                for (; e + 1 < e1; e += 2) {
                    const GatherEntry g0 = m.gent[e];
                    const GatherEntry g1 = m.gent[e + 1];
                    const double q0 = *reinterpret_cast<const double*>(qb + (g0 & 0xffffu) + lane * 8);
                    const double q1 = *reinterpret_cast<const double*>(qb + (g1 & 0xffffu) + lane * 8);
                    a = fma(double(int16_t(g0 >> 16)), q0, a);
                    b = fma(double(int16_t(g1 >> 16)), q1, b);
                }
                if (e < e1) {
                    const GatherEntry g0 = m.gent[e];
                    a = fma(double(int16_t(g0 >> 16)),
                            *reinterpret_cast<const double*>(qb + (g0 & 0xffffu) + lane * 8), a);
                }
                acc[i] = a + b;
            }
        }
    }
    if constexpr (NQ) {
        // D: register i of lane l is cell 4 i + l/16, species l % 16 of the block
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int k = 16 * (nq_sb + 2 * b) + (lane & 15);
            if (k < m.S) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t ci = int64_t(blockIdx.x) * kTile + 16 * nq_cb + 4 * i + (lane >> 4);
                    if (ci < n) wdot[size_t(k) * ld + ci] = wacc[b][i];
                }
            }
        }
    } else if (valid) {
#pragma unroll
        for (int i = 0; i < MAXOWN; ++i)
            if (i < nown) wdot[size_t(own[i]) * ld + cell] = acc[i];
    }
}

template <int WAVES, int MAXOWN, int MAXPD, bool RKC, bool MM, bool NQ>
hipError_t launch_f64(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                      const double* T, const double* Y, double* wdot,
                      const double* params, hipStream_t stream, const int64_t* n_dev) {
    const size_t lds = production_rates_lds_bytes(m, RKC, MM);
    const int64_t blocks = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL((wdot_f64_kernel<WAVES, MAXOWN, MAXPD, RKC, MM, NQ>), dim3(unsigned(blocks)),
                       dim3(WAVES * 64), lds, stream, m->dev, n, ld, rho, T, Y, wdot,
                       params ? params : m->dev.params, n_dev);
    return hipGetLastError();
}

// Kernel instances: (wavefronts, species owned per wave, [M] slots per wave,
// variant).  With 2 kWaves wavefronts (large mechanisms, reaction variant
// only) a wave owns at most 16 species.
template <int WAVES, int MAXOWN, int MAXPD, bool RKC, bool MM, bool NQ>
hipError_t set_lds(int bytes) {
    return hipFuncSetAttribute(
        reinterpret_cast<const void*>(&wdot_f64_kernel<WAVES, MAXOWN, MAXPD, RKC, MM, NQ>),
        hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// the NQ instances exist for at most 16 species per wave (NQ needs S <= 64)
template <int MAXPD, bool RKC, bool MM, bool NQ>
hipError_t dispatch_own(const pyro_mech* m, int64_t n, int64_t ld, const double* r,
                        const double* t, const double* y, double* o, const double* params,
                        hipStream_t stream, const int64_t* nd) {
    if constexpr (RKC && !NQ) {
        if (m->fw_waves != kWaves) {
            if (m->max_own <= 8)
                return launch_f64<2 * kWaves, 8, MAXPD, RKC, MM, false>(m, n, ld, r, t, y, o, params, stream, nd);
            return launch_f64<2 * kWaves, 16, MAXPD, RKC, MM, false>(m, n, ld, r, t, y, o, params, stream, nd);
        }
    }
    if (m->max_own <= 8) return launch_f64<kWaves, 8, MAXPD, RKC, MM, NQ>(m, n, ld, r, t, y, o, params, stream, nd);
    if (NQ || m->max_own <= 16)
        return launch_f64<kWaves, 16, MAXPD, RKC, MM, NQ>(m, n, ld, r, t, y, o, params, stream, nd);
    if (m->max_own <= 32) return launch_f64<kWaves, 32, MAXPD, RKC, MM, false>(m, n, ld, r, t, y, o, params, stream, nd);
    return launch_f64<kWaves, 64, MAXPD, RKC, MM, false>(m, n, ld, r, t, y, o, params, stream, nd);
}

template <bool RKC, bool MM, bool NQ>
hipError_t set_lds_variant(const pyro_mech* m, int bytes) {
    hipError_t e = hipSuccess;
    if constexpr (RKC && !NQ) {
        if (m->fw_waves != kWaves) {
            const hipError_t big[] = {
                set_lds<2 * kWaves, 8, 8, RKC, MM, false>(bytes),
                set_lds<2 * kWaves, 16, 8, RKC, MM, false>(bytes),
                MM ? hipSuccess : set_lds<2 * kWaves, 8, 16, RKC, MM, false>(bytes),
                MM ? hipSuccess : set_lds<2 * kWaves, 16, 16, RKC, MM, false>(bytes)};
            for (hipError_t x : big)
                if (x != hipSuccess) e = x;
            return e;
        }
    }
    // the MFMA third-body variant holds no per-wave [M] slots: one MAXPD instance
    const hipError_t all[] = {
        set_lds<kWaves, 8, 8, RKC, MM, NQ>(bytes),  set_lds<kWaves, 16, 8, RKC, MM, NQ>(bytes),
        NQ ? hipSuccess : set_lds<kWaves, 32, 8, RKC, MM, false>(bytes),
        NQ ? hipSuccess : set_lds<kWaves, 64, 8, RKC, MM, false>(bytes),
        MM ? hipSuccess : set_lds<kWaves, 8, 16, RKC, MM, NQ>(bytes),
        MM ? hipSuccess : set_lds<kWaves, 16, 16, RKC, MM, NQ>(bytes),
        MM || NQ ? hipSuccess : set_lds<kWaves, 32, 16, RKC, MM, false>(bytes),
        MM || NQ ? hipSuccess : set_lds<kWaves, 64, 16, RKC, MM, false>(bytes)};
    for (hipError_t x : all)
        if (x != hipSuccess) e = x;
    return e;
}

template <bool RKC, bool MM, bool NQ>
hipError_t dispatch_variant(const pyro_mech* m, int64_t n, int64_t ld, const double* r,
                            const double* t, const double* y, double* o, const double* params,
                            hipStream_t stream, const int64_t* nd) {
    if (MM || m->max_pdw <= 8) return dispatch_own<8, RKC, MM, NQ>(m, n, ld, r, t, y, o, params, stream, nd);
    return dispatch_own<16, RKC, MM, NQ>(m, n, ld, r, t, y, o, params, stream, nd);
}

}  // namespace

size_t production_rates_lds_bytes(const pyro_mech* m, bool reaction_equilibrium,
                                  bool mfma_third_body) {
    return size_t(m->S) * (reaction_equilibrium ? kRowC : kRow) +
           2 * size_t(m->fw_waves) * kRxnPerWave * kTile * 8 +
           (mfma_third_body ? size_t((m->n_tb + m->n_fo + 15) / 16 * 16) * kTile * 8 : 0);
}

hipError_t prepare_production_rates(const pyro_mech* m) {
    hipError_t e = hipSuccess;
    for (const int v : {0, 1, 2, 3, 4, 5, 6, 7}) {
        const bool rkc = v & 1, mm = v & 2, nq = v & 4;
        const size_t bytes = production_rates_lds_bytes(m, rkc, mm);
        if (bytes > 160 * 1024 || (rkc && !m->kc_ok) || (nq && !nq_supported(m))) continue;
        hipError_t x;
        switch (v) {
            case 0: x = set_lds_variant<false, false, false>(m, int(bytes)); break;
            case 1: x = set_lds_variant<true, false, false>(m, int(bytes)); break;
            case 2: x = set_lds_variant<false, true, false>(m, int(bytes)); break;
            case 3: x = set_lds_variant<true, true, false>(m, int(bytes)); break;
            case 4: x = set_lds_variant<false, false, true>(m, int(bytes)); break;
            case 5: x = set_lds_variant<true, false, true>(m, int(bytes)); break;
            case 6: x = set_lds_variant<false, true, true>(m, int(bytes)); break;
            default: x = set_lds_variant<true, true, true>(m, int(bytes));
        }
        if (x != hipSuccess) e = x;
    }
    return e;
}

bool nq_supported(const pyro_mech* m) {
    return m->S <= 64 && m->max_own <= 16 && m->fw_waves == kWaves;
}

hipError_t launch_production_rates(const pyro_mech* m, int64_t n, int64_t ld, int dtype,
                                   const void* rho, const void* T, const void* Y,
                                   void* wdot, const double* params, hipStream_t stream,
                                   const int64_t* n_dev) {
    (void)dtype;
    const double* r = static_cast<const double*>(rho);
    const double* t = static_cast<const double*>(T);
    const double* y = static_cast<const double*>(Y);
    double* o = static_cast<double*>(wdot);
    switch (m->wdot_variant) {
        case 1: return dispatch_variant<true, false, false>(m, n, ld, r, t, y, o, params, stream, n_dev);
        case 2: return dispatch_variant<false, true, false>(m, n, ld, r, t, y, o, params, stream, n_dev);
        case 3: return dispatch_variant<true, true, false>(m, n, ld, r, t, y, o, params, stream, n_dev);
        case 4: return dispatch_variant<false, false, true>(m, n, ld, r, t, y, o, params, stream, n_dev);
        case 5: return dispatch_variant<true, false, true>(m, n, ld, r, t, y, o, params, stream, n_dev);
        case 6: return dispatch_variant<false, true, true>(m, n, ld, r, t, y, o, params, stream, n_dev);
        case 7: return dispatch_variant<true, true, true>(m, n, ld, r, t, y, o, params, stream, n_dev);
        default: return dispatch_variant<false, false, false>(m, n, ld, r, t, y, o, params, stream, n_dev);
    }
}

}  // namespace pyro
