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
// Log-space variant (LOG, with RKC): the species rows hold C_k and ln C_k,
// and each rate is one exponential of a sum,
//     R_f = exp(ln k + sum_r nu'_r ln C_r),
//     R_r = exp(ln k + dg_j + dnu ln(R T/p0) + sum_p nu''_p ln C_p),
// with ln [M] added for third-body reactions and ln(P_r/(1+P_r)) + ln F for
// falloff ones: no intermediate (k, 1/K_c, products of C) can overflow or
// underflow, so a rate is out of range only when the rate itself is.  The
// kernel is templated on its arithmetic type; the FP32 production rates are
// this variant in float (FP64 runs it too, as a selectable variant).
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

// g0/(R T) = c0 (1 - ln T) + c1 T + c2 T^2 + c3 T^3 + c4 T^4 + c5/T + c6
// (double coefficients, evaluated in the kernel's arithmetic type).
template <typename real>
__device__ inline real gibbs_poly(const double* c, real T, real omlnT, real invT) {
    return fma(real(c[0]), omlnT, fma(real(c[5]), invT, real(c[6]))) +
           T * fma(T, fma(T, fma(T, real(c[4]), real(c[3])), real(c[2])), real(c[1]));
}

// ln k of the Arrhenius triple in row ``row`` of ``params``.
template <typename real>
__device__ inline real log_arrhenius(const double* __restrict__ params, int row, real lnT,
                                     real invRT) {
    const double* p = params + 3 * row;
    return fma(-real(p[2]), invRT, fma(real(p[1]), lnT, real(p[0])));
}

// ln(x/(1+x)) from u = ln x, for any u (both limits without overflow)
template <typename real>
__device__ inline real log_blend(real u) {
    return u > real(0) ? -log1p(exp(-u)) : u - log1p(exp(u));
}

// Head of the wave's queue of third-body concentrations; the queue is
// popped by shifting, so the values stay in registers with static indices.
template <typename real, int N>
__device__ inline real pop_front(real (&v)[N]) {
    const real head = v[0];
#pragma unroll
    for (int i = 0; i + 1 < N; ++i) v[i] = v[i + 1];
    return head;
}

// C of the species at byte offset ``off`` of a species row (RKC rows are
// half as long as the C/G rows the offsets are given for)
__device__ inline double lds_c(const unsigned char* lds, int off, int lane) {
    return reinterpret_cast<const double*>(lds + (off >> 1))[lane];
}

// ln C of the species at byte offset ``off`` (given for double C/G rows) of
// a log-space row: C[64] then ln C[64] in the kernel's type
template <typename real>
__device__ inline real lds_lnc(const unsigned char* lds, int off, int lane) {
    constexpr int sh = sizeof(real) == 4 ? 1 : 0;
    return reinterpret_cast<const real*>(lds + (off >> sh))[kTile + lane];
}

// Log-space rate of progress (see the LOG variant above).  LP: the sums
// sum_k nu'_kj ln C_k and sum_k nu''_kj ln C_k come from the tile's
// matrix-core contraction (lpf, lpr: this lane's values for the reaction).
template <typename real, bool LP = false>
__device__ inline real rate_of_progress_log(const DevMech& m, const RxnRec& r,
                                            const double* __restrict__ params,
                                            const unsigned char* lds, int lane, real lnk,
                                            real M, real Tc, real lnT, real invT, real invRT,
                                            real ln_rtp, cptr<double> kc, real lpf = 0,
                                            real lpr = 0) {
    if (r.cls >= kLindemann) {
        // ln P_r = ln k0 + ln [M] - ln k_inf; ln k += ln(P_r/(1+P_r)) + ln F
        const real lpr = log_arrhenius<real>(params, m.R + r.fo, lnT, invRT) + log(M) - lnk;
        real lnF = 0;
        if (r.cls == kTroe) {
            // ln F_cent of its three exponential terms without forming them
            // (log-sum-exp), then both logarithms floored at log10 = -300 as
            // F_cent and P_r are in the linear form
            const FalloffRec f = m.falloff[r.fo];
            const real t3 = log(real(1) - real(f.alpha)) + Tc * real(f.a3);
            const real t1 = log(real(f.alpha)) + Tc * real(f.a1);
            const real t2 = real(f.a2) * invT;
            const real tm = fmax(t1, fmax(t2, t3));
            const real lnfc = tm + log(exp(t1 - tm) + exp(t2 - tm) + exp(t3 - tm));
            const real log10e = real(0.43429448190325182765);
            const real lfc = fmax(lnfc * log10e, real(-300));
            const real c = real(-0.4) - real(0.67) * lfc;
            const real nn = real(0.75) - real(1.27) * lfc;
            const real x = fmax(lpr * log10e, real(-300)) + c;
            const real f1 = x / (nn - real(0.14) * x);
            lnF = lfc / (real(1) + f1 * f1) * real(2.30258509299404568402);
        }
        lnk += log_blend(lpr) + lnF;
    }
    real xf = lnk;
    if constexpr (LP) {
        xf += lpf;
    } else {
        xf += lds_lnc<real>(lds, r.r[0], lane);
        if (r.nr > 1) {
            xf += lds_lnc<real>(lds, r.r[1], lane);
            if (r.nr > 2) xf += lds_lnc<real>(lds, r.r[2], lane);
        }
    }
    const real lm = r.cls == kThirdBody ? log(M) : real(0);
    real q = exp(xf + lm);
    if (r.rev) {
        real xr = lnk + real(r.dnu) * ln_rtp;
        if constexpr (LP) {
            xr += lpr;
        } else {
            xr += lds_lnc<real>(lds, r.p[0], lane);
            if (r.np > 1) {
                xr += lds_lnc<real>(lds, r.p[1], lane);
                if (r.np > 2) xr += lds_lnc<real>(lds, r.p[2], lane);
            }
        }
        const double lo[7] = {kc[0], kc[1], kc[2], kc[3], kc[4], kc[5], kc[6]};
        const double hi[7] = {kc[7], kc[8], kc[9], kc[10], kc[11], kc[12], kc[13]};
        const real omlnT = real(1) - lnT;
        const real d_lo = gibbs_poly<real>(lo, Tc, omlnT, invT);
        const real d_hi = gibbs_poly<real>(hi, Tc, omlnT, invT);
        q -= exp(xr + (Tc <= real(kc[14]) ? d_lo : d_hi) + lm);
    }
    return q;
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
        const double k0 = exp(log_arrhenius<double>(params, m.R + r.fo, lnT, invRT));
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
            const double d_lo = gibbs_poly<double>(lo, Tc, omlnT, invT);
            const double d_hi = gibbs_poly<double>(hi, Tc, omlnT, invT);
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

// real: the arithmetic and cell-array type (double, or float with LOG).
template <typename real, int WAVES, int MAXOWN, int MAXPD, bool RKC, bool MM, bool NQ, bool LOG,
          bool LP = false>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(LP ? 4 : 1))) void wdot_kernel(
    DevMech m, int64_t n, int64_t ld, const real* __restrict__ rho,
    const real* __restrict__ T, const real* __restrict__ Y,
    real* __restrict__ wdot, const double* __restrict__ params,
    const int64_t* __restrict__ n_dev) {
    static_assert(!LOG || RKC, "the log-space form uses the combined Gibbs coefficients");
    static_assert(sizeof(real) == 8 || (LOG && !MM && !NQ), "float runs the log-space form only");
    static_assert(!LP || (LOG && sizeof(real) == 8 && !MM && !NQ),
                  "the matrix-core log products are an FP64 log-space form");
    // byte offsets in the tables are given for double rows and slots
    constexpr int sh = sizeof(real) == 4 ? 1 : 0;
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

    const real Tc = T[c];
    const real rc = rho[c];
    const real lnT = log(Tc);
    const real invT = real(1) / Tc;
    const real invRT = invT * real(1.0 / kGasConstant);
    const real rtp = real(kGasConstant / kOneAtm) * Tc;
    const real irtp = real(1) / rtp;
    const real ln_rtp = LOG ? log(rtp) : real(0);
    const real omlnT = real(1) - lnT;

    // ---- species phase: all of this wave's mass-fraction loads first
    const int nown = m.n_own[w];
    const int32_t* own = m.own + w * kMaxOwn;
    real y[MAXOWN];
#pragma unroll
    for (int i = 0; i < MAXOWN; ++i)
        if (i < nown) y[i] = Y[size_t(own[i]) * ld + c];
    // row bytes: C and G (species variant), C (reaction variant), C and ln C (log)
    constexpr int rowb = (LOG ? kRow : RKC ? kRowC : kRow) >> sh;
#pragma unroll
    for (int i = 0; i < MAXOWN; ++i) {
        if (i < nown) {
            const int k = own[i];
            const SpeciesRec& s = m.species[k];
            const real Ck = rc * fmax(y[i], real(0)) * real(s.inv_w);
            real* row = reinterpret_cast<real*>(lds + k * rowb) + lane;
            row[0] = Ck;
            if constexpr (LP) {
                // a finite floor for ln 0: the dense contraction multiplies
                // every ln C by the (mostly zero) coefficients
                // (a select, not fmax: a NaN stays NaN)
                const real lc = log(Ck);
                row[kTile] = lc < real(-kLnFloor) ? real(-kLnFloor) : lc;
            } else if constexpr (LOG) {
                row[kTile] = log(Ck);
            } else if constexpr (!RKC) {
                // both ranges from scalar loads, then a per-lane select of the
                // value (selecting the coefficient address would turn the
                // uniform table reads into per-lane vector loads)
                const real g_lo = gibbs_poly<real>(s.lo, Tc, omlnT, invT);
                const real g_hi = gibbs_poly<real>(s.hi, Tc, omlnT, invT);
                const real gRT = Tc <= real(s.t_mid) ? g_lo : g_hi;
                row[kTile] = exp(gRT);
            }
        }
    }
    __syncthreads();

    unsigned char* qbase = lds + size_t(m.S) * rowb;
    constexpr int qbuf = WAVES * kRxnPerWave * kTile * sizeof(real);   // bytes per chunk buffer
    double* Ml = reinterpret_cast<double*>(qbase + 2 * qbuf);  // MM: [n_pd16][64]
    // LP: sum_k nu''_kj ln C_k of the chunk's slots [slot][64]; the forward
    // sums go into the chunk buffer itself, each slot overwritten by its q
    // by the wave that read it
    double* lpr_l = reinterpret_cast<double*>(qbase + 2 * qbuf);
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
    real Mr[MAXPD];
#pragma unroll
    for (int i = 0; i < MAXPD; ++i) Mr[i] = real(0);
    if (!MM && m.n_pdw[w] > 0) {
        const double* ew = m.effw + size_t(w) * m.S * MAXPD;
        for (int k = 0; k < m.S; ++k) {
            const real ck = reinterpret_cast<const real*>(lds + k * rowb)[lane];
#pragma unroll
            for (int i = 0; i < MAXPD; ++i) Mr[i] = fma(real(ew[k * MAXPD + i]), ck, Mr[i]);
        }
    }

    // ---- reaction chunks and gathering
    real acc[NQ ? 1 : MAXOWN];
#pragma unroll
    for (int i = 0; i < (NQ ? 1 : MAXOWN); ++i) acc[i] = real(0);
    // NQ: omega[64 cells x S] accumulated on the matrix cores over the chunks,
    // omega += q[cells x K slots] nu[K slots x S] with K = 2 WAVES; wave w
    // holds the 16-cell x 16-species output blocks of cell block w & 3 and
    // species blocks (w >> 2) + b WAVES/4, b < NQB (those below ceil(S/16))
    constexpr int NQB = WAVES == kWaves ? 2 : 3;    // S <= 64 (8 waves), <= 192 (16)
    constexpr int NKS = WAVES * kRxnPerWave / 4;     // K-steps per chunk
    // species blocks held in the fragment table: four with kWaves wavefronts
    // (zero-filled beyond S, so every block multiplies unconditionally)
    const int nq_cb = w & 3, nq_sb = w >> 2;
    const int nq_nsb = WAVES == kWaves ? 4 : (m.S + 15) / 16;
    d4 wacc[NQB];
#pragma unroll
    for (int b = 0; b < NQB; ++b) wacc[b] = d4{0.0, 0.0, 0.0, 0.0};
    static_assert(kRxnPerWave == 2, "the reaction phase handles reactions in pairs");
    for (int ch = 0; ch < m.n_chunks; ++ch) {
        unsigned char* qb = qbase + (ch & 1) * qbuf;
        // NQ: this chunk's B fragments of nu, [chunk][species block][K-step][lane]
        double nub[NQB][NKS];
        auto load_nub = [&]() {
#pragma unroll
            for (int b = 0; b < NQB; ++b) {
                const int sb = nq_sb + b * (WAVES / 4);
#pragma unroll
                for (int kk = 0; kk < NKS; ++kk)
                    nub[b][kk] = (WAVES == kWaves || sb < nq_nsb)
                        ? m.nu_frag[((size_t(ch) * nq_nsb + sb) * NKS + kk) * 64 + lane] : 0.0;
            }
        };
        // (8 waves: loaded before the rates are evaluated; 16 waves, with
        // three blocks of eight K-steps, after them to spare registers)
        if constexpr (NQ && WAVES == kWaves) load_nub();
        if constexpr (LP) {
            // the chunk's log products on the matrix cores: D[cell][slot] =
            // sum_k ln C[cell][k] nu[k][slot] for nu' (side 0, into the chunk
            // buffer) and nu'' (side 1); wave w computes the 16-cell x
            // 16-slot block of cell block w & 3, slot block (w >> 2) % NSB,
            // side (w >> 2) / NSB
            constexpr int NSB = WAVES * kRxnPerWave / 16;
            const int cb = w & 3, sb = (w >> 2) % NSB, side = (w >> 2) / NSB;
            const double* bf = m.lp_frag + ((size_t(ch) * 2 + side) * NSB + sb) * m.lp_nks * 64 + lane;
            d4 acc4 = {0.0, 0.0, 0.0, 0.0};
            for (int kk = 0; kk < m.lp_nks; ++kk) {
                const int k = 4 * kk + (lane >> 4);
                // zero beyond S (the B fragments are zero there too, but LDS
                // past the rows is not)
                const double a = k < m.S
                    ? reinterpret_cast<const double*>(lds + k * kRow)[kTile + 16 * cb + (lane & 15)]
                    : 0.0;
                acc4 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bf[size_t(kk) * 64], acc4, 0, 0, 0);
            }
            // D: register i of lane l is cell 16 cb + 4 i + l/16, slot 16 sb + l%16
            double* dst = side == 0 ? reinterpret_cast<double*>(qb) : lpr_l;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                dst[(16 * sb + (lane & 15)) * kTile + 16 * cb + 4 * i + (lane >> 4)] = acc4[i];
            __syncthreads();
        }
        const RxnRec* rb = m.rxn + (size_t(ch) * WAVES + w) * kRxnPerWave;
        const RxnRec r0 = rb[0];
        const RxnRec r1 = rb[1];
        // the wave meets its third-body/falloff reactions in queue order
        real M0 = real(1), M1 = real(1);
        if constexpr (MM) {
            if (r0.cls >= kThirdBody) M0 = Ml[r0.pd * kTile + lane];
            if (r1.cls >= kThirdBody) M1 = Ml[r1.pd * kTile + lane];
        } else {
            M0 = r0.cls >= kThirdBody ? pop_front(Mr) : real(1);
            M1 = r1.cls >= kThirdBody ? pop_front(Mr) : real(1);
        }
        const cptr<double> kc = cst(m.rxn_kc) + (size_t(ch) * WAVES + w) * kRxnPerWave * 16;
        real q0 = real(0), q1 = real(0);
        if constexpr (LOG) {
            const real lk0 = log_arrhenius<real>(params, r0.prow, lnT, invRT);
            const real lk1 = log_arrhenius<real>(params, r1.prow, lnT, invRT);
            real f0 = 0, f1 = 0, b0 = 0, b1 = 0;
            if constexpr (LP) {
                // this wave's slots, read before its q overwrites them
                f0 = *reinterpret_cast<const real*>(qb + r0.qoff + lane * 8);
                f1 = *reinterpret_cast<const real*>(qb + r1.qoff + lane * 8);
                b0 = *reinterpret_cast<const real*>(reinterpret_cast<const unsigned char*>(lpr_l) + r0.qoff + lane * 8);
                b1 = *reinterpret_cast<const real*>(reinterpret_cast<const unsigned char*>(lpr_l) + r1.qoff + lane * 8);
            }
            if (r0.cls != kNoReaction)
                q0 = rate_of_progress_log<real, LP>(m, r0, params, lds, lane, lk0, M0, Tc, lnT, invT,
                                                    invRT, ln_rtp, kc, f0, b0);
            if (r1.cls != kNoReaction)
                q1 = rate_of_progress_log<real, LP>(m, r1, params, lds, lane, lk1, M1, Tc, lnT, invT,
                                                    invRT, ln_rtp, kc + 16, f1, b1);
        } else {
            // both Arrhenius exponentials in one block, so they interleave
            const double kf0 = exp(log_arrhenius<double>(params, r0.prow, lnT, invRT));
            const double kf1 = exp(log_arrhenius<double>(params, r1.prow, lnT, invRT));
            if (r0.cls != kNoReaction)
                q0 = rate_of_progress<RKC>(m, r0, params, lds, lane, kf0, M0, Tc, lnT, invT,
                                           invRT, rtp, irtp, kc);
            if (r1.cls != kNoReaction)
                q1 = rate_of_progress<RKC>(m, r1, params, lds, lane, kf1, M1, Tc, lnT, invT,
                                           invRT, rtp, irtp, kc + 16);
        }
        if (r0.cls != kNoReaction)
            *reinterpret_cast<real*>(qb + (r0.qoff >> sh) + lane * sizeof(real)) = q0;
        else if (NQ)   // empty slots enter the dense product: zero, not stale LDS
            *reinterpret_cast<real*>(qb + (2 * w) * kTile * sizeof(real) + lane * sizeof(real)) = real(0);
        if (r1.cls != kNoReaction)
            *reinterpret_cast<real*>(qb + (r1.qoff >> sh) + lane * sizeof(real)) = q1;
        else if (NQ)
            *reinterpret_cast<real*>(qb + (2 * w + 1) * kTile * sizeof(real) + lane * sizeof(real)) = real(0);
        if constexpr (NQ && WAVES != kWaves) load_nub();
        __syncthreads();
        if constexpr (NQ) {
            // A[cell][slot]: slot 4 kk + l/16, cell 16 cb + l%16 of the chunk buffer
#pragma unroll
            for (int kk = 0; kk < NKS; ++kk) {
                const double a = reinterpret_cast<const double*>(
                    qb + (4 * kk + (lane >> 4)) * kTile * 8)[16 * nq_cb + (lane & 15)];
#pragma unroll
                for (int b = 0; b < NQB; ++b)
                    if (WAVES == kWaves || nq_sb + b * (WAVES / 4) < nq_nsb)
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
        const unsigned char* ql = qb + lane * sizeof(real);
#pragma unroll
        for (int i = 0; i < MAXOWN; ++i) {
            if (i < nown) {
                real a = acc[i], b = real(0);
                int e = bound[i];
                const int e1 = bound[i + 1];
                for (; e + 1 < e1; e += 2) {
                    const GatherEntry g0 = m.gent[e];
                    const GatherEntry g1 = m.gent[e + 1];
                    const real v0 = *reinterpret_cast<const real*>(ql + ((g0 & 0xffffu) >> sh));
                    const real v1 = *reinterpret_cast<const real*>(ql + ((g1 & 0xffffu) >> sh));
                    a = fma(real(int16_t(g0 >> 16)), v0, a);
                    b = fma(real(int16_t(g1 >> 16)), v1, b);
                }
                if (e < e1) {
                    const GatherEntry g0 = m.gent[e];
                    a = fma(real(int16_t(g0 >> 16)),
                            *reinterpret_cast<const real*>(ql + ((g0 & 0xffffu) >> sh)), a);
                }
                acc[i] = a + b;
            }
        }
    }
    if constexpr (NQ) {
        // D: register i of lane l is cell 4 i + l/16, species l % 16 of the block
#pragma unroll
        for (int b = 0; b < NQB; ++b) {
            const int k = 16 * (nq_sb + b * (WAVES / 4)) + (lane & 15);
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

template <typename real, int WAVES, int MAXOWN, int MAXPD, bool RKC, bool MM, bool NQ, bool LOG,
          bool LP = false>
hipError_t launch_k(const pyro_mech* m, int64_t n, int64_t ld, const real* rho, const real* T,
                    const real* Y, real* wdot, const double* params, hipStream_t stream,
                    const int64_t* n_dev) {
    const size_t lds = production_rates_lds_bytes(m, RKC, MM, LOG, sizeof(real), LP);
    const int64_t blocks = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL((wdot_kernel<real, WAVES, MAXOWN, MAXPD, RKC, MM, NQ, LOG, LP>),
                       dim3(unsigned(blocks)), dim3(WAVES * 64), lds, stream, m->dev, n, ld, rho,
                       T, Y, wdot, params ? params : m->dev.params, n_dev);
    return hipGetLastError();
}

// Kernel instances: (type, wavefronts, species owned per wave, [M] slots per
// wave, variant).  With 2 kWaves wavefronts (large mechanisms, reaction
// variant only) a wave owns at most 16 species.
template <typename real, int WAVES, int MAXOWN, int MAXPD, bool RKC, bool MM, bool NQ, bool LOG,
          bool LP = false>
hipError_t set_lds(int bytes) {
    return hipFuncSetAttribute(
        reinterpret_cast<const void*>(&wdot_kernel<real, WAVES, MAXOWN, MAXPD, RKC, MM, NQ, LOG, LP>),
        hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// the NQ instances exist for at most 16 species per wave (NQ needs S <= 64)
template <typename real, int MAXPD, bool RKC, bool MM, bool NQ, bool LOG, bool LP = false>
hipError_t dispatch_own(const pyro_mech* m, int64_t n, int64_t ld, const real* r, const real* t,
                        const real* y, real* o, const double* params, hipStream_t stream,
                        const int64_t* nd) {
    if constexpr (RKC) {
        if (m->fw_waves != kWaves) {
            if (!NQ && m->max_own <= 8)
                return launch_k<real, 2 * kWaves, 8, MAXPD, RKC, MM, false, LOG, LP>(m, n, ld, r, t, y, o, params, stream, nd);
            return launch_k<real, 2 * kWaves, 16, MAXPD, RKC, MM, NQ, LOG, LP>(m, n, ld, r, t, y, o, params, stream, nd);
        }
    }
    if (m->max_own <= 8) return launch_k<real, kWaves, 8, MAXPD, RKC, MM, NQ, LOG, LP>(m, n, ld, r, t, y, o, params, stream, nd);
    if (NQ || m->max_own <= 16)
        return launch_k<real, kWaves, 16, MAXPD, RKC, MM, NQ, LOG, LP>(m, n, ld, r, t, y, o, params, stream, nd);
    if (m->max_own <= 32) return launch_k<real, kWaves, 32, MAXPD, RKC, MM, false, LOG, LP>(m, n, ld, r, t, y, o, params, stream, nd);
    return launch_k<real, kWaves, 64, MAXPD, RKC, MM, false, LOG, LP>(m, n, ld, r, t, y, o, params, stream, nd);
}

template <typename real, bool RKC, bool MM, bool NQ, bool LOG, bool LP = false>
hipError_t set_lds_variant(const pyro_mech* m, int bytes) {
    hipError_t e = hipSuccess;
    if constexpr (RKC) {
        if (m->fw_waves != kWaves) {
            const hipError_t big[] = {
                NQ ? hipSuccess : set_lds<real, 2 * kWaves, 8, 8, RKC, MM, false, LOG, LP>(bytes),
                set_lds<real, 2 * kWaves, 16, 8, RKC, MM, NQ, LOG, LP>(bytes),
                MM || NQ ? hipSuccess : set_lds<real, 2 * kWaves, 8, 16, RKC, MM, false, LOG, LP>(bytes),
                MM ? hipSuccess : set_lds<real, 2 * kWaves, 16, 16, RKC, MM, NQ, LOG, LP>(bytes)};
            for (hipError_t x : big)
                if (x != hipSuccess) e = x;
            return e;
        }
    }
    // the MFMA third-body variant holds no per-wave [M] slots: one MAXPD instance
    const hipError_t all[] = {
        set_lds<real, kWaves, 8, 8, RKC, MM, NQ, LOG, LP>(bytes),
        set_lds<real, kWaves, 16, 8, RKC, MM, NQ, LOG, LP>(bytes),
        NQ ? hipSuccess : set_lds<real, kWaves, 32, 8, RKC, MM, false, LOG, LP>(bytes),
        NQ ? hipSuccess : set_lds<real, kWaves, 64, 8, RKC, MM, false, LOG, LP>(bytes),
        MM ? hipSuccess : set_lds<real, kWaves, 8, 16, RKC, MM, NQ, LOG, LP>(bytes),
        MM ? hipSuccess : set_lds<real, kWaves, 16, 16, RKC, MM, NQ, LOG, LP>(bytes),
        MM || NQ ? hipSuccess : set_lds<real, kWaves, 32, 16, RKC, MM, false, LOG, LP>(bytes),
        MM || NQ ? hipSuccess : set_lds<real, kWaves, 64, 16, RKC, MM, false, LOG, LP>(bytes)};
    for (hipError_t x : all)
        if (x != hipSuccess) e = x;
    return e;
}

template <typename real, bool RKC, bool MM, bool NQ, bool LOG, bool LP = false>
hipError_t dispatch_variant(const pyro_mech* m, int64_t n, int64_t ld, const void* r,
                            const void* t, const void* y, void* o, const double* params,
                            hipStream_t stream, const int64_t* nd) {
    const real* rr = static_cast<const real*>(r);
    const real* tt = static_cast<const real*>(t);
    const real* yy = static_cast<const real*>(y);
    real* oo = static_cast<real*>(o);
    if (MM || m->max_pdw <= 8)
        return dispatch_own<real, 8, RKC, MM, NQ, LOG, LP>(m, n, ld, rr, tt, yy, oo, params, stream, nd);
    return dispatch_own<real, 16, RKC, MM, NQ, LOG, LP>(m, n, ld, rr, tt, yy, oo, params, stream, nd);
}

}  // namespace

size_t production_rates_lds_bytes(const pyro_mech* m, bool reaction_equilibrium,
                                  bool mfma_third_body, bool log_space, int real_bytes,
                                  bool log_products) {
    // species rows: C and G (species variant), C (reaction variant) or C and
    // ln C (log-space), 64 values each; two chunk buffers of rates; [M]
    // block; the reverse-side log products of a chunk
    const size_t row = size_t(kTile) * real_bytes * (log_space || !reaction_equilibrium ? 2 : 1);
    const size_t chunk = size_t(m->fw_waves) * kRxnPerWave * kTile * real_bytes;
    return size_t(m->S) * row + 2 * chunk +
           (mfma_third_body ? size_t((m->n_tb + m->n_fo + 15) / 16 * 16) * kTile * 8 : 0) +
           (log_products ? chunk : 0);
}

bool log_products_supported(const pyro_mech* m) {
    return m->kc_ok && m->dev.lp_nks > 0 &&
           production_rates_lds_bytes(m, true, false, true, 8, true) <= 160 * 1024;
}

bool log_space_supported(const pyro_mech* m, int real_bytes) {
    return m->kc_ok && production_rates_lds_bytes(m, true, false, true, real_bytes) <= 160 * 1024;
}

hipError_t prepare_production_rates(const pyro_mech* m) {
    hipError_t e = hipSuccess;
    for (const int v : {0, 1, 2, 3, 4, 5, 6, 7}) {
        const bool rkc = v & 1, mm = v & 2, nq = v & 4;
        const size_t bytes = production_rates_lds_bytes(m, rkc, mm);
        if (bytes > 160 * 1024 || (rkc && !m->kc_ok) || (nq && !nq_supported(m))) continue;
        hipError_t x;
        switch (v) {
            case 0: x = set_lds_variant<double, false, false, false, false>(m, int(bytes)); break;
            case 1: x = set_lds_variant<double, true, false, false, false>(m, int(bytes)); break;
            case 2: x = set_lds_variant<double, false, true, false, false>(m, int(bytes)); break;
            case 3: x = set_lds_variant<double, true, true, false, false>(m, int(bytes)); break;
            case 4: x = set_lds_variant<double, false, false, true, false>(m, int(bytes)); break;
            case 5: x = set_lds_variant<double, true, false, true, false>(m, int(bytes)); break;
            case 6: x = set_lds_variant<double, false, true, true, false>(m, int(bytes)); break;
            default: x = set_lds_variant<double, true, true, true, false>(m, int(bytes));
        }
        if (x != hipSuccess) e = x;
    }
    if (log_space_supported(m, 8)) {
        const hipError_t x = set_lds_variant<double, true, false, false, true>(
            m, int(production_rates_lds_bytes(m, true, false, true, 8)));
        if (x != hipSuccess) e = x;
    }
    if (log_space_supported(m, 4)) {
        const hipError_t x = set_lds_variant<float, true, false, false, true>(
            m, int(production_rates_lds_bytes(m, true, false, true, 4)));
        if (x != hipSuccess) e = x;
    }
    if (log_products_supported(m)) {
        const hipError_t x = set_lds_variant<double, true, false, false, true, true>(
            m, int(production_rates_lds_bytes(m, true, false, true, 8, true)));
        if (x != hipSuccess) e = x;
    }
    return e;
}

bool nq_supported(const pyro_mech* m) {
    // blocks per wave: 2 with kWaves wavefronts, 3 with 2 kWaves
    return m->max_own <= 16 && (m->fw_waves == kWaves ? m->S <= 64 : m->S <= 192);
}

hipError_t launch_production_rates(const pyro_mech* m, int64_t n, int64_t ld, int dtype,
                                   const void* r, const void* t, const void* y, void* o,
                                   const double* params, hipStream_t stream,
                                   const int64_t* nd) {
    // FP32: the log-space form in float (the only float instance)
    if (dtype == PYRO_F32)
        return dispatch_variant<float, true, false, false, true>(m, n, ld, r, t, y, o, params, stream, nd);
    switch (m->wdot_variant) {
        case 1: return dispatch_variant<double, true, false, false, false>(m, n, ld, r, t, y, o, params, stream, nd);
        case 2: return dispatch_variant<double, false, true, false, false>(m, n, ld, r, t, y, o, params, stream, nd);
        case 3: return dispatch_variant<double, true, true, false, false>(m, n, ld, r, t, y, o, params, stream, nd);
        case 4: return dispatch_variant<double, false, false, true, false>(m, n, ld, r, t, y, o, params, stream, nd);
        case 5: return dispatch_variant<double, true, false, true, false>(m, n, ld, r, t, y, o, params, stream, nd);
        case 6: return dispatch_variant<double, false, true, true, false>(m, n, ld, r, t, y, o, params, stream, nd);
        case 7: return dispatch_variant<double, true, true, true, false>(m, n, ld, r, t, y, o, params, stream, nd);
        case 9: return dispatch_variant<double, true, false, false, true>(m, n, ld, r, t, y, o, params, stream, nd);
        case 25: return dispatch_variant<double, true, false, false, true, true>(m, n, ld, r, t, y, o, params, stream, nd);
        default: return dispatch_variant<double, false, false, false, false>(m, n, ld, r, t, y, o, params, stream, nd);
    }
}

}  // namespace pyro
