// Reverse-mode product (VJP) of the net production rates: given wbar =
// dL/d omega for every cell, the gradients of L = sum_cells sum_k wbar_k
// omega_k with respect to Y and T per cell and with respect to every
// Arrhenius triple (ln A, b, Ea) summed over cells, at fixed density
// (Appendix A.1: eq. production_rates, eq. reaction_rates, eq. rate_coeff,
// eq. equil_constants, eq. nasa_poly, eq. concentrations).
//
// Per reaction j, with D = Rf - Rr (before the third-body factor phi) and
// qbar = sum_k nu_kj wbar_k, the adjoints are
//   Dbar = qbar phi,   xbar = Dbar D         (adjoint of ln k),
//   a_j = Dbar Rf,     b_j = Dbar Rr,
// and per species, summed over its reactions,
//   Cbar_k C_k = sum_j nu'_kj a_j - nu''_kj b_j,
//   Gbar_k G_k = sum_j (nu'_kj - nu''_kj) b_j,
// so the species sums reuse the forward kernel's chunk/gather structure with
// two LDS values per reaction.  Falloff reactions split xbar between the
// high- and low-pressure triples through s = d ln k / d ln P_r.
//
// A workgroup of 16 wavefronts works on one 64-cell tile at a time (one
// reaction per wavefront per chunk of 16, from a schedule of its own), with
// double-buffered chunk planes and one barrier per chunk.  The sums over the
// tile's cells of xbar (1, ln T, -1/(R T)) are one four-value lane sum; the
// owning wavefront adds them to the workgroup's accumulator in LDS, and a
// second kernel adds the per-workgroup accumulators in a fixed order, so the
// results are bitwise reproducible.
#include <algorithm>
#include <mutex>

#include "pyro_internal.h"

namespace pyro {
namespace {

constexpr int kVRow = kVjpRow;                      // C[64], G[64], wbar[64]
constexpr int kPlane = kChunk * kTile * 8;          // a, b or q: [slot][cell]
static_assert(kVjpWaves == kChunk, "one reaction per wavefront fills a chunk's slots");

struct CGW {
    double c, g, w;
};

// row_off: byte offset of the species row (species * kVRow)
__device__ inline CGW lds_row(const unsigned char* lds, int row_off, int lane) {
    const double* p = reinterpret_cast<const double*>(lds + row_off) + lane;
    return CGW{p[0], p[kTile], p[2 * kTile]};
}

__device__ inline double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

__device__ inline double gibbs_poly(const double* c, double T, double omlnT, double invT) {
    return fma(c[0], omlnT, fma(c[5], invT, c[6])) +
           T * fma(T, fma(T, fma(T, c[4], c[3]), c[2]), c[1]);
}

// h/(R T) from NASA7 a1..a6
__device__ inline double enthalpy_poly(const double* a, double T, double invT) {
    return a[0] + a[5] * invT +
           T * (a[1] * 0.5 + T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + T * (a[4] * 0.2))));
}

// A gathering entry: slot byte offset and the coefficients nu', -nu'' and
// nu' - nu'' rebuilt from the upper 16 bits of their doubles (wave-uniform,
// so they stay scalar operands of the FMAs; no conversions)
struct GatherCoef {
    int off;
    double nf, mnr, d;
};

__device__ inline GatherCoef gather_coef(uint32_t w0, uint32_t w1) {
    return GatherCoef{int(w0 & 0xffffu), from_top16(w0 >> 16), from_top16(w1 & 0xffffu),
                      from_top16(w1 >> 16)};
}

template <int N>
__device__ inline double pop_front(double (&v)[N]) {
    const double head = v[0];
#pragma unroll
    for (int i = 0; i + 1 < N; ++i) v[i] = v[i + 1];
    return head;
}

// per-cell temperature terms; 1/(R T), R T/p0 and p0/(R T) are derived on use
struct CellState {
    double T, lnT, invT;
    __device__ double invRT() const { return invT * (1.0 / kGasConstant); }
    __device__ double rtp() const { return T * (kGasConstant / kOneAtm); }
    __device__ double irtp() const { return invT * (kOneAtm / kGasConstant); }
};

struct RevOut {
    double a, b, q, xbar, xbar0, Mbar, Tbar;
};

// Forward recomputation and reverse sweep of one reaction for one cell.
__device__ inline RevOut reaction_vjp(const DevMech& m, const RxnRec& r,
                                      const double* __restrict__ params,
                                      const unsigned char* lds, int lane, double M,
                                      const CellState& cs) {
    const cptr<double> pr = cst(params) + 3 * r.prow;
    const double kinf = exp(fma(-pr[2], cs.invRT(), fma(pr[1], cs.lnT, pr[0])));
    const double dxdT = fma(pr[2] * cs.invRT(), cs.invT, pr[1] * cs.invT);
    double keff = kinf, s = 0.0, dlnF_dT = 0.0, k0 = 0.0, F = 1.0, Pr = 0.0;
    double dlnF_dlnPr = 0.0, dx0dT = 0.0;
    if (r.cls >= kLindemann) {
        const cptr<double> pl = cst(params) + 3 * (m.R + r.fo);
        k0 = exp(fma(-pl[2], cs.invRT(), fma(pl[1], cs.lnT, pl[0])));
        dx0dT = fma(pl[2] * cs.invRT(), cs.invT, pl[1] * cs.invT);
        Pr = k0 * M / kinf;
        if (r.cls == kTroe) {
            const FalloffRec f = cst(m.falloff)[r.fo];
            const double e3 = exp(cs.T * f.a3), e1 = exp(cs.T * f.a1), e2 = exp(f.a2 * cs.invT);
            const double Fc_raw = (1.0 - f.alpha) * e3 + f.alpha * e1 + e2;
            const bool fc_ok = Fc_raw > 1e-300;
            const double Fcent = fc_ok ? Fc_raw : 1e-300;
            const double dFcent =
                (1.0 - f.alpha) * f.a3 * e3 + f.alpha * f.a1 * e1 - e2 * f.a2 * cs.invT * cs.invT;
            const double Lc = log10(Fcent);
            const bool pr_ok = Pr > 1e-300;
            const double X = log10(pr_ok ? Pr : 1e-300) + (-0.4 - 0.67 * Lc);
            const double nn = 0.75 - 1.27 * Lc;
            const double den = nn - 0.14 * X;
            const double iden = 1.0 / den;
            const double f1 = X * iden;
            const double w1 = 1.0 / (1.0 + f1 * f1);
            const double lF = Lc * w1;
            F = exp10(lF);
            // d log10 F / dX at fixed L_c, and d log10 F / d L_c at fixed P_r
            const double df1_dX = nn * iden * iden;
            dlnF_dlnPr = pr_ok ? -2.0 * Lc * f1 * df1_dX * w1 * w1 : 0.0;
            const double df1_dLc = (-0.67 * den + 1.1762 * X) * iden * iden;
            const double dlF_dLc = w1 - 2.0 * Lc * f1 * df1_dLc * w1 * w1;
            dlnF_dT = fc_ok ? dlF_dLc * dFcent / Fcent : 0.0;
        }
        const double ipr = 1.0 / (1.0 + Pr);
        keff = kinf * (Pr * ipr) * F;
        s = ipr + dlnF_dlnPr;
    }
    // forward products and the sum of nu wbar over the participants
    CGW x = lds_row(lds, r.r[0], lane);
    double cr = x.c, gr = x.g, qbar = -x.w;
    if (r.nr > 1) {
        x = lds_row(lds, r.r[1], lane);
        cr *= x.c;
        gr *= x.g;
        qbar -= x.w;
        if (r.nr > 2) {
            x = lds_row(lds, r.r[2], lane);
            cr *= x.c;
            gr *= x.g;
            qbar -= x.w;
        }
    }
    x = lds_row(lds, r.p[0], lane);
    double cgp = x.c * x.g;
    qbar += x.w;
    if (r.np > 1) {
        x = lds_row(lds, r.p[1], lane);
        cgp *= x.c * x.g;
        qbar += x.w;
        if (r.np > 2) {
            x = lds_row(lds, r.p[2], lane);
            cgp *= x.c * x.g;
            qbar += x.w;
        }
    }
    double rev = 0.0;  // pw prod_p (C G) / prod_r G: Rr per unit k
    if (r.rev) {
        double pw = 1.0;
        if (r.dnu > 0)
            for (int i = 0; i < r.dnu; ++i) pw *= cs.rtp();
        else
            for (int i = 0; i < -r.dnu; ++i) pw *= cs.irtp();
        rev = pw * cgp * recip(gr);
    }
    const double Rf = keff * cr;
    const double Rr = keff * rev;
    const double D = Rf - Rr;
    const double phi = r.cls == kThirdBody ? M : 1.0;
    const double Dbar = qbar * phi;
    RevOut o;
    o.q = phi * D;
    o.a = Dbar * Rf;
    o.b = Dbar * Rr;
    const double xeff = Dbar * D;
    o.Tbar = -o.b * double(r.dnu) * cs.invT;
    o.Mbar = 0.0;
    if (r.cls == kThirdBody) o.Mbar = qbar * D;
    if (r.cls >= kLindemann) {
        const double ipr = 1.0 / (1.0 + Pr);
        o.xbar = xeff * (1.0 - s);
        o.xbar0 = xeff * s;
        o.Mbar = Dbar * (cr - rev) * k0 * F * (ipr * ipr + dlnF_dlnPr * ipr);
        o.Tbar += o.xbar * dxdT + o.xbar0 * dx0dT + xeff * dlnF_dT;
    } else {
        o.xbar = xeff;
        o.xbar0 = 0.0;
        o.Tbar += xeff * dxdT;
    }
    return o;
}

// one DPP move of a double (both halves with the same control); lanes of
// rows outside ROW_MASK receive unspecified values
template <int CTRL, int ROW_MASK>
__device__ inline double dpp(double v) {
    const int2 h = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_mov_dpp(h.x, CTRL, ROW_MASK, 0xf, false);
    r.y = __builtin_amdgcn_mov_dpp(h.y, CTRL, ROW_MASK, 0xf, false);
    return __builtin_bit_cast(double, r);
}

// v[l] + v[l ^ 16] and v[l] + v[l ^ 32]: the row and half-wave swaps of
// gfx950 (v_permlane16_swap, v_permlane32_swap) applied to both halves of a
// double; with both operands equal to v, the two results are v and its
// partner in either order, so their sum is the pair sum in every lane
__device__ inline double add_xor16(double v) {
    const int2 h = __builtin_bit_cast(int2, v);
    const auto lo = __builtin_amdgcn_permlane16_swap(h.x, h.x, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(h.y, h.y, false, false);
    return __builtin_bit_cast(double, int2{int(lo[0]), int(hi[0])}) +
           __builtin_bit_cast(double, int2{int(lo[1]), int(hi[1])});
}

__device__ inline double add_xor32(double v) {
    const int2 h = __builtin_bit_cast(int2, v);
    const auto lo = __builtin_amdgcn_permlane32_swap(h.x, h.x, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(h.y, h.y, false, false);
    return __builtin_bit_cast(double, int2{int(lo[0]), int(hi[0])}) +
           __builtin_bit_cast(double, int2{int(lo[1]), int(hi[1])});
}

// Sums over the 64 lanes of four values at once, in a fixed order and without
// LDS traffic: afterwards every lane l holds the total of value l & 3.  Two
// reduce-scatter exchanges inside each quad (each lane keeps one value of a
// pair and adds its partner's copy of it), then rotations by 4 and 8 within
// each row and the row and half-wave swaps, all of which keep a lane's
// position in its quad.  33 VALU instructions against 54 for three separate
// butterflies.
__device__ inline double wave_sum4(double a, double b, double c, double d, int lane) {
    const bool o1 = lane & 1, o2 = lane & 2;
    const double u = (o1 ? b : a) + dpp<0xb1, 0xf>(o1 ? a : b);   // quad_perm [1, 0, 3, 2]
    const double v = (o1 ? d : c) + dpp<0xb1, 0xf>(o1 ? c : d);
    double z = (o2 ? v : u) + dpp<0x4e, 0xf>(o2 ? u : v);          // quad_perm [2, 3, 0, 1]
    z += dpp<0x124, 0xf>(z);   // row_ror:4
    z += dpp<0x128, 0xf>(z);   // row_ror:8
    z = add_xor16(z);
    return add_xor32(z);
}

// LDS of the reverse sweep: species rows, then a region holding the two
// chunk buffers during the chunk loop and, after it, Mbar [n_pd][64], the
// per-wave temperature partials [kVjpWaves][64] and (Jacobian rows) the
// per-wave heat-capacity partials [kVjpWaves][64], then the parameter sums
__host__ __device__ inline size_t vjp_region_bytes(int n_pd) {
    const size_t chunks = 2 * 3 * size_t(kPlane);
    const size_t after = (size_t(n_pd) + 2 * kVjpWaves) * kTile * 8;
    return chunks > after ? chunks : after;
}

// c_p/R of NASA7 a1..a5
__device__ inline double cp_poly(const double* a, double T) {
    return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
}

// The schedule a launch runs: the reverse sweep's, or a Jacobian row's.
template <int JAC>
__device__ inline DevSched sched_of(const DevMech& m, int unit) {
    if constexpr (JAC != 0) {
        return m.jac_rows[unit];
    } else {
        return m.vjp;
    }
}

// WITH_W: also the net production rates, gathered from a third plane (q).
// JAC (0: the VJP; 1, 2: one row of the chemical Jacobian): the cotangent is
// W_unit on species ``unit`` and zero elsewhere (not read from wbar), so Ybar
// receives row ``unit`` of dS/dY with S_k = W_k omega_k at fixed T and Tbar
// dS_unit/dT; reactions without species ``unit`` have a zero cotangent and
// are skipped, and no parameter sums are formed.  JAC == 2 adds the
// dependence of T on Y at fixed internal energy, dT/dY_k = -e_k/c_v.
// LNT: ln T comes from lnTg (a pre-pass) instead of a logarithm per tile;
// keeping the logarithm's constants live across the persistent tile loop
// spilled them to scratch, reloaded on every tile.
template <int MAXOWN, int MAXPD, bool WITH_W, int JAC = 0, bool LNT = false>
__global__ __launch_bounds__(kVjpWaves * 64) void vjp_kernel(
    DevMech m, int64_t n, int64_t ld, const double* __restrict__ rho,
    const double* __restrict__ T, const double* __restrict__ Y,
    const double* __restrict__ wbar, double* __restrict__ Ybar, double* __restrict__ Tbar,
    double* __restrict__ wdot, double* __restrict__ partial, const double* __restrict__ params,
    int unit = -1, const double* __restrict__ lnTg = nullptr, int64_t out_ld = 0,
    int64_t out_tile = 0, int passes = 1) {
    static_assert(JAC == 0 || !WITH_W, "Jacobian rows do not return omega");
    constexpr int kBuf = (WITH_W ? 3 : 2) * kPlane;   // one chunk buffer: a, b (, q) planes
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    // A Jacobian row runs the row's own schedule: only the reactions with a
    // nonzero net coefficient of the unit species (the others have a zero
    // cotangent), packed into as few chunks as they fill.  The rows share the
    // reverse sweep's species ownership.
    const DevSched sc0 = m.vjp;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned char* bufs = lds + size_t(m.S) * kVRow;
    double* mbar = reinterpret_cast<double*>(bufs);                           // after the loop
    double* tb = mbar + size_t(m.n_pd) * kTile;                               // after the loop
    double* cvb = tb + size_t(kVjpWaves) * kTile;                              // JAC: after the loop
    double* pacc = reinterpret_cast<double*>(bufs + vjp_region_bytes(m.n_pd)); // [R + n_fo][3]
    const int n_rows = m.R + m.n_fo;
    if (JAC == 0)
        for (int i = threadIdx.x; i < 3 * n_rows; i += kVjpWaves * 64) pacc[i] = 0.0;
    const int nown = cst(sc0.n_own)[w];
    const cptr<int32_t> own = cst(sc0.own) + w * kMaxOwn;

    const int64_t n_tiles = (n + kTile - 1) / kTile;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t cell = tile * kTile + lane;
        const bool valid = cell < n;
        // Jacobian rows: element k of this cell's row at Ybar[k out_ld + ocell]
        // (out_ld = ld, out_tile = 64: the species-major layout; out_ld = 64,
        // out_tile = S S 64: 64-cell tiles of whole matrices)
        const int64_t ocell = JAC ? tile * out_tile + lane : cell;
        const int64_t old = JAC ? out_ld : ld;
        const int64_t c = valid ? cell : n - 1;
        CellState cs;
        cs.T = T[c];
        const double rc = rho[c];
        if constexpr (LNT) {
            cs.lnT = lnTg[c];
        } else {
            cs.lnT = log(cs.T);
        }
        cs.invT = 1.0 / cs.T;
        const double omlnT = 1.0 - cs.lnT;

        // ---- species phase: C, G and wbar (zero for cells past n, so those
        // lanes contribute nothing to any sum)
        double cvp = 0.0;   // JAC == 2: this wave's part of c_v = sum_k Y_k c_v,k
#pragma unroll
        for (int i = 0; i < MAXOWN; ++i) {
            if (i < nown) {
                const int k = own[i];
                const SpeciesRec s = cst(m.species)[k];
                const double y = Y[size_t(k) * ld + c];
                double wb;
                if constexpr (JAC != 0) {
                    wb = valid && k == unit ? cst(m.w)[unit] : 0.0;
                } else {
                    wb = valid ? wbar[size_t(k) * ld + c] : 0.0;
                }
                if constexpr (JAC == 2) {
                    // c_v,k = (c_p,k - R)/W_k, Y as given (eq. cv)
                    const NewtonSpecies ns = cst(m.newton)[k];
                    const double cpr = cs.T <= s.t_mid ? cp_poly(ns.lo, cs.T) : cp_poly(ns.hi, cs.T);
                    cvp = fma(y * kGasConstant * s.inv_w, cpr - 1.0, cvp);
                }
                const double g_lo = gibbs_poly(s.lo, cs.T, omlnT, cs.invT);
                const double g_hi = gibbs_poly(s.hi, cs.T, omlnT, cs.invT);
                double* row = reinterpret_cast<double*>(lds + k * kVRow) + lane;
                row[0] = rc * fmax(y, 0.0) * s.inv_w;
                row[kTile] = exp(cs.T <= s.t_mid ? g_lo : g_hi);
                row[2 * kTile] = wb;
            }
        }
        __syncthreads();

        // The reverse sweep takes its pass count (1) as a kernel argument:
        // as a loop of a count unknown at compile time, its tile body
        // compiles without the scratch spill of the straight-line form (17.8
        // against 18.5 ms on 2^22 config-1 cells, same box); the Jacobian rows
        // run faster straight-line (about 16.5 against 17.2 ms on 2^18 cells).
        const int n_pass = JAC ? 1 : passes;
        for (int pass = 0; pass < n_pass; ++pass) {
            // the row's (the sweep's) schedule and outputs
            const DevSched sc = sched_of<JAC>(m, unit);
            const int npdw = cst(sc.n_pdw)[w];
            double* const Yrow = JAC ? Ybar + size_t(unit) * m.S * out_ld : Ybar;
            double* const Trow = JAC && Tbar ? Tbar + size_t(unit) * ld : Tbar;

            // ---- third-body concentrations of this wave's reactions
            double Mr[MAXPD];
#pragma unroll
            for (int i = 0; i < MAXPD; ++i) Mr[i] = 0.0;
            if (npdw > 0) {
                // scalar efficiencies of the wave's queue slots, MAXPD per species
                const cptr<double> ew = cst(sc.effw) + size_t(w) * m.S * MAXPD;
                int k = 0;
                for (; k + 4 <= m.S; k += 4) {
                    double ck[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        ck[u] = reinterpret_cast<const double*>(lds + (k + u) * kVRow)[lane];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int i = 0; i < MAXPD; ++i)
                            Mr[i] = fma(ew[(k + u) * MAXPD + i], ck[u], Mr[i]);
                }
                for (; k < m.S; ++k) {
                    const double ck = reinterpret_cast<const double*>(lds + k * kVRow)[lane];
#pragma unroll
                    for (int i = 0; i < MAXPD; ++i) Mr[i] = fma(ew[k * MAXPD + i], ck, Mr[i]);
                }
            }

            double cc[MAXOWN], gam[MAXOWN], ws[MAXOWN];
#pragma unroll
            for (int i = 0; i < MAXOWN; ++i) cc[i] = gam[i] = ws[i] = 0.0;
            double tbar = 0.0;

            for (int ch = 0; ch < sc.n_chunks; ++ch) {
                unsigned char* plane_a = bufs + (ch & 1) * kBuf;
                unsigned char* plane_b = plane_a + kPlane;
                unsigned char* plane_q = plane_b + kPlane;
                const RxnRec r = cst(sc.rxn)[size_t(ch) * kVjpWaves + w];
                if (r.cls != kNoReaction) {
                    const double M = r.cls >= kThirdBody ? pop_front(Mr) : 1.0;
                    const RevOut o = reaction_vjp(m, r, params, lds, lane, M, cs);
                    *reinterpret_cast<double*>(plane_a + r.qoff + lane * 8) = o.a;
                    *reinterpret_cast<double*>(plane_b + r.qoff + lane * 8) = o.b;
                    if (WITH_W) *reinterpret_cast<double*>(plane_q + r.qoff + lane * 8) = o.q;
                    // the consumed [M] slot now holds this reaction's Mbar: after
                    // the loop the queue's tail holds them in chunk order
                    if (r.cls >= kThirdBody) Mr[MAXPD - 1] = o.Mbar;
                    tbar += o.Tbar;
                    if constexpr (JAC == 0) {
                        // cell sums of xbar (1, ln T, -1/(R T)) into this reaction's
                        // rows: lanes 0, 1, 2 hold the three totals
                        const double sx = wave_sum4(o.xbar, o.xbar * cs.lnT, -o.xbar * cs.invRT(), 0.0, lane);
                        double sf = 0.0;
                        if (r.cls >= kLindemann)
                            sf = wave_sum4(o.xbar0, o.xbar0 * cs.lnT, -o.xbar0 * cs.invRT(), 0.0, lane);
                        if (lane < 3) {
                            pacc[3 * r.prow + lane] += sx;
                            if (r.cls >= kLindemann) pacc[3 * (m.R + r.fo) + lane] += sf;
                        }
                    }
                }
                __syncthreads();
                // species sums of this chunk (the next chunk fills the other buffer)
                const cptr<int32_t> gp = cst(sc.gptr) + (size_t(ch) * kVjpWaves + w) * (kMaxOwn + 1);
                const cptr<uint32_t> gent = cst(sc.gent);
                int32_t bound[MAXOWN + 1];
#pragma unroll
                for (int i = 0; i <= MAXOWN; ++i) bound[i] = gp[i];
#pragma unroll
                for (int i = 0; i < MAXOWN; ++i) {
                    if (i < nown) {
                        // two entries (four words) per step, their loads issued
                        // together; the coefficients are scalar doubles
                        double sc0 = cc[i], sg0 = gam[i], sc1 = 0.0, sg1 = 0.0;
                        double sw0 = ws[i], sw1 = 0.0;
                        int e = bound[i];
                        for (; e + 4 <= bound[i + 1]; e += 4) {
                            const GatherCoef g0 = gather_coef(gent[e], gent[e + 1]);
                            const GatherCoef g1 = gather_coef(gent[e + 2], gent[e + 3]);
                            const int o0 = g0.off + lane * 8, o1 = g1.off + lane * 8;
                            const double a0 = *reinterpret_cast<const double*>(plane_a + o0);
                            const double b0 = *reinterpret_cast<const double*>(plane_b + o0);
                            const double a1 = *reinterpret_cast<const double*>(plane_a + o1);
                            const double b1 = *reinterpret_cast<const double*>(plane_b + o1);
                            sc0 = fma(g0.nf, a0, fma(g0.mnr, b0, sc0));
                            sg0 = fma(g0.d, b0, sg0);
                            sc1 = fma(g1.nf, a1, fma(g1.mnr, b1, sc1));
                            sg1 = fma(g1.d, b1, sg1);
                            if (WITH_W) {
                                const double q0 = *reinterpret_cast<const double*>(plane_q + o0);
                                const double q1 = *reinterpret_cast<const double*>(plane_q + o1);
                                sw0 = fma(-g0.d, q0, sw0);
                                sw1 = fma(-g1.d, q1, sw1);
                            }
                        }
                        if (e < bound[i + 1]) {
                            const GatherCoef g = gather_coef(gent[e], gent[e + 1]);
                            const int off = g.off + lane * 8;
                            const double av = *reinterpret_cast<const double*>(plane_a + off);
                            const double bv = *reinterpret_cast<const double*>(plane_b + off);
                            sc0 = fma(g.nf, av, fma(g.mnr, bv, sc0));
                            sg0 = fma(g.d, bv, sg0);
                            if (WITH_W)
                                sw0 = fma(-g.d, *reinterpret_cast<const double*>(plane_q + off), sw0);
                        }
                        cc[i] = sc0 + sc1;
                        gam[i] = sg0 + sg1;
                        ws[i] = sw0 + sw1;
                    }
                }
            }

            // ---- Mbar of this wave's third-body reactions into LDS, once every
            // wave is done with the chunk buffers (a Jacobian row writes and
            // later reads only its own third-body rows)
            __syncthreads();
            {
                const cptr<int32_t> pl = cst(sc.pd_list) + w * kMaxPd;
#pragma unroll
                for (int p = 0; p < MAXPD; ++p)
                    if (p >= MAXPD - npdw) mbar[size_t(pl[p - (MAXPD - npdw)]) * kTile + lane] = Mr[p];
            }
            __syncthreads();
            // ---- sum_j eps_jk Mbar_j for the wave's species: each Mbar row is
            // read once for all of them, the efficiencies of a row (contiguous per
            // wave) are scalar operands
            double cmv[MAXOWN];
#pragma unroll
            for (int i = 0; i < MAXOWN; ++i) cmv[i] = 0.0;
            if constexpr (JAC != 0) {
                // a Jacobian row: only its own third-body rows have M-bar
                const cptr<double> eo = cst(sc.effo) + size_t(w) * m.n_pd * MAXOWN;
                const cptr<int32_t> pr = cst(sc.pd_rows);
                for (int t = 0; t < sc.n_pd_rows; ++t) {
                    const int j = pr[t];
                    const double mb = mbar[size_t(j) * kTile + lane];
#pragma unroll
                    for (int i = 0; i < MAXOWN; ++i) cmv[i] = fma(eo[j * MAXOWN + i], mb, cmv[i]);
                }
            } else {
                const cptr<double> eo = cst(sc.effo) + size_t(w) * m.n_pd * MAXOWN;
                int j = 0;
                for (; j + 4 <= m.n_pd; j += 4) {
                    double mb[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) mb[u] = mbar[size_t(j + u) * kTile + lane];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int i = 0; i < MAXOWN; ++i)
                            cmv[i] = fma(eo[(j + u) * MAXOWN + i], mb[u], cmv[i]);
                }
                for (; j < m.n_pd; ++j) {
                    const double mb = mbar[size_t(j) * kTile + lane];
#pragma unroll
                    for (int i = 0; i < MAXOWN; ++i) cmv[i] = fma(eo[j * MAXOWN + i], mb, cmv[i]);
                }
            }
            // ---- species results
#pragma unroll
            for (int i = 0; i < MAXOWN; ++i) {
                if (i < nown) {
                    const int k = own[i];
                    const double cm = cmv[i];  // sum_j eps_jk Mbar_j
                    // dL/dY_k = Cbar_k rho/W_k = (Cbar_k C_k) rho/(W_k C_k), with C_k
                    // still in this tile's LDS row (zero where Y_k <= 0)
                    const double ck = reinterpret_cast<const double*>(lds + k * kVRow)[lane];
                    const SpeciesRec sp = cst(m.species)[k];
                    const double rw = rc * sp.inv_w;
                    const double ybar = ck > 0.0 ? cc[i] * rw / ck + rw * cm : 0.0;
                    const NewtonSpecies ns = cst(m.newton)[k];
                    const double h_lo = enthalpy_poly(ns.lo, cs.T, cs.invT);
                    const double h_hi = enthalpy_poly(ns.hi, cs.T, cs.invT);
                    const double hRT = cs.T <= sp.t_mid ? h_lo : h_hi;
                    tbar -= gam[i] * hRT * cs.invT;
                    // (fixed energy: completed below, once dS/dT is known; the
                    // partial row goes to memory rather than being held in
                    // registers across the sums)
                    if (valid) {
                        Yrow[size_t(k) * old + ocell] = ybar;
                        if (WITH_W) wdot[size_t(k) * ld + cell] = ws[i];
                    }
                }
            }
            // ---- temperature: per-wave partials summed in wave order
            tb[w * kTile + lane] = tbar;
            if (JAC == 2) cvb[w * kTile + lane] = cvp;
            __syncthreads();
            if constexpr (JAC == 2) {
                // every wave forms the same sums in the same order, then applies
                // dS/dY_k += dS/dT dT/dY_k with dT/dY_k = -e_k/c_v at fixed e
                double st = 0.0, cv = 0.0;
                for (int v = 0; v < kVjpWaves; ++v) {
                    st += tb[v * kTile + lane];
                    cv += cvb[v * kTile + lane];
                }
                const double g = st / cv;
#pragma unroll
                for (int i = 0; i < MAXOWN; ++i) {
                    if (i < nown && valid) {
                        // e_k = (h_k - R T)/W_k (eq. int_energy), formed again
                        const int k = own[i];
                        const SpeciesRec sp = cst(m.species)[k];
                        const NewtonSpecies ns = cst(m.newton)[k];
                        const double h_lo = enthalpy_poly(ns.lo, cs.T, cs.invT);
                        const double h_hi = enthalpy_poly(ns.hi, cs.T, cs.invT);
                        const double hRT = cs.T <= sp.t_mid ? h_lo : h_hi;
                        const double ek = kGasConstant * cs.T * (hRT - 1.0) * sp.inv_w;
                        double* o = Yrow + size_t(k) * old + ocell;
                        *o = fma(-g, ek, *o);
                    }
                }
                if (w == 0 && valid && Trow) Trow[cell] = st;
            } else if (w == 0) {
                double s = 0.0;
                for (int v = 0; v < kVjpWaves; ++v) s += tb[v * kTile + lane];
                if (valid && (JAC == 0 || Trow)) Trow[cell] = s;
            }
        }   // pass
    }
    if constexpr (JAC == 0) {
        // ---- this workgroup's parameter sums: [block][R + n_fo][3]
        __syncthreads();
        double* p = partial + size_t(blockIdx.x) * 3 * n_rows;
        for (int i = threadIdx.x; i < 3 * n_rows; i += kVjpWaves * 64) p[i] = pacc[i];
    }
}

// ln T of every cell, read by the reverse sweep's LNT instances
__global__ void log_temperature_kernel(int64_t n, const double* __restrict__ T,
                                       double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = log(T[i]);
}

// pbar[row][f] = sum over workgroups of their sums, in workgroup order.
__global__ void vjp_reduce_kernel(int rows3, int blocks, const double* __restrict__ partial,
                                  double* __restrict__ pbar) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows3) return;
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += partial[size_t(b) * rows3 + idx];
    pbar[idx] = s;
}

template <int MAXOWN, int MAXPD, bool WITH_W, int JAC = 0, bool LNT = false>
hipError_t set_lds_vjp(int bytes) {
    return hipFuncSetAttribute(
        reinterpret_cast<const void*>(&vjp_kernel<MAXOWN, MAXPD, WITH_W, JAC, LNT>),
        hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

struct VjpArgs {
    int blocks;
    int64_t n, ld;
    const double *rho, *T, *Y, *wbar;
    double *Ybar, *Tbar, *wdot, *partial;
    const double* params;
    const double* lnT;     // ln T per cell, or NULL to evaluate it per tile
};

template <int MAXOWN, int MAXPD, bool LNT>
hipError_t launch_vjp_lnt(const pyro_mech* m, const VjpArgs& a, hipStream_t stream) {
    const size_t lds = vjp_lds_bytes(m);
    if (a.wdot)
        hipLaunchKernelGGL((vjp_kernel<MAXOWN, MAXPD, true, 0, LNT>), dim3(unsigned(a.blocks)),
                           dim3(kVjpWaves * 64), lds, stream, m->dev, a.n, a.ld, a.rho, a.T, a.Y,
                           a.wbar, a.Ybar, a.Tbar, a.wdot, a.partial, a.params, -1, a.lnT);
    else
        hipLaunchKernelGGL((vjp_kernel<MAXOWN, MAXPD, false, 0, LNT>), dim3(unsigned(a.blocks)),
                           dim3(kVjpWaves * 64), lds, stream, m->dev, a.n, a.ld, a.rho, a.T, a.Y,
                           a.wbar, a.Ybar, a.Tbar, a.wdot, a.partial, a.params, -1, a.lnT);
    return hipGetLastError();
}

template <int MAXOWN, int MAXPD>
hipError_t launch_vjp(const pyro_mech* m, const VjpArgs& a, hipStream_t stream) {
    return a.lnT ? launch_vjp_lnt<MAXOWN, MAXPD, true>(m, a, stream)
                 : launch_vjp_lnt<MAXOWN, MAXPD, false>(m, a, stream);
}

template <int MAXOWN>
hipError_t launch_vjp_own(const pyro_mech* m, const VjpArgs& a, hipStream_t stream) {
    if (m->vjp_max_pdw <= 4) return launch_vjp<MAXOWN, 4>(m, a, stream);
    if (m->vjp_max_pdw <= 8) return launch_vjp<MAXOWN, 8>(m, a, stream);
    return launch_vjp<MAXOWN, 16>(m, a, stream);
}

template <int MAXOWN>
hipError_t set_lds_own(int bytes) {
    hipError_t e = hipSuccess;
    const hipError_t all[] = {
        set_lds_vjp<MAXOWN, 4, false>(bytes), set_lds_vjp<MAXOWN, 8, false>(bytes),
        set_lds_vjp<MAXOWN, 16, false>(bytes), set_lds_vjp<MAXOWN, 4, true>(bytes),
        set_lds_vjp<MAXOWN, 8, true>(bytes), set_lds_vjp<MAXOWN, 16, true>(bytes),
        set_lds_vjp<MAXOWN, 4, false, 0, true>(bytes), set_lds_vjp<MAXOWN, 8, false, 0, true>(bytes),
        set_lds_vjp<MAXOWN, 16, false, 0, true>(bytes), set_lds_vjp<MAXOWN, 4, true, 0, true>(bytes),
        set_lds_vjp<MAXOWN, 8, true, 0, true>(bytes), set_lds_vjp<MAXOWN, 16, true, 0, true>(bytes),
        set_lds_vjp<MAXOWN, 4, false, 1>(bytes), set_lds_vjp<MAXOWN, 8, false, 1>(bytes),
        set_lds_vjp<MAXOWN, 16, false, 1>(bytes), set_lds_vjp<MAXOWN, 4, false, 2>(bytes),
        set_lds_vjp<MAXOWN, 8, false, 2>(bytes), set_lds_vjp<MAXOWN, 16, false, 2>(bytes)};
    for (hipError_t x : all)
        if (x != hipSuccess) e = x;
    return e;
}

// One launch per Jacobian row: row j's cotangent is W_j on species j.
template <int MAXOWN, int MAXPD, int JAC>
hipError_t launch_jacobian_rows(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                                const double* T, const double* Y, double* J, double* dSdT,
                                const double* params, bool tiled, hipStream_t stream) {
    const int64_t n_tiles = (n + kTile - 1) / kTile;
    const int blocks = int(std::min<int64_t>(n_tiles, int64_t(m->n_cu)));
    const size_t lds = vjp_lds_bytes(m);
    const int64_t S = m->S;
    const int64_t out_ld = tiled ? kTile : ld, out_tile = tiled ? S * S * kTile : kTile;
    // one launch per row (the rows looped inside each tile, after one
    // species phase, took longer: 17.6 against 16.2 ms for 2^18 cells)
    for (int j = 0; j < m->S; ++j) {
        hipLaunchKernelGGL((vjp_kernel<MAXOWN, MAXPD, false, JAC>), dim3(unsigned(blocks)),
                           dim3(kVjpWaves * 64), lds, stream, m->dev, n, ld, rho, T, Y, nullptr,
                           J, dSdT, nullptr, nullptr, params, j, nullptr, out_ld, out_tile, 1);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int MAXOWN, int JAC>
hipError_t launch_jacobian_own(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                               const double* T, const double* Y, double* J, double* dSdT,
                               const double* params, bool tiled, hipStream_t stream) {
    if (m->vjp_max_pdw <= 4)
        return launch_jacobian_rows<MAXOWN, 4, JAC>(m, n, ld, rho, T, Y, J, dSdT, params, tiled,
                                                    stream);
    if (m->vjp_max_pdw <= 8)
        return launch_jacobian_rows<MAXOWN, 8, JAC>(m, n, ld, rho, T, Y, J, dSdT, params, tiled,
                                                    stream);
    return launch_jacobian_rows<MAXOWN, 16, JAC>(m, n, ld, rho, T, Y, J, dSdT, params, tiled,
                                                 stream);
}

template <int JAC>
hipError_t launch_jacobian_mode(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                                const double* T, const double* Y, double* J, double* dSdT,
                                const double* params, bool tiled, hipStream_t stream) {
    if (m->vjp_max_own <= 4)
        return launch_jacobian_own<4, JAC>(m, n, ld, rho, T, Y, J, dSdT, params, tiled, stream);
    if (m->vjp_max_own <= 8)
        return launch_jacobian_own<8, JAC>(m, n, ld, rho, T, Y, J, dSdT, params, tiled, stream);
    return launch_jacobian_own<16, JAC>(m, n, ld, rho, T, Y, J, dSdT, params, tiled, stream);
}

// zeroes n doubles (a kernel rather than a memset node, for callers that
// capture the call in a graph)
__global__ void fill_zero_kernel(int n, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = 0.0;
}

hipError_t launch_vjp_with(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                           const double* T, const double* Y, const double* wbar, double* Ybar,
                           double* Tbar, double* params_bar, double* wdot, const double* params,
                           double* partial, int blocks, hipStream_t stream,
                           double* lnT = nullptr) {
    const int rows3 = 3 * (m->R + m->n_fo);
    if (lnT) {
        hipLaunchKernelGGL(log_temperature_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0,
                           stream, n, T, lnT);
        const hipError_t e0 = hipGetLastError();
        if (e0 != hipSuccess) return e0;
    }
    const VjpArgs a{blocks, n, ld, rho, T, Y, wbar, Ybar, Tbar, wdot, partial,
                    params ? params : m->dev.params, lnT};
    hipError_t e;
    if (m->vjp_max_own <= 4)
        e = launch_vjp_own<4>(m, a, stream);
    else if (m->vjp_max_own <= 8)
        e = launch_vjp_own<8>(m, a, stream);
    else
        e = launch_vjp_own<16>(m, a, stream);
    if (e == hipSuccess && rows3 > 0) {
        hipLaunchKernelGGL(vjp_reduce_kernel, dim3((rows3 + 255) / 256), dim3(256), 0, stream,
                           rows3, blocks, a.partial, params_bar);
        e = hipGetLastError();
    }
    return e;
}

// The allocation-free entry point's scratch: the per-workgroup parameter
// partials live in this fixed array, one copy per device, its address looked
// up once per device when a mechanism is loaded there.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// The fixed device array itself (host code uses the address looked up per
// device, never this name: in host code it is only a stand-in symbol).
static __device__ __align__(256) double scratch[kVjpScratchDoubles];

hipError_t vjp_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
    return hipSuccess;
}

int vjp_scratch_blocks(const pyro_mech* m, int64_t n) {
    const int64_t n_tiles = (n + kTile - 1) / kTile;
    return int(std::min<int64_t>(n_tiles, int64_t(m->n_cu)));
}

hipError_t launch_production_rates_vjp_noalloc(const pyro_mech* m, int64_t n, int64_t ld,
                                               const double* rho, const double* T,
                                               const double* Y, const double* wbar,
                                               double* Ybar, double* Tbar, double* params_bar,
                                               double* wdot, const double* params,
                                               hipStream_t stream) {
    double* ptr = nullptr;   // this device's copy of the scratch array
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (m->device >= 0 && m->device < kMaxDevices) ptr = g_scratch_ptr[m->device];
    }
    if (!ptr) return hipErrorNotInitialized;
    const int rows3 = 3 * (m->R + m->n_fo);
    if (n == 0) {
        if (rows3 > 0)
            hipLaunchKernelGGL(fill_zero_kernel, dim3((rows3 + 255) / 256), dim3(256), 0, stream,
                               rows3, params_bar);
        return hipGetLastError();
    }
    return launch_vjp_with(m, n, ld, rho, T, Y, wbar, Ybar, Tbar, params_bar, wdot, params,
                           ptr, vjp_scratch_blocks(m, n), stream);
}

hipError_t launch_chemical_jacobian(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                                    const double* T, const double* Y, int fixed_energy,
                                    double* J, double* dSdT, const double* params,
                                    hipStream_t stream) {
    const double* p = params ? params : m->dev.params;
    if (fixed_energy)
        return launch_jacobian_mode<2>(m, n, ld, rho, T, Y, J, dSdT, p, false, stream);
    return launch_jacobian_mode<1>(m, n, ld, rho, T, Y, J, dSdT, p, false, stream);
}

hipError_t launch_chemical_jacobian_tiled(const pyro_mech* m, int64_t n, int64_t ld,
                                          const double* rho, const double* T, const double* Y,
                                          double* J, hipStream_t stream) {
    return launch_jacobian_mode<2>(m, n, ld, rho, T, Y, J, nullptr, m->dev.params, true, stream);
}

size_t vjp_lds_bytes(const pyro_mech* m) {
    return size_t(m->S) * kVRow + vjp_region_bytes(m->n_tb + m->n_fo) +
           size_t(m->R + m->n_fo) * 3 * 8;
}

hipError_t prepare_vjp(const pyro_mech* m) {
    // the allocation-free entry point's scratch address on this device
    const hipError_t es = vjp_scratch_init(m->device);
    if (es != hipSuccess) return es;
    const size_t bytes = vjp_lds_bytes(m);
    if (bytes > 160 * 1024) return hipSuccess;  // the VJP call reports it as unsupported
    const int lds = int(bytes);
    hipError_t e = hipSuccess;
    const hipError_t all[] = {set_lds_own<4>(lds), set_lds_own<8>(lds), set_lds_own<16>(lds)};
    for (hipError_t x : all)
        if (x != hipSuccess) e = x;
    return e;
}

hipError_t launch_production_rates_vjp(const pyro_mech* m, int64_t n, int64_t ld,
                                       const double* rho, const double* T, const double* Y,
                                       const double* wbar, double* Ybar, double* Tbar,
                                       double* params_bar, double* wdot, const double* params,
                                       hipStream_t stream) {
    const int blocks = vjp_scratch_blocks(m, n);
    const int rows3 = 3 * (m->R + m->n_fo);
    // workspace: the per-workgroup parameter partials, then ln T per cell
    const size_t pbytes = (size_t(blocks) * rows3 + size_t(n)) * sizeof(double);
    void* partial = nullptr;
    hipError_t e = hipMallocAsync(&partial, pbytes > 0 ? pbytes : 8, stream);
    if (e != hipSuccess) return e;
    double* pd = static_cast<double*>(partial);
    e = launch_vjp_with(m, n, ld, rho, T, Y, wbar, Ybar, Tbar, params_bar, wdot, params, pd,
                        blocks, stream, pd + size_t(blocks) * rows3);
    const hipError_t ef = hipFreeAsync(partial, stream);
    return e != hipSuccess ? e : ef;
}

}  // namespace pyro
