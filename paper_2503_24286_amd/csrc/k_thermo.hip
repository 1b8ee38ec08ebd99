// Per-cell mixture thermodynamics: Newton inversion of T from the internal
// energy (Appendix A.3.1: eq. int_energy, eq. delta_temp, eq. cv), the
// mixture internal energy, and the equation of state (Appendix A.1, eq. eos).
//
// The mixture energy is linear in the NASA7 coefficients, so one pass over
// the species folds them, weighted by X_k = Y_k/W_k, into six mixture
// coefficients per range (and per distinct T_mid); every Newton iterate then
// costs a handful of FMAs instead of a pass over the species:
//   e(T)   = R [ A1 T + A2 T^2/2 + A3 T^3/3 + A4 T^4/4 + A5 T^5/5 + A6 - T sum X ]
//   c_v(T) = R [ A1 + A2 T + A3 T^2 + A4 T^3 + A5 T^4 - sum X ]
// with A_m = sum_k X_k a_m,k over the species whose range holds T.  The pass
// reads Y once (coalesced), so the kernel is bound by HBM bandwidth.
#include "pyro_internal.h"

namespace pyro {
namespace {

constexpr int kBlock = 256;

struct Mixture {
    double A[kMaxTmidGroups][2][6];
    double xsum;
};

// (ysum, when given, receives sum_k Y_k from the same pass)
template <int NG>
__device__ inline void fold(const DevMech& m, const double* __restrict__ Y, int64_t ld,
                            int64_t c, Mixture& mx, double* ysum = nullptr) {
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int q = 0; q < 6; ++q) mx.A[g][r][q] = 0.0;
    mx.xsum = 0.0;
    double ys = 0.0;
    auto add = [&](int k, double y) {
        const NewtonSpecies& s = m.newton[k];
        const double X = y * s.inv_w;
        ys += y;
        mx.xsum += X;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (s.group == g) {
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    mx.A[g][0][q] = fma(X, s.lo[q], mx.A[g][0][q]);
                    mx.A[g][1][q] = fma(X, s.hi[q], mx.A[g][1][q]);
                }
            }
        }
    };
    // eight loads in flight at a time, then their terms in species order
    int k = 0;
    for (; k + 8 <= m.S; k += 8) {
        double y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) y[u] = Y[size_t(k + u) * ld + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) add(k + u, y[u]);
    }
    for (; k < m.S; ++k) add(k, Y[size_t(k) * ld + c]);
    if (ysum) *ysum = ys;
}

// fold over values already in registers, y[k] for k < S <= NR (same
// arithmetic and order as fold)
template <int NG, int NR>
__device__ inline void fold_values(const DevMech& m, const double* y, Mixture& mx,
                                   double* ysum) {
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int q = 0; q < 6; ++q) mx.A[g][r][q] = 0.0;
    mx.xsum = 0.0;
    double ys = 0.0;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        if (k < m.S) {
            const NewtonSpecies& s = m.newton[k];
            const double X = y[k] * s.inv_w;
            ys += y[k];
            mx.xsum += X;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                if (s.group == g) {
#pragma unroll
                    for (int q = 0; q < 6; ++q) {
                        mx.A[g][0][q] = fma(X, s.lo[q], mx.A[g][0][q]);
                        mx.A[g][1][q] = fma(X, s.hi[q], mx.A[g][1][q]);
                    }
                }
            }
        }
    }
    *ysum = ys;
}

// Divides the folded coefficients by d (a fold over partial densities
// rho_k then gives the fold over Y_k = rho_k/rho).
template <int NG>
__device__ inline void scale(Mixture& mx, double d) {
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int q = 0; q < 6; ++q) mx.A[g][r][q] /= d;
    mx.xsum /= d;
}

// e(T)/R and c_v(T)/R of the folded mixture, or with ENTHALPY h(T)/R and
// c_p(T)/R (the same sums without the -R T and -R per mole of species).
template <int NG, bool ENTHALPY = false>
__device__ inline void energy(const DevMech& m, const Mixture& mx, double T, double& e_R,
                              double& cv_R) {
    double h = 0.0, cp = 0.0;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const bool low = T <= m.t_mid_group[g];
        double a[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) a[q] = low ? mx.A[g][0][q] : mx.A[g][1][q];
        h += a[5] + T * (a[0] + T * (a[1] * 0.5 + T * (a[2] * (1.0 / 3.0) +
                              T * (a[3] * 0.25 + T * (a[4] * 0.2)))));
        cp += a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
    }
    if constexpr (ENTHALPY) {
        e_R = h;
        cv_R = cp;
    } else {
        e_R = h - T * mx.xsum;
        cv_R = cp - mx.xsum;
    }
}

// Newton updates T <- T - (value(T) - target)/slope(T) until the first
// update with |dT| <= rtol |T| (status = updates taken) or max_iter updates
// (status = -max_iter); the loop runs while any lane of the wave is active.
template <int NG, bool ENTHALPY>
__device__ inline double newton_solve(const DevMech& m, const Mixture& mx, double target_R,
                                      double T, bool valid, int max_iter, double rtol,
                                      int32_t& st) {
    st = -max_iter;
    bool active = valid;
    for (int it = 0; it < max_iter; ++it) {
        if (!__any(active)) break;
        if (active) {
            double eR, cvR;
            energy<NG, ENTHALPY>(m, mx, T, eR, cvR);
            const double dT = -(eR - target_R) / cvR;
            T += dT;
            if (fabs(dT) <= rtol * fabs(T)) {
                st = it + 1;
                active = false;
            }
        }
    }
    return T;
}

// ENTHALPY: the target is the mass-specific enthalpy (the variant closing
// Sec. A.3.1), else the internal energy (eq. delta_temp).
template <int NG, bool ENTHALPY>
__global__ __launch_bounds__(kBlock) void newton_kernel(
    DevMech m, int64_t n, int64_t ld, const double* __restrict__ e,
    const double* __restrict__ Y, const double* __restrict__ Tg, double Tg_value,
    double* __restrict__ T_out, int32_t* __restrict__ status, int max_iter, double rtol) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const bool valid = i < n;
    const int64_t c = valid ? i : n - 1;
    Mixture mx;
    fold<NG>(m, Y, ld, c, mx);
    int32_t st;
    const double T = newton_solve<NG, ENTHALPY>(m, mx, e[c] * (1.0 / kGasConstant),
                                                Tg ? Tg[c] : Tg_value, valid, max_iter, rtol, st);
    if (valid) {
        T_out[i] = T;
        status[i] = st;
    }
}

// Primitive from conserved variables per cell, in the order of the paper's
// equation-of-state routine (Sec. "Python Code Generation and Immediate
// Execution using NumPy"): rho = sum_k rho_k, Y_k = rho_k/rho, u = m/rho,
// e = E/rho - |u|^2/2, T by the Newton inversion of e, p = rho R T/W.  The
// partial densities are read once to form rho and the energy fold (over
// rho_k/W_k, then divided by rho) in one pass; with NR > 0 (S <= NR) they stay
// in registers for Y, else they are read again to write Y.
template <int NG, int NR>
__global__ __launch_bounds__(kBlock) void primitive_kernel(
    DevMech m, int64_t n, int64_t ld, int dim, const double* __restrict__ rhok,
    const double* __restrict__ mom, const double* __restrict__ E,
    const double* __restrict__ Tg, double Tg_value, double* __restrict__ rho_out,
    double* __restrict__ Y_out, double* __restrict__ u_out, double* __restrict__ T_out,
    double* __restrict__ p_out, int32_t* __restrict__ status, int max_iter, double rtol) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const bool valid = i < n;
    const int64_t c = valid ? i : n - 1;
    Mixture mx;
    double rho;
    double rk[NR > 0 ? NR : 1];
    if constexpr (NR > 0) {
        // all loads issued together (species past S read species S - 1)
#pragma unroll
        for (int k = 0; k < NR; ++k) rk[k] = rhok[size_t(k < m.S ? k : m.S - 1) * ld + c];
        fold_values<NG, NR>(m, rk, mx, &rho);
    } else {
        fold<NG>(m, rhok, ld, c, mx, &rho);   // coefficients weighted by rho_k/W_k
    }
    scale<NG>(mx, rho);             // now weighted by Y_k/W_k; xsum = 1/W
    double kin = 0.0;
    for (int d = 0; d < dim; ++d) {
        const double u = mom[size_t(d) * ld + c] / rho;
        kin = fma(u, u, kin);
        if (valid) u_out[size_t(d) * ld + i] = u;
    }
    const double e = E[c] / rho - 0.5 * kin;
    int32_t st;
    const double T = newton_solve<NG, false>(m, mx, e * (1.0 / kGasConstant),
                                             Tg ? Tg[c] : Tg_value, valid, max_iter, rtol, st);
    if (!valid) return;
    if constexpr (NR > 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k)
            if (k < m.S) Y_out[size_t(k) * ld + i] = rk[k] / rho;
    } else {
        for (int k = 0; k < m.S; ++k) Y_out[size_t(k) * ld + i] = rhok[size_t(k) * ld + i] / rho;
    }
    rho_out[i] = rho;
    T_out[i] = T;
    p_out[i] = rho * kGasConstant * T * mx.xsum;
    status[i] = st;
}

template <int NG>
__global__ __launch_bounds__(kBlock) void energy_kernel(DevMech m, int64_t n, int64_t ld,
                                                        const double* __restrict__ T,
                                                        const double* __restrict__ Y,
                                                        double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    Mixture mx;
    fold<NG>(m, Y, ld, i, mx);
    double eR, cvR;
    energy<NG>(m, mx, T[i], eR, cvR);
    out[i] = eR * kGasConstant;
}

// mode 0: a = p, out = rho; mode 1: a = rho, out = p
__global__ __launch_bounds__(kBlock) void eos_kernel(DevMech m, int64_t n, int64_t ld, int mode,
                                                     const double* __restrict__ a,
                                                     const double* __restrict__ T,
                                                     const double* __restrict__ Y,
                                                     double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    double x = 0.0;
    for (int k = 0; k < m.S; ++k) x += Y[size_t(k) * ld + i] * m.newton[k].inv_w;
    // x = 1/W (mixture)
    const double RT = kGasConstant * T[i];
    out[i] = mode == 0 ? a[i] / (x * RT) : a[i] * RT * x;
}

unsigned grid(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

}  // namespace

namespace {
template <bool ENTHALPY>
hipError_t launch_newton(const pyro_mech* m, int64_t n, int64_t ld, const double* e,
                         const double* Y, const double* T_guess, double T_guess_value,
                         double* T_out, int32_t* status, int max_iter, double rtol,
                         hipStream_t stream) {
    switch (m->dev.n_groups) {
        case 1:
            hipLaunchKernelGGL((newton_kernel<1, ENTHALPY>), dim3(grid(n)), dim3(kBlock), 0,
                               stream, m->dev, n, ld, e, Y, T_guess, T_guess_value, T_out, status,
                               max_iter, rtol);
            break;
        case 2:
            hipLaunchKernelGGL((newton_kernel<2, ENTHALPY>), dim3(grid(n)), dim3(kBlock), 0,
                               stream, m->dev, n, ld, e, Y, T_guess, T_guess_value, T_out, status,
                               max_iter, rtol);
            break;
        default:
            hipLaunchKernelGGL((newton_kernel<kMaxTmidGroups, ENTHALPY>), dim3(grid(n)),
                               dim3(kBlock), 0, stream, m->dev, n, ld, e, Y, T_guess,
                               T_guess_value, T_out, status, max_iter, rtol);
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_temperature(const pyro_mech* m, int64_t n, int64_t ld, const double* e,
                              const double* Y, const double* T_guess, double T_guess_value,
                              double* T_out, int32_t* status, int max_iter, double rtol,
                              hipStream_t stream, bool enthalpy) {
    if (enthalpy)
        return launch_newton<true>(m, n, ld, e, Y, T_guess, T_guess_value, T_out, status,
                                   max_iter, rtol, stream);
    return launch_newton<false>(m, n, ld, e, Y, T_guess, T_guess_value, T_out, status, max_iter,
                                rtol, stream);
}

hipError_t launch_primitive(const pyro_mech* m, int64_t n, int64_t ld, int dim,
                            const double* rhok, const double* mom, const double* E,
                            const double* T_guess, double T_guess_value, double* rho_out,
                            double* Y_out, double* u_out, double* T_out, double* p_out,
                            int32_t* status, int max_iter, double rtol, hipStream_t stream) {
    // partial densities held in registers up to 64 species with one T_mid
    // group (one read of them); several groups' folds leave no room for them
    const int S = m->S;
    const auto k = m->dev.n_groups != 1 ? primitive_kernel<kMaxTmidGroups, 0>
                 : S <= 32              ? primitive_kernel<1, 32>
                 : S <= 56              ? primitive_kernel<1, 56>
                 : S <= 64              ? primitive_kernel<1, 64>
                                        : primitive_kernel<1, 0>;
    hipLaunchKernelGGL(k, dim3(grid(n)), dim3(kBlock), 0, stream, m->dev, n, ld, dim, rhok, mom, E,
                       T_guess, T_guess_value, rho_out, Y_out, u_out, T_out, p_out, status,
                       max_iter, rtol);
    return hipGetLastError();
}

hipError_t launch_internal_energy(const pyro_mech* m, int64_t n, int64_t ld, const double* T,
                                  const double* Y, double* e_out, hipStream_t stream) {
    if (m->dev.n_groups == 1)
        hipLaunchKernelGGL(energy_kernel<1>, dim3(grid(n)), dim3(kBlock), 0, stream, m->dev, n, ld,
                           T, Y, e_out);
    else
        hipLaunchKernelGGL(energy_kernel<kMaxTmidGroups>, dim3(grid(n)), dim3(kBlock), 0, stream,
                           m->dev, n, ld, T, Y, e_out);
    return hipGetLastError();
}

hipError_t launch_eos(const pyro_mech* m, int64_t n, int64_t ld, int mode, const double* a,
                      const double* T, const double* Y, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(eos_kernel, dim3(grid(n)), dim3(kBlock), 0, stream, m->dev, n, ld, mode, a,
                       T, Y, out);
    return hipGetLastError();
}

}  // namespace pyro
