// Homogeneous adiabatic isochoric reactor steps at constant density and
// internal energy (eq. massfrac_ode: rho dY/dt = W omega), the temperature
// of every evaluation coming from the Newton kernel:
//
//  * classical Runge-Kutta, four stages (the paper's explicit marching):
//    the stage kernel turns the production rates of a stage into
//    k = W omega/rho, accumulates b_s k and forms the next stage state;
//  * Crank-Nicolson solved by Newton (eq. crank_nicol_rhs,
//    eq. crank_nicol_newton_update, eq. crank_nicol_jac): per update, the
//    solve kernel forms F = Y - Y^m - dt/(2 rho) (S + S^m) and
//    A = I - dt/(2 rho) J in place of J, factors A by Gaussian elimination
//    with partial pivoting and applies Y <- Y + A^-1 (-F).  Up to 64
//    species, one cell per wavefront: lane r holds row r of A in registers,
//    each column's pivot is the largest row not yet a pivot (a wave maximum),
//    the pivot row reaches the other lanes by v_readlane, and the column
//    leaves every other row (Gauss-Jordan, so no back substitution; rows are
//    never moved).  Past 64 species, one cell per lane with the matrix in
//    device memory, Gaussian elimination and back substitution.  The
//    Jacobian comes in 64-cell tiles of whole matrices (one cell's matrix
//    within 64 S^2 doubles, not spread over S^2 rows of all cells, which
//    costs a translation miss per element at 2^18 cells), and once some cells
//    have converged, the Jacobian and the solve run on the others only,
//    gathered in ascending order.
#include <type_traits>

#include "pyro_internal.h"
#include "surrogate_internal.h"

namespace pyro {
namespace {

constexpr int kRBlock = 256;

// Runge-Kutta stage s (0..3): k = W w/rho; acc (+)= b_s k; for s < 3 the next
// stage state Ys = Y + c_{s+1} dt k, for s == 3 the new state Y += dt acc.
// Stage status folds into ok (cleared by the first failed inversion).
__global__ __launch_bounds__(kRBlock) void rk4_stage_kernel(
    DevMech m, int64_t n, int64_t ld, int s, const double* __restrict__ rho,
    const double* __restrict__ dt, double dt_value, const double* __restrict__ w,
    double* __restrict__ acc, double* __restrict__ Ys, double* __restrict__ Y,
    const int32_t* __restrict__ st, int32_t* __restrict__ ok) {
    const int64_t i = int64_t(blockIdx.x) * kRBlock + threadIdx.x;
    if (i >= n) return;
    const double h = dt ? dt[i] : dt_value;
    const double ir = 1.0 / rho[i];
    const double b = (s == 0 || s == 3) ? 1.0 / 6.0 : 1.0 / 3.0;
    const double cnext = s < 2 ? 0.5 : 1.0;
    const cptr<double> W = cst(m.w);
    for (int k = 0; k < m.S; ++k) {
        const size_t o = size_t(k) * ld + i;
        const double kk = W[k] * w[o] * ir;
        const double a = s == 0 ? b * kk : fma(b, kk, acc[o]);
        if (s < 3) {
            acc[o] = a;
            Ys[o] = fma(cnext * h, kk, Y[o]);
        } else {
            Y[o] = fma(h, a, Y[o]);
        }
    }
    ok[i] = (s == 0 ? 1 : ok[i]) & (st[i] > 0 ? 1 : 0);
}

// f = W w/rho (the right-hand side dY/dt)
__global__ __launch_bounds__(kRBlock) void rhs_kernel(DevMech m, int64_t n, int64_t ld,
                                                      const double* __restrict__ rho,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ f) {
    const int64_t i = int64_t(blockIdx.x) * kRBlock + threadIdx.x;
    if (i >= n) return;
    const double ir = 1.0 / rho[i];
    const cptr<double> W = cst(m.w);
    for (int k = 0; k < m.S; ++k) f[size_t(k) * ld + i] = W[k] * w[size_t(k) * ld + i] * ir;
}

// One Newton update of the Crank-Nicolson system for every cell still
// active.  Work item j is cell idx[j] (cell j when idx is null); J holds
// dS/dY at the iterate of work item j in 64-item tiles of whole matrices
// (element (r, q) at J[((j / 64) S S + r S + q) 64 + j % 64]) and is
// overwritten by the factors of A = I - dt/(2 rho) J, F [S][ldj] by the
// update.
__global__ __launch_bounds__(kRBlock) void cn_solve_kernel(
    DevMech m, int64_t nwork, int64_t ld, const int64_t* __restrict__ idx, int64_t ldj, int it,
    double tol, const double* __restrict__ rho, const double* __restrict__ dt, double dt_value,
    const double* __restrict__ Y0, const double* __restrict__ f0, const double* __restrict__ w,
    double* __restrict__ Yk, double* __restrict__ J, double* __restrict__ F,
    uint8_t* __restrict__ active, int32_t* __restrict__ status) {
    const int64_t j = int64_t(blockIdx.x) * kRBlock + threadIdx.x;
    if (j >= nwork) return;
    const int64_t i = idx ? idx[j] : j;
    if (!active[i]) return;
    const int S = m.S;
    const double hh = 0.5 * (dt ? dt[i] : dt_value);
    const double c = hh / rho[i];
    const cptr<double> W = cst(m.w);
    double* Jc = J + (j >> 6) * S * S * 64 + (j & 63);
    auto a = [&](int r, int col) -> double& { return Jc[(size_t(r) * S + col) * 64]; };
    auto v = [&](int r) -> double& { return F[size_t(r) * ldj + j]; };
    // right-hand side -F and the matrix A = I - c J
    for (int r = 0; r < S; ++r) {
        const size_t o = size_t(r) * ld + i;
        const double fr = W[r] * w[o] / rho[i];
        v(r) = -(Yk[o] - Y0[o] - hh * (fr + f0[o]));
        for (int col = 0; col < S; ++col) {
            const double x = -c * a(r, col);
            a(r, col) = r == col ? 1.0 + x : x;
        }
    }
    // Gaussian elimination with partial pivoting (rows swapped in place)
    for (int col = 0; col < S; ++col) {
        int p = col;
        double best = fabs(a(col, col));
        for (int r = col + 1; r < S; ++r) {
            const double x = fabs(a(r, col));
            if (x > best) {
                best = x;
                p = r;
            }
        }
        if (p != col) {
            for (int q = col; q < S; ++q) {
                const double t = a(col, q);
                a(col, q) = a(p, q);
                a(p, q) = t;
            }
            const double t = v(col);
            v(col) = v(p);
            v(p) = t;
        }
        const double inv = 1.0 / a(col, col);
        for (int r = col + 1; r < S; ++r) {
            const double l = a(r, col) * inv;
            if (l != 0.0) {
                for (int q = col + 1; q < S; ++q) a(r, q) = fma(-l, a(col, q), a(r, q));
                v(r) = fma(-l, v(col), v(r));
            }
        }
    }
    // back substitution, update and the stopping test
    double dmax = 0.0;
    for (int r = S - 1; r >= 0; --r) {
        double x = v(r);
        for (int q = r + 1; q < S; ++q) x = fma(-a(r, q), v(q), x);
        x /= a(r, r);
        v(r) = x;
        Yk[size_t(r) * ld + i] += x;
        dmax = fmax(dmax, fabs(x));
    }
    if (dmax <= tol) {
        active[i] = 0;
        status[i] = it + 1;
    }
}

// ---- one cell per wavefront (S <= 64)

constexpr int kWBlock = 512;   // eight cells per workgroup

// the maximum over the 64 lanes, in every lane (NaN lanes ignored)
__device__ inline float wave_max(float x) {
    auto dpp = [](float v, auto ctrl) {
        return __builtin_bit_cast(
            float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), decltype(ctrl)::value,
                                            0xf, 0xf, false));
    };
    x = fmaxf(x, dpp(x, std::integral_constant<int, 0x121>{}));   // row_ror:1
    x = fmaxf(x, dpp(x, std::integral_constant<int, 0x122>{}));   // row_ror:2
    x = fmaxf(x, dpp(x, std::integral_constant<int, 0x124>{}));   // row_ror:4
    x = fmaxf(x, dpp(x, std::integral_constant<int, 0x128>{}));   // row_ror:8
    const int b = __builtin_bit_cast(int, x);
    const auto s16 = __builtin_amdgcn_permlane16_swap(b, b, false, false);
    x = fmaxf(__builtin_bit_cast(float, int(s16[0])), __builtin_bit_cast(float, int(s16[1])));
    const int c = __builtin_bit_cast(int, x);
    const auto s32 = __builtin_amdgcn_permlane32_swap(c, c, false, false);
    return fmaxf(__builtin_bit_cast(float, int(s32[0])), __builtin_bit_cast(float, int(s32[1])));
}

// 1/d to within an ulp or so: the hardware estimate and two Newton steps
__device__ inline double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return fma(r, fma(-d, r, 1.0), r);
}

__device__ inline double read_lane(double v, int l) {
    const int2 h = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(
        double, int2{__builtin_amdgcn_readlane(h.x, l), __builtin_amdgcn_readlane(h.y, l)});
}

__device__ inline int first_lane(uint64_t mask) { return int(__builtin_ctzll(mask)); }

// Workgroups are dealt round-robin over the eight XCDs; renumbering them so
// that each XCD runs one contiguous range of cells keeps the cells that share
// a cache line of J in one L2.
__device__ inline int64_t xcd_contiguous(int64_t b, int64_t nb) {
    const int64_t x = b % 8, j = b / 8, q = nb / 8, r = nb % 8;
    return x * q + (x < r ? x : r) + j;
}

// One Newton update (as cn_solve_kernel, work item j for cell idx[j]) for
// the cells still active, one cell per wavefront, NC >= S columns of the
// cell's row per lane.
template <int NC>
__global__ __launch_bounds__(kWBlock) __attribute__((amdgpu_waves_per_eu(3))) void cn_solve_wave_kernel(
    DevMech m, int64_t nwork, int64_t ld, const int64_t* __restrict__ idx, int64_t ldj, int it,
    double tol, const double* __restrict__ rho, const double* __restrict__ dt, double dt_value,
    const double* __restrict__ Y0, const double* __restrict__ f0, const double* __restrict__ w,
    double* __restrict__ Yk, const double* __restrict__ J, uint8_t* __restrict__ active,
    int32_t* __restrict__ status) {
    const int lane = threadIdx.x & 63;
    const int64_t blk = xcd_contiguous(blockIdx.x, gridDim.x);
    const int64_t j = blk * (kWBlock / 64) + (threadIdx.x >> 6);
    if (j >= nwork) return;   // uniform over the wavefront
    const int64_t i = idx ? idx[j] : j;
    if (!active[i]) return;
    const int S = m.S;
    const bool row = lane < S;
    const double hh = 0.5 * (dt ? dt[i] : dt_value);
    const double c = hh / rho[i];
    // row r of A = I - c J (zero past column S) and of the right-hand side -F
    double a[NC];
    double v = 0.0;
    if (row) {
        const size_t o = size_t(lane) * ld + i;
        const double fr = m.w[lane] * w[o] / rho[i];
        v = -(Yk[o] - Y0[o] - hh * (fr + f0[o]));
    }
    // (every lane loads, the lanes past S from row 0 and the columns past S
    // from column S - 1; the empty asm makes each value live in every lane,
    // so that the compiler does not move the loads into branches, one wait
    // each, but issues them all before the first use)
    const double* Jr = J + (j >> 6) * S * S * 64 + (j & 63) + size_t(row ? lane : 0) * S * 64;
#pragma unroll
    for (int q = 0; q < NC; ++q) a[q] = Jr[size_t(q < S ? q : S - 1) * 64];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        asm volatile("" : "+v"(a[q]));
        const double x = -c * a[q];
        a[q] = row && q < S ? (lane == q ? 1.0 + x : x) : 0.0;
    }
    // Gauss-Jordan elimination with each row shifted one register left per
    // column, so that the current column is always a[0]: column col leaves
    // every row but the pivot's, and the pivot row keeps its diagonal in
    // diag.  Columns go in tiers of eight; the loop over a tier's columns is
    // not unrolled (a fully unrolled elimination outgrows the instruction
    // cache), and tier t updates the NC - 8 t registers that can still hold
    // a column below S.
    bool done = !row;
    int mycol = 0;
    double diag = 1.0;
#pragma unroll
    for (int t = 0; t < NC / 8; ++t) {
#pragma nounroll
        for (int u = 0; u < 8; ++u) {
            const int col = 8 * t + u;
            if (col >= S) break;
            // the pivot: the largest |a| of the rows not yet pivots, compared
            // in single precision (a row within a float rounding of the
            // largest serves as well)
            const float key = done ? -1.0f : float(fabs(a[0]));
            const float best = wave_max(key);
            uint64_t hit = __ballot(!done && key == best);
            if (hit == 0) hit = __ballot(!done);   // a column of NaN
            const int p = first_lane(hit);
            const double d = read_lane(a[0], p);
            const bool me = lane == p;
            if (me) {
                done = true;
                mycol = col;
                diag = d;
            }
            const double l = me ? 0.0 : a[0] * recip(d);
#pragma unroll
            for (int q = 1; q < NC - 8 * t; ++q) a[q - 1] = fma(-l, read_lane(a[q], p), a[q]);
            a[NC - 8 * t - 1] = 0.0;
            v = fma(-l, read_lane(v, p), v);
        }
    }
    // the row that was pivot of column k now reads diag x_k = v
    const double x = v / diag;
    if (row) Yk[size_t(mycol) * ld + i] += x;
    // converged once every component of the update is within tol
    if (__ballot(row && !(fabs(x) <= tol)) == 0 && lane == 0) {
        active[i] = 0;
        status[i] = it + 1;
    }
}

__global__ __launch_bounds__(kRBlock) void cn_init_kernel(int64_t n, int32_t max_iter,
                                                          uint8_t* __restrict__ active,
                                                          int32_t* __restrict__ status) {
    const int64_t i = int64_t(blockIdx.x) * kRBlock + threadIdx.x;
    if (i >= n) return;
    active[i] = 1;
    status[i] = -max_iter;
}

// status of the step: the Newton count, or 0 where a temperature inversion
// failed on the way (ok == 0)
__global__ __launch_bounds__(kRBlock) void fold_status_kernel(int64_t n,
                                                              const int32_t* __restrict__ ok,
                                                              int32_t* __restrict__ status) {
    const int64_t i = int64_t(blockIdx.x) * kRBlock + threadIdx.x;
    if (i < n && !ok[i]) status[i] = 0;
}

unsigned rgrid(int64_t n) { return unsigned((n + kRBlock - 1) / kRBlock); }

// cells spanned by the tiled Jacobian (whole 64-cell tiles), at least ld
size_t jcols(int64_t n, int64_t ld) {
    const int64_t t = (n + 63) / 64 * 64;
    return size_t(t > ld ? t : ld);
}

// workspace carve-up: 256-byte aligned pieces
struct Carve {
    char* p;
    size_t used = 0;
    template <typename T>
    T* take(size_t count) {
        T* r = reinterpret_cast<T*>(p + used);
        used += (count * sizeof(T) + 255) / 256 * 256;
        return r;
    }
};

}  // namespace

size_t reactor_workspace_bytes(const pyro_mech* m, int64_t n, int64_t ld, int method) {
    Carve c{nullptr};
    const size_t sl = size_t(m->S) * ld;
    if (method == 0) {
        c.take<double>(sl); c.take<double>(sl); c.take<double>(sl);   // acc, Ys, w
        c.take<double>(n); c.take<int32_t>(n); c.take<int32_t>(n);     // T, stage status, ok
    } else {
        c.take<double>(sl); c.take<double>(sl); c.take<double>(sl);   // f0, Y0, w
        c.take<double>(size_t(m->S) * m->S * jcols(n, ld));           // J, 64-cell tiles
        c.take<double>(sl);                                           // F
        c.take<double>(n); c.take<int32_t>(n); c.take<uint8_t>(n);     // Tk, st, active
        c.take<int64_t>(size_t(compaction_blocks(n)));                // block offsets
        c.take<int64_t>(1); c.take<int64_t>(n);                        // count, idx
        c.take<double>(n); c.take<double>(n);                          // rho, T gathered
        c.take<double>(size_t(m->S) * n);                             // Y gathered
    }
    return c.used;
}

hipError_t launch_rk4_step(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                           const double* e, double* Y, double* T, const double* dt,
                           double dt_value, int32_t* status, void* ws, hipStream_t s) {
    Carve c{static_cast<char*>(ws)};
    const size_t sl = size_t(m->S) * ld;
    double* acc = c.take<double>(sl);
    double* Ys = c.take<double>(sl);
    double* w = c.take<double>(sl);
    double* Ts = c.take<double>(n);
    int32_t* st = c.take<int32_t>(n);
    int32_t* ok = c.take<int32_t>(n);
    hipError_t e1;
    for (int stg = 0; stg < 4; ++stg) {
        const double* Yin = stg == 0 ? Y : Ys;
        e1 = launch_temperature(m, n, ld, e, Yin, stg == 0 ? T : Ts, 0.0, Ts, st, 50, 1e-12, s);
        if (e1 != hipSuccess) return e1;
        e1 = launch_production_rates(m, n, ld, PYRO_F64, rho, Ts, Yin, w, nullptr, s);
        if (e1 != hipSuccess) return e1;
        hipLaunchKernelGGL(rk4_stage_kernel, dim3(rgrid(n)), dim3(kRBlock), 0, s, m->dev, n, ld,
                           stg, rho, dt, dt_value, w, acc, Ys, Y, st, ok);
        e1 = hipGetLastError();
        if (e1 != hipSuccess) return e1;
    }
    e1 = launch_temperature(m, n, ld, e, Y, Ts, 0.0, T, status, 50, 1e-12, s);
    if (e1 != hipSuccess) return e1;
    hipLaunchKernelGGL(fold_status_kernel, dim3(rgrid(n)), dim3(kRBlock), 0, s, n, ok, status);
    return hipGetLastError();
}

hipError_t launch_cn_step(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                          const double* e, double* Y, double* T, const double* dt,
                          double dt_value, double tol, int max_iter, int32_t* status, void* ws,
                          hipStream_t s) {
    Carve c{static_cast<char*>(ws)};
    const int S = m->S;
    const size_t sl = size_t(S) * ld;
    double* f0 = c.take<double>(sl);
    double* Y0 = c.take<double>(sl);
    double* w = c.take<double>(sl);
    double* J = c.take<double>(size_t(S) * S * jcols(n, ld));
    double* F = c.take<double>(sl);
    double* Tk = c.take<double>(n);
    int32_t* st = c.take<int32_t>(n);
    uint8_t* active = c.take<uint8_t>(n);
    int64_t* offs = c.take<int64_t>(size_t(compaction_blocks(n)));
    int64_t* count = c.take<int64_t>(1);
    int64_t* idx = c.take<int64_t>(n);
    double* rc = c.take<double>(n);
    double* Tc = c.take<double>(n);
    double* Yc = c.take<double>(size_t(S) * n);
    hipError_t e1;
    // S^m at the old state; Y0 keeps Y^m, Y becomes the iterate
    e1 = launch_temperature(m, n, ld, e, Y, T, 0.0, Tk, st, 50, 1e-12, s);
    if (e1 != hipSuccess) return e1;
    e1 = launch_production_rates(m, n, ld, PYRO_F64, rho, Tk, Y, w, nullptr, s);
    if (e1 != hipSuccess) return e1;
    hipLaunchKernelGGL(rhs_kernel, dim3(rgrid(n)), dim3(kRBlock), 0, s, m->dev, n, ld, rho, w, f0);
    e1 = hipMemcpy2DAsync(Y0, ld * sizeof(double), Y, ld * sizeof(double), n * sizeof(double),
                          S, hipMemcpyDeviceToDevice, s);
    if (e1 != hipSuccess) return e1;
    hipLaunchKernelGGL(cn_init_kernel, dim3(rgrid(n)), dim3(kRBlock), 0, s, n, max_iter, active,
                       status);
    // left: cells still iterating; once some have converged, the Jacobian
    // and the solve run on the others only, gathered in ascending order
    // into dense arrays (the production rates and temperatures stay
    // full-size: they cost a few percent of an update)
    int64_t left = n;
    for (int it = 0; it < max_iter; ++it) {
        e1 = launch_temperature(m, n, ld, e, Y, Tk, 0.0, Tk, st, 50, 1e-12, s);
        if (e1 != hipSuccess) return e1;
        e1 = launch_production_rates(m, n, ld, PYRO_F64, rho, Tk, Y, w, nullptr, s);
        if (e1 != hipSuccess) return e1;
        const bool packed = left < n;
        const int64_t ldj = packed ? left : ld;
        const int64_t* map = packed ? idx : nullptr;
        if (packed) {
            e1 = launch_gather(S, left, ld, count, idx, rho, Tk, Y, rc, Tc, Yc, s);
            if (e1 != hipSuccess) return e1;
            e1 = launch_chemical_jacobian_tiled(m, left, left, rc, Tc, Yc, J, s);
        } else {
            e1 = launch_chemical_jacobian_tiled(m, n, ld, rho, Tk, Y, J, s);
        }
        if (e1 != hipSuccess) return e1;
        if (S <= 64) {
            const unsigned wg = unsigned((left + kWBlock / 64 - 1) / (kWBlock / 64));
            const auto k = S <= 16 ? cn_solve_wave_kernel<16>
                         : S <= 32 ? cn_solve_wave_kernel<32>
                         : S <= 48 ? cn_solve_wave_kernel<48>
                         : S <= 56 ? cn_solve_wave_kernel<56>
                                   : cn_solve_wave_kernel<64>;
            hipLaunchKernelGGL(k, dim3(wg), dim3(kWBlock), 0, s, m->dev, left, ld, map, ldj, it,
                               tol, rho, dt, dt_value, Y0, f0, w, Y, J, active, status);
        } else {
            hipLaunchKernelGGL(cn_solve_kernel, dim3(rgrid(left)), dim3(kRBlock), 0, s, m->dev,
                               left, ld, map, ldj, it, tol, rho, dt, dt_value, Y0, f0, w, Y, J, F,
                               active, status);
        }
        e1 = hipGetLastError();
        if (e1 != hipSuccess) return e1;
        // the cells still active, and their number (stop once it is zero:
        // the remaining iterations would recompute Jacobians for nothing)
        e1 = launch_compaction(n, active, offs, count, idx, s);
        if (e1 != hipSuccess) return e1;
        e1 = hipMemcpyAsync(&left, count, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e1 == hipSuccess) e1 = hipStreamSynchronize(s);
        if (e1 != hipSuccess) return e1;
        if (left == 0) break;
    }
    return launch_temperature(m, n, ld, e, Y, Tk, 0.0, T, st, 50, 1e-12, s);
}

}  // namespace pyro
