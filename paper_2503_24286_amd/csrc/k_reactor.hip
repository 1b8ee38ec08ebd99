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
//    with partial pivoting and applies Y <- Y + A^-1 (-F).  One cell per
//    lane; the matrix of a cell stays in its (species-major, cell-strided)
//    device storage, so the loads of a lane group are coalesced except in
//    the rows it swapped.
#include "pyro_internal.h"

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
// active: J [S][S][ld] (dS/dY at the iterate) is overwritten by the factors
// of A = I - dt/(2 rho) J, F [S][ld] by the update.
__global__ __launch_bounds__(kRBlock) void cn_solve_kernel(
    DevMech m, int64_t n, int64_t ld, int it, double tol, const double* __restrict__ rho,
    const double* __restrict__ dt, double dt_value, const double* __restrict__ Y0,
    const double* __restrict__ f0, const double* __restrict__ w, double* __restrict__ Yk,
    double* __restrict__ J, double* __restrict__ F, int32_t* __restrict__ active,
    int32_t* __restrict__ status) {
    const int64_t i = int64_t(blockIdx.x) * kRBlock + threadIdx.x;
    if (i >= n || !active[i]) return;
    const int S = m.S;
    const double hh = 0.5 * (dt ? dt[i] : dt_value);
    const double c = hh / rho[i];
    const cptr<double> W = cst(m.w);
    auto a = [&](int r, int col) -> double& { return J[(size_t(r) * S + col) * ld + i]; };
    auto v = [&](int r) -> double& { return F[size_t(r) * ld + i]; };
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

// number of cells still iterating, in one workgroup (fixed order)
__global__ __launch_bounds__(kRBlock) void count_active_kernel(int64_t n,
                                                               const int32_t* __restrict__ active,
                                                               int32_t* __restrict__ count) {
    __shared__ int32_t part[kRBlock];
    int32_t c = 0;
    for (int64_t i = threadIdx.x; i < n; i += kRBlock) c += active[i];
    part[threadIdx.x] = c;
    __syncthreads();
    for (int h = kRBlock / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = part[0];
}

__global__ __launch_bounds__(kRBlock) void cn_init_kernel(int64_t n, int32_t max_iter,
                                                          int32_t* __restrict__ active,
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
        c.take<double>(sl); c.take<double>(sl); c.take<double>(sl);   // f0, Yk (unused), w
        c.take<double>(size_t(m->S) * sl);                            // J
        c.take<double>(sl);                                           // F
        c.take<double>(n); c.take<int32_t>(n); c.take<int32_t>(n); c.take<int32_t>(n);
        c.take<int32_t>(1);                                           // active count
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
    const size_t sl = size_t(m->S) * ld;
    double* f0 = c.take<double>(sl);
    double* Y0 = c.take<double>(sl);
    double* w = c.take<double>(sl);
    double* J = c.take<double>(size_t(m->S) * sl);
    double* F = c.take<double>(sl);
    double* Tk = c.take<double>(n);
    int32_t* st = c.take<int32_t>(n);
    int32_t* ok = c.take<int32_t>(n);
    int32_t* active = c.take<int32_t>(n);
    int32_t* count = c.take<int32_t>(1);
    hipError_t e1;
    // S^m at the old state; Y0 keeps Y^m, Y becomes the iterate
    e1 = launch_temperature(m, n, ld, e, Y, T, 0.0, Tk, st, 50, 1e-12, s);
    if (e1 != hipSuccess) return e1;
    e1 = launch_production_rates(m, n, ld, PYRO_F64, rho, Tk, Y, w, nullptr, s);
    if (e1 != hipSuccess) return e1;
    hipLaunchKernelGGL(rhs_kernel, dim3(rgrid(n)), dim3(kRBlock), 0, s, m->dev, n, ld, rho, w, f0);
    e1 = hipMemcpy2DAsync(Y0, ld * sizeof(double), Y, ld * sizeof(double), n * sizeof(double),
                          m->S, hipMemcpyDeviceToDevice, s);
    if (e1 != hipSuccess) return e1;
    hipLaunchKernelGGL(cn_init_kernel, dim3(rgrid(n)), dim3(kRBlock), 0, s, n, max_iter, active,
                       status);
    for (int it = 0; it < max_iter; ++it) {
        e1 = launch_temperature(m, n, ld, e, Y, Tk, 0.0, Tk, st, 50, 1e-12, s);
        if (e1 != hipSuccess) return e1;
        e1 = launch_production_rates(m, n, ld, PYRO_F64, rho, Tk, Y, w, nullptr, s);
        if (e1 != hipSuccess) return e1;
        e1 = launch_chemical_jacobian(m, n, ld, rho, Tk, Y, 1, J, nullptr, nullptr, s);
        if (e1 != hipSuccess) return e1;
        hipLaunchKernelGGL(cn_solve_kernel, dim3(rgrid(n)), dim3(kRBlock), 0, s, m->dev, n, ld,
                           it, tol, rho, dt, dt_value, Y0, f0, w, Y, J, F, active, status);
        hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(kRBlock), 0, s, n, active, count);
        e1 = hipGetLastError();
        if (e1 != hipSuccess) return e1;
        // stop once every cell has converged (the last iterations would
        // recompute every Jacobian for nothing)
        int32_t left = 0;
        e1 = hipMemcpyAsync(&left, count, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e1 == hipSuccess) e1 = hipStreamSynchronize(s);
        if (e1 != hipSuccess) return e1;
        if (left == 0) break;
    }
    return launch_temperature(m, n, ld, e, Y, Tk, 0.0, T, st, 50, 1e-12, s);
}

}  // namespace pyro
