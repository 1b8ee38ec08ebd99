// C ABI of libpyro (include/pyro.h): argument validation, error reporting
// and dispatch to the kernel launchers.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "pyro_internal.h"

namespace pyro {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }

int fail(int code, const std::string& msg) {
    g_error = msg;
    return code;
}

int hip_fail(hipError_t err, const char* what) {
    g_error = std::string(what) + ": " + hipGetErrorString(err);
    return PYRO_E_HIP;
}

namespace {

int check_mech(const pyro_mech* m) {
    if (!m) return fail(PYRO_E_ARG, "null mechanism handle");
    int dev = -1;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return hip_fail(err, "hipGetDevice");
    if (dev != m->device)
        return fail(PYRO_E_ARG, "mechanism was loaded on device " + std::to_string(m->device) +
                                    " but device " + std::to_string(dev) + " is current");
    return PYRO_OK;
}

int check_sizes(int64_t n, int64_t ld) {
    if (n < 0) return fail(PYRO_E_ARG, "n must be >= 0");
    if (ld < n) return fail(PYRO_E_ARG, "ld must be >= n");
    if (n > (int64_t(1) << 40)) return fail(PYRO_E_ARG, "n too large");
    return PYRO_OK;
}

int check_ptrs(std::initializer_list<const void*> ptrs, const char* what) {
    for (const void* p : ptrs)
        if (!p) return fail(PYRO_E_ARG, std::string("null pointer: ") + what);
    return PYRO_OK;
}

int launched(hipError_t err, const char* what) {
    if (err != hipSuccess) return hip_fail(err, what);
    return PYRO_OK;
}

}  // namespace
}  // namespace pyro

using namespace pyro;

extern "C" {

const char* pyro_last_error(void) { return g_error.c_str(); }

int pyro_mech_load(const char* path, pyro_mech** out) {
    clear_error();
    if (!path || !out) return fail(PYRO_E_ARG, "null argument to pyro_mech_load");
    *out = nullptr;
    return load_mechanism(path, out);
}

void pyro_mech_free(pyro_mech* mech) {
    if (!mech) return;
    if (mech->blob) (void)hipFree(mech->blob);
    delete mech;
}

int pyro_mech_get_info(const pyro_mech* m, pyro_mech_info* info) {
    clear_error();
    if (!m || !info) return fail(PYRO_E_ARG, "null argument to pyro_mech_get_info");
    info->n_species = m->S;
    info->n_reactions = m->R;
    info->n_elements = m->E;
    info->n_third_body = m->n_tb;
    info->n_falloff = m->n_fo;
    info->n_params = m->R + m->n_fo;
    info->nnz_reactant = m->nnz_f;
    info->nnz_product = m->nnz_r;
    info->nnz_net = m->nnz_net;
    info->wdot_variant = m->wdot_variant;
    return PYRO_OK;
}

int pyro_mech_set_wdot_variant(pyro_mech* m, int variant) {
    clear_error();
    if (!m) return fail(PYRO_E_ARG, "null mechanism handle");
    if (variant < 0 || variant > (PYRO_WDOT_REACTION_EQUILIBRIUM | PYRO_WDOT_MFMA_THIRD_BODY |
                                  PYRO_WDOT_MFMA_NET_RATES | PYRO_WDOT_LOG_SPACE |
                                  PYRO_WDOT_MFMA_LOG_PRODUCTS))
        return fail(PYRO_E_ARG, "unknown production-rate variant");
    if ((variant & PYRO_WDOT_MFMA_LOG_PRODUCTS) && !(variant & PYRO_WDOT_LOG_SPACE))
        return fail(PYRO_E_ARG, "PYRO_WDOT_MFMA_LOG_PRODUCTS is a flag of PYRO_WDOT_LOG_SPACE");
    if (variant & PYRO_WDOT_LOG_SPACE) {
        // the log-space form implies the reaction-equilibrium coefficients
        if (variant & (PYRO_WDOT_MFMA_THIRD_BODY | PYRO_WDOT_MFMA_NET_RATES))
            return fail(PYRO_E_UNSUPPORTED, "the log-space form has no third-body or net-rate "
                                            "matrix-core flags");
        if (!log_space_supported(m, 8))
            return fail(PYRO_E_UNSUPPORTED, m->kc_ok ? "mechanism too large for the log-space tile"
                                                     : "reactions mix species with different NASA7 T_mid");
        if ((variant & PYRO_WDOT_MFMA_LOG_PRODUCTS) && !log_products_supported(m))
            return fail(PYRO_E_UNSUPPORTED, "mechanism too large for the log-space tile with its "
                                            "log products on the matrix cores");
        m->wdot_variant = PYRO_WDOT_LOG_SPACE | PYRO_WDOT_REACTION_EQUILIBRIUM |
                          (variant & PYRO_WDOT_MFMA_LOG_PRODUCTS);
        return PYRO_OK;
    }
    const bool rkc = variant & PYRO_WDOT_REACTION_EQUILIBRIUM;
    const bool mm = variant & PYRO_WDOT_MFMA_THIRD_BODY;
    const bool nq = variant & PYRO_WDOT_MFMA_NET_RATES;
    if (rkc && !m->kc_ok)
        return fail(PYRO_E_UNSUPPORTED, "reactions mix species with different NASA7 T_mid");
    if (nq && !nq_supported(m))
        return fail(PYRO_E_UNSUPPORTED, "the matrix-core net rates need at most 64 species (192 "
                                        "with the 16-wavefront schedule of large mechanisms)");
    if (production_rates_lds_bytes(m, rkc, mm) > 160 * 1024)
        return fail(PYRO_E_UNSUPPORTED, rkc ? "mechanism too large for the LDS tile"
                                            : "species rows of this mechanism exceed the LDS tile");
    m->wdot_variant = variant;
    return PYRO_OK;
}

int pyro_mech_molecular_weights(const pyro_mech* m, double* W_out) {
    clear_error();
    if (!m || !W_out) return fail(PYRO_E_ARG, "null argument to pyro_mech_molecular_weights");
    for (int k = 0; k < m->S; ++k) W_out[k] = m->W[k];
    return PYRO_OK;
}

int pyro_mech_arrhenius(const pyro_mech* m, double* params_out) {
    clear_error();
    if (!m || !params_out) return fail(PYRO_E_ARG, "null argument to pyro_mech_arrhenius");
    for (size_t i = 0; i < m->params.size(); ++i) params_out[i] = m->params[i];
    return PYRO_OK;
}

int pyro_production_rates(const pyro_mech* m, int64_t n, int64_t ld, int dtype, const void* rho,
                          const void* T, const void* Y, void* wdot, const double* params,
                          void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (dtype != PYRO_F64 && dtype != PYRO_F32) return fail(PYRO_E_ARG, "unknown dtype");
    if (int rc = check_mech(m)) return rc;
    if (dtype == PYRO_F32 && !log_space_supported(m, 4))
        return fail(PYRO_E_UNSUPPORTED, "the FP32 (log-space) kernel cannot run this mechanism");
    if (n == 0) return PYRO_OK;
    if (int rc = check_ptrs({rho, T, Y, wdot}, "rho, T, Y and wdot")) return rc;
    return launched(launch_production_rates(m, n, ld, dtype, rho, T, Y, wdot, params,
                                            static_cast<hipStream_t>(stream)),
                    "production-rate kernel launch");
}

int pyro_production_rates_vjp(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                              const double* T, const double* Y, const double* wbar, double* Ybar,
                              double* Tbar, double* params_bar, double* wdot,
                              const double* params, void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (int rc = check_mech(m)) return rc;
    if (!params_bar) return fail(PYRO_E_ARG, "null pointer: params_bar");
    if (vjp_lds_bytes(m) > 160 * 1024)
        return fail(PYRO_E_UNSUPPORTED, "mechanism too large for the VJP tile");
    if (m->vjp_max_own > 16) return fail(PYRO_E_UNSUPPORTED, "too many species for the VJP kernel");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n == 0) {
        // no cells: every parameter gradient is zero
        return launched(hipMemsetAsync(params_bar, 0, size_t(m->R + m->n_fo) * 3 * sizeof(double), s),
                        "hipMemsetAsync");
    }
    if (int rc = check_ptrs({rho, T, Y, wbar, Ybar, Tbar}, "rho, T, Y, wbar, Ybar and Tbar")) return rc;
    return launched(launch_production_rates_vjp(m, n, ld, rho, T, Y, wbar, Ybar, Tbar, params_bar,
                                                wdot, params, s),
                    "VJP kernel launch");
}

int pyro_production_rates_vjp_noalloc(const pyro_mech* m, int64_t n, int64_t ld,
                                      const double* rho, const double* T, const double* Y,
                                      const double* wbar, double* Ybar, double* Tbar,
                                      double* params_bar, double* wdot, const double* params,
                                      void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (int rc = check_mech(m)) return rc;
    if (!params_bar) return fail(PYRO_E_ARG, "null pointer: params_bar");
    if (vjp_lds_bytes(m) > 160 * 1024)
        return fail(PYRO_E_UNSUPPORTED, "mechanism too large for the VJP tile");
    if (m->vjp_max_own > 16) return fail(PYRO_E_UNSUPPORTED, "too many species for the VJP kernel");
    const size_t need = size_t(vjp_scratch_blocks(m, std::max<int64_t>(n, 1))) * 3 *
                        size_t(m->R + m->n_fo);
    if (need > kVjpScratchDoubles)
        return fail(PYRO_E_UNSUPPORTED,
                    "the parameter partials (" + std::to_string(need) +
                        " doubles) exceed the fixed scratch of " +
                        std::to_string(kVjpScratchDoubles) + " doubles");
    if (n > 0)
        if (int rc = check_ptrs({rho, T, Y, wbar, Ybar, Tbar}, "rho, T, Y, wbar, Ybar and Tbar"))
            return rc;
    return launched(launch_production_rates_vjp_noalloc(m, n, ld, rho, T, Y, wbar, Ybar, Tbar,
                                                        params_bar, wdot, params,
                                                        static_cast<hipStream_t>(stream)),
                    "allocation-free VJP launch");
}

int pyro_chemical_jacobian(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                           const double* T, const double* Y, int fixed_energy, double* J,
                           double* dSdT, const double* params, void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (int rc = check_mech(m)) return rc;
    if (fixed_energy != 0 && fixed_energy != 1) return fail(PYRO_E_ARG, "fixed_energy must be 0 or 1");
    if (vjp_lds_bytes(m) > 160 * 1024)
        return fail(PYRO_E_UNSUPPORTED, "mechanism too large for the reverse-sweep tile");
    if (m->vjp_max_own > 16) return fail(PYRO_E_UNSUPPORTED, "too many species for the reverse sweep");
    if (n == 0) return PYRO_OK;
    if (int rc = check_ptrs({rho, T, Y, J}, "rho, T, Y and J")) return rc;
    return launched(launch_chemical_jacobian(m, n, ld, rho, T, Y, fixed_energy, J, dSdT, params,
                                             static_cast<hipStream_t>(stream)),
                    "Jacobian kernel launch");
}

int pyro_temperature(const pyro_mech* m, int64_t n, int64_t ld, const double* e, const double* Y,
                     const double* T_guess, double T_guess_value, double* T_out, int32_t* status,
                     int max_iter, double rtol, void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (max_iter < 1) return fail(PYRO_E_ARG, "max_iter must be >= 1");
    if (!(rtol >= 0)) return fail(PYRO_E_ARG, "rtol must be >= 0");
    if (!T_guess && !(std::isfinite(T_guess_value) && T_guess_value > 0))
        return fail(PYRO_E_ARG, "T_guess_value must be positive and finite");
    if (int rc = check_mech(m)) return rc;
    if (n == 0) return PYRO_OK;
    if (int rc = check_ptrs({e, Y, T_out, status}, "e, Y, T_out and status")) return rc;
    return launched(launch_temperature(m, n, ld, e, Y, T_guess, T_guess_value, T_out, status,
                                       max_iter, rtol, static_cast<hipStream_t>(stream)),
                    "Newton kernel launch");
}

int pyro_temperature_from_enthalpy(const pyro_mech* m, int64_t n, int64_t ld, const double* h,
                                   const double* Y, const double* T_guess, double T_guess_value,
                                   double* T_out, int32_t* status, int max_iter, double rtol,
                                   void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (max_iter < 1) return fail(PYRO_E_ARG, "max_iter must be >= 1");
    if (!(rtol >= 0)) return fail(PYRO_E_ARG, "rtol must be >= 0");
    if (!T_guess && !(std::isfinite(T_guess_value) && T_guess_value > 0))
        return fail(PYRO_E_ARG, "T_guess_value must be positive and finite");
    if (int rc = check_mech(m)) return rc;
    if (n == 0) return PYRO_OK;
    if (int rc = check_ptrs({h, Y, T_out, status}, "h, Y, T_out and status")) return rc;
    return launched(launch_temperature(m, n, ld, h, Y, T_guess, T_guess_value, T_out, status,
                                       max_iter, rtol, static_cast<hipStream_t>(stream), true),
                    "Newton kernel launch");
}

int pyro_primitive_from_conserved(const pyro_mech* m, int64_t n, int64_t ld, int dim,
                                  const double* partial_densities, const double* momentum,
                                  const double* total_energy, const double* T_guess,
                                  double T_guess_value, double* rho_out, double* Y_out,
                                  double* u_out, double* T_out, double* p_out, int32_t* status,
                                  int max_iter, double rtol, void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (dim < 0 || dim > 3) return fail(PYRO_E_ARG, "dim must be 0, 1, 2 or 3");
    if (max_iter < 1) return fail(PYRO_E_ARG, "max_iter must be >= 1");
    if (!(rtol >= 0)) return fail(PYRO_E_ARG, "rtol must be >= 0");
    if (!T_guess && !(std::isfinite(T_guess_value) && T_guess_value > 0))
        return fail(PYRO_E_ARG, "T_guess_value must be positive and finite");
    if (int rc = check_mech(m)) return rc;
    if (n == 0) return PYRO_OK;
    if (int rc = check_ptrs({partial_densities, total_energy, rho_out, Y_out, T_out, p_out, status},
                            "partial_densities, total_energy, rho_out, Y_out, T_out, p_out and "
                            "status"))
        return rc;
    if (dim > 0)
        if (int rc = check_ptrs({momentum, u_out}, "momentum and u_out")) return rc;
    return launched(launch_primitive(m, n, ld, dim, partial_densities, momentum, total_energy,
                                     T_guess, T_guess_value, rho_out, Y_out, u_out, T_out, p_out,
                                     status, max_iter, rtol, static_cast<hipStream_t>(stream)),
                    "primitive kernel launch");
}

int pyro_transport_create(const pyro_mech* m, const double* visc, const double* cond,
                          const double* diff, pyro_transport** out) {
    clear_error();
    if (!out) return fail(PYRO_E_ARG, "null argument to pyro_transport_create");
    *out = nullptr;
    if (int rc = check_mech(m)) return rc;
    if (!visc || !cond || !diff) return fail(PYRO_E_ARG, "null fit coefficients");
    const int S = m->S;
    for (size_t q = 0; q < size_t(S) * 5; ++q)
        if (!std::isfinite(visc[q]) || !std::isfinite(cond[q]))
            return fail(PYRO_E_ARG, "non-finite viscosity or conductivity coefficient");
    for (size_t q = 0; q < size_t(S) * S * 5; ++q)
        if (!std::isfinite(diff[q])) return fail(PYRO_E_ARG, "non-finite diffusivity coefficient");
    // one allocation: 1/W [S], visc [S][5], cond [S][5], pairs [S][S][8]
    std::vector<double> host(size_t(S) * 11 + size_t(S) * S * 8, 0.0);
    double* inv_w = host.data();
    double* hv = inv_w + S;
    double* hc = hv + size_t(S) * 5;
    double* hp = hc + size_t(S) * 5;
    for (int k = 0; k < S; ++k) {
        inv_w[k] = 1.0 / m->W[k];
        for (int q = 0; q < 5; ++q) {
            hv[k * 5 + q] = visc[k * 5 + q];
            hc[k * 5 + q] = cond[k * 5 + q];
        }
    }
    for (int j = 0; j < S; ++j)
        for (int k = 0; k < S; ++k) {
            double* r = hp + (size_t(j) * S + k) * 8;
            r[0] = std::pow(m->W[j] / m->W[k], 0.25);               // w_kj
            r[1] = 1.0 / std::sqrt(8.0 * (1.0 + m->W[k] / m->W[j]));  // v_kj
            for (int q = 0; q < 5; ++q) r[2 + q] = diff[(size_t(k) * S + j) * 5 + q];
        }
    auto* t = new pyro_transport;
    t->device = m->device;
    t->S = S;
    hipError_t e = hipMalloc(&t->blob, host.size() * sizeof(double));
    if (e != hipSuccess) {
        delete t;
        return fail(PYRO_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    e = hipMemcpy(t->blob, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(t->blob);
        delete t;
        return hip_fail(e, "hipMemcpy");
    }
    const double* b = static_cast<const double*>(t->blob);
    t->tt = TransportTables{b, b + S, b + S + size_t(S) * 5, b + S + size_t(S) * 10};
    *out = t;
    return PYRO_OK;
}

void pyro_transport_free(pyro_transport* t) {
    if (!t) return;
    if (t->blob) hipFree(t->blob);
    delete t;
}

int pyro_mixture_transport(const pyro_mech* m, const pyro_transport* t, int64_t n, int64_t ld,
                           const double* T, const double* Y, double* mu, double* kappa,
                           double* D, void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (int rc = check_mech(m)) return rc;
    if (!t || t->S != m->S || t->device != m->device)
        return fail(PYRO_E_ARG, "transport tables missing or made for another mechanism/device");
    if (n == 0) return PYRO_OK;
    if (int rc = check_ptrs({T, Y, mu, kappa, D}, "T, Y, mu, kappa and D")) return rc;
    return launched(launch_transport(m, t->tt, n, ld, T, Y, mu, kappa, D,
                                     static_cast<hipStream_t>(stream)),
                    "transport kernel launch");
}

size_t pyro_reactor_workspace_size(const pyro_mech* m, int64_t n, int64_t ld, int method) {
    if (!m || n < 0 || ld < n || (method != PYRO_REACTOR_RK4 && method != PYRO_REACTOR_CN))
        return 0;
    return reactor_workspace_bytes(m, n, ld, method);
}

int pyro_reactor_step(const pyro_mech* m, int method, int64_t n, int64_t ld, const double* rho,
                      const double* e, double* Y, double* T, const double* dt, double dt_value,
                      double tol, int max_newton, int32_t* status, void* workspace,
                      size_t workspace_bytes, void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (method != PYRO_REACTOR_RK4 && method != PYRO_REACTOR_CN)
        return fail(PYRO_E_ARG, "unknown reactor method");
    if (int rc = check_mech(m)) return rc;
    if (method == PYRO_REACTOR_CN) {
        if (max_newton < 1) return fail(PYRO_E_ARG, "max_newton must be >= 1");
        if (!(tol >= 0)) return fail(PYRO_E_ARG, "tol must be >= 0");
        if (vjp_lds_bytes(m) > 160 * 1024 || m->vjp_max_own > 16)
            return fail(PYRO_E_UNSUPPORTED, "the Jacobian of this mechanism is not supported");
    }
    if (!dt && !std::isfinite(dt_value)) return fail(PYRO_E_ARG, "dt_value must be finite");
    if (n == 0) return PYRO_OK;
    if (int rc = check_ptrs({rho, e, Y, T, status, workspace}, "rho, e, Y, T, status and workspace"))
        return rc;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
        return fail(PYRO_E_ARG, "workspace must be 256-byte aligned");
    if (workspace_bytes < reactor_workspace_bytes(m, n, ld, method))
        return fail(PYRO_E_ARG, "workspace too small (see pyro_reactor_workspace_size)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (method == PYRO_REACTOR_RK4)
        return launched(launch_rk4_step(m, n, ld, rho, e, Y, T, dt, dt_value, status, workspace, s),
                        "Runge-Kutta step");
    return launched(launch_cn_step(m, n, ld, rho, e, Y, T, dt, dt_value, tol, max_newton, status,
                                   workspace, s),
                    "Crank-Nicolson step");
}

int pyro_density(const pyro_mech* m, int64_t n, int64_t ld, const double* p, const double* T,
                 const double* Y, double* rho_out, void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (int rc = check_mech(m)) return rc;
    if (n == 0) return PYRO_OK;
    if (int rc = check_ptrs({p, T, Y, rho_out}, "p, T, Y and rho_out")) return rc;
    return launched(launch_eos(m, n, ld, 0, p, T, Y, rho_out, static_cast<hipStream_t>(stream)),
                    "EOS kernel launch");
}

int pyro_pressure(const pyro_mech* m, int64_t n, int64_t ld, const double* rho, const double* T,
                  const double* Y, double* p_out, void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (int rc = check_mech(m)) return rc;
    if (n == 0) return PYRO_OK;
    if (int rc = check_ptrs({rho, T, Y, p_out}, "rho, T, Y and p_out")) return rc;
    return launched(launch_eos(m, n, ld, 1, rho, T, Y, p_out, static_cast<hipStream_t>(stream)),
                    "EOS kernel launch");
}

int pyro_internal_energy(const pyro_mech* m, int64_t n, int64_t ld, const double* T,
                         const double* Y, double* e_out, void* stream) {
    clear_error();
    if (int rc = check_sizes(n, ld)) return rc;
    if (int rc = check_mech(m)) return rc;
    if (n == 0) return PYRO_OK;
    if (int rc = check_ptrs({T, Y, e_out}, "T, Y and e_out")) return rc;
    return launched(launch_internal_energy(m, n, ld, T, Y, e_out, static_cast<hipStream_t>(stream)),
                    "energy kernel launch");
}

}  // extern "C"
