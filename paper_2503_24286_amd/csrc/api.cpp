// C ABI of libpyro (include/pyro.h): argument validation, error reporting
// and dispatch to the kernel launchers.
#include <cmath>
#include <string>

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
                                  PYRO_WDOT_MFMA_NET_RATES))
        return fail(PYRO_E_ARG, "unknown production-rate variant");
    const bool rkc = variant & PYRO_WDOT_REACTION_EQUILIBRIUM;
    const bool mm = variant & PYRO_WDOT_MFMA_THIRD_BODY;
    const bool nq = variant & PYRO_WDOT_MFMA_NET_RATES;
    if (rkc && !m->kc_ok)
        return fail(PYRO_E_UNSUPPORTED, "reactions mix species with different NASA7 T_mid");
    if (nq && !nq_supported(m))
        return fail(PYRO_E_UNSUPPORTED, "the matrix-core net rates need at most 64 species");
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
    if (dtype == PYRO_F32) return fail(PYRO_E_UNSUPPORTED, "PYRO_F32 is not built yet");
    if (int rc = check_mech(m)) return rc;
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
