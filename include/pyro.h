/*
 * pyro.h - C ABI of libpyro, per-cell ideal-gas thermochemistry on AMD
 * Instinct MI355X (gfx950).
 *
 * The library evaluates the kinetics and thermodynamics formulation of
 * Appendix A of "Pyrometheus: Symbolic abstractions for XPU and automatically
 * differentiated computation of combustion kinetics and thermodynamics"
 * (arXiv:2503.24286) for many independent cells at once.
 *
 * Conventions shared by every call
 * --------------------------------
 * Units are SI on a mole basis: T in K, p in Pa, rho in kg/m^3, molar masses
 * in kg/mol, concentrations in mol/m^3, production rates in mol m^-3 s^-1,
 * activation energies in J/mol, internal energy in J/kg.
 *
 * Cell arrays are device pointers in structure-of-arrays layout.  Per-cell
 * scalars (rho, T, p, e, ...) hold n contiguous values.  Per-species arrays
 * (Y, wdot, ...) are species-major: the value of species k in cell i sits at
 * index k*ld + i, with ld >= n (the paper's (N_s, nx, ny) layout, Sec. 4.1).
 * The caller owns every cell array; the library never allocates or frees
 * them.  Output arrays are overwritten for cells 0..n-1 only.
 *
 * Calls are asynchronous on the given HIP stream (a hipStream_t passed as
 * void*; NULL means the default stream).  A return value of PYRO_OK means the
 * arguments were valid and the work was enqueued; numerical trouble in a
 * cell is not an error (NaN/Inf propagate; the Newton call reports per-cell
 * status).  On any other return nothing was enqueued and pyro_last_error()
 * describes the problem.  n == 0 is a valid no-op.
 *
 * A mechanism handle belongs to the device that was current when it was
 * loaded; calls must be made with that device current.  Handles may be used
 * from several threads at once; calls on one stream are ordered as usual.
 */
#ifndef PYRO_H
#define PYRO_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define PYRO_API __attribute__((visibility("default")))
#else
#define PYRO_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum pyro_status {
    PYRO_OK = 0,
    PYRO_E_ARG = -1,          /* invalid argument (null pointer, ld < n, ...) */
    PYRO_E_IO = -2,           /* the mechanism file cannot be read           */
    PYRO_E_FORMAT = -3,       /* malformed or inconsistent mechanism file    */
    PYRO_E_HIP = -4,          /* a HIP runtime call failed (no device, ...)  */
    PYRO_E_NOMEM = -5,        /* device or host allocation failed            */
    PYRO_E_UNSUPPORTED = -6   /* valid input outside what the kernels handle */
};

enum pyro_dtype {
    PYRO_F64 = 0,             /* double cell arrays, double arithmetic       */
    PYRO_F32 = 1              /* float cell arrays, float arithmetic         */
};

/* How the production-rate kernel forms the equilibrium constants
 * (eq. equil_constants): both compute the same quantity. */
enum pyro_wdot_variant {
    /* per species G_k = exp(g0_k/RT) in LDS, 1/K_c as products of G: S
     * exponentials per cell, 1 KB of LDS per species for a 64-cell tile */
    PYRO_WDOT_SPECIES_EQUILIBRIUM = 0,
    /* per reaction exp(sum_k nu_kj g0_k/RT) from coefficients combined at
     * load time: one exponential per reversible reaction, 512 B of LDS per
     * species; needs every reaction's species to share one NASA7 T_mid */
    PYRO_WDOT_REACTION_EQUILIBRIUM = 1,
    /* flag, combinable with either: the third-body concentrations
     * [M]_j = sum_k eps_jk C_k (a dense contraction) of a 64-cell tile on the
     * FP64 matrix cores (v_mfma_f64_16x16x4f64) instead of per-wave FMA
     * passes; [M] is then held in LDS (512 B per third-body reaction) */
    PYRO_WDOT_MFMA_THIRD_BODY = 2,
    /* flag, combinable with the others: the net production rates
     * omega = nu q (eq. production_rates) of a 64-cell tile accumulated on
     * the FP64 matrix cores over the reaction chunks with the dense nu
     * (v_mfma_f64_16x16x4f64), instead of the sparse per-species gathering;
     * at most 64 species, or 192 for mechanisms large enough to run the
     * 16-wavefront schedule */
    PYRO_WDOT_MFMA_NET_RATES = 4,
    /* log-space form (implies the reaction-equilibrium coefficients, no
     * matrix-core flags): each rate is one exponential of a sum of logarithms,
     * R_f = exp(ln k + sum_k nu'_kj ln C_k) and R_r = exp(ln k + dg_j +
     * dnu_j ln(R T/p0) + sum_k nu''_kj ln C_k) (ln [M] added for third-body
     * reactions, ln(P_r/(1+P_r)) + ln F for falloff), so no intermediate
     * overflows before the rate itself; LDS rows hold C and ln C.  Every
     * PYRO_F32 call uses this form. */
    PYRO_WDOT_LOG_SPACE = 8,
    /* flag of PYRO_WDOT_LOG_SPACE only (FP64): the stoichiometric log sums
     * sum_k nu'_kj ln C_k and sum_k nu''_kj ln C_k of a chunk of reactions
     * over the 64-cell tile as dense products ln C [cells x S] nu [S x slots]
     * on the FP64 matrix cores (v_mfma_f64_16x16x4f64), ln 0 floored at
     * -1e30, instead of the per-reaction sums of LDS reads; reads back as
     * PYRO_WDOT_LOG_SPACE | PYRO_WDOT_REACTION_EQUILIBRIUM |
     * PYRO_WDOT_MFMA_LOG_PRODUCTS */
    PYRO_WDOT_MFMA_LOG_PRODUCTS = 16
};

typedef struct pyro_mech pyro_mech;

typedef struct pyro_mech_info {
    int32_t n_species;        /* S                                           */
    int32_t n_reactions;      /* R                                           */
    int32_t n_elements;       /* E                                           */
    int32_t n_third_body;     /* plain third-body reactions                  */
    int32_t n_falloff;        /* Lindemann and Troe falloff reactions        */
    int32_t n_params;         /* R + n_falloff Arrhenius triples             */
    int32_t nnz_reactant;     /* nonzero nu'_kj (species, reaction) pairs     */
    int32_t nnz_product;      /* nonzero nu''_kj pairs                       */
    int32_t nnz_net;          /* nonzero nu_kj = nu''_kj - nu'_kj pairs      */
    int32_t wdot_variant;     /* current enum pyro_wdot_variant              */
} pyro_mech_info;

/* Message of the last failed call on this thread ("" if none).  The string
 * stays valid until the next libpyro call on the same thread. */
PYRO_API const char* pyro_last_error(void);

/*
 * Mechanism handling
 * ------------------
 * pyro_mech_load parses a .pyromech version-1 file (header, species,
 * NASA7 thermodynamics, reactions with integer stoichiometry, Arrhenius,
 * falloff, Troe and third-body data; see the file-format description in the
 * library sources) and uploads the tables the kernels read to the current
 * device.  It rejects a truncated or corrupted file (checksum), an unknown
 * version, non-finite parameters, out-of-range indices and inconsistent
 * counts (PYRO_E_FORMAT), and mechanisms beyond the kernels' limits, such as
 * more than three molecules on one side of a reaction (PYRO_E_UNSUPPORTED).
 * On success *out owns host and device memory until pyro_mech_free.
 */
PYRO_API int pyro_mech_load(const char* path, pyro_mech** out);
PYRO_API void pyro_mech_free(pyro_mech* mech);
PYRO_API int pyro_mech_get_info(const pyro_mech* mech, pyro_mech_info* info);
/* Selects the production-rate kernel variant (enum pyro_wdot_variant, an
 * equilibrium variant optionally or-ed with PYRO_WDOT_MFMA_THIRD_BODY and
 * PYRO_WDOT_MFMA_NET_RATES, or PYRO_WDOT_LOG_SPACE optionally or-ed with
 * PYRO_WDOT_MFMA_LOG_PRODUCTS, which reads back with
 * PYRO_WDOT_REACTION_EQUILIBRIUM added) used by FP64
 * pyro_production_rates calls and the surrogate's fallback.  The loader picks the
 * species variant when its LDS tile fits and the reaction variant otherwise;
 * PYRO_E_UNSUPPORTED if the requested variant cannot run this mechanism.
 * Not thread-safe against concurrent calls on the same handle. */
PYRO_API int pyro_mech_set_wdot_variant(pyro_mech* mech, int variant);
/* Copies the S molar masses (kg/mol) into host memory W_out[S]. */
PYRO_API int pyro_mech_molecular_weights(const pyro_mech* mech, double* W_out);
/* Copies the default Arrhenius triples (ln A, b, Ea) into host memory
 * params_out[3*n_params]: rows 0..R-1 are the reactions' own (high-pressure
 * for falloff) triples, rows R.. the falloff low-pressure triples. */
PYRO_API int pyro_mech_arrhenius(const pyro_mech* mech, double* params_out);

/*
 * Net production rates (Appendix A.1: eq. concentrations, eq. nasa_poly,
 * eq. gibbs, eq. rate_coeff, eq. equil_constants, eq. reaction_rates,
 * eq. production_rates; third-body and Lindemann/Troe falloff forms for the
 * rate coefficients the paper names but does not write).
 *
 *   rho[n], T[n]   density and temperature
 *   Y[S*ld]        mass fractions (negative values count as zero; the sum is
 *                  not required to be one)
 *   wdot[S*ld]     output omega_k
 *   params         device array of 3*n_params doubles (ln A, b, Ea) that
 *                  replaces the mechanism's Arrhenius triples, or NULL
 *   dtype          PYRO_F64: rho, T, Y, wdot are double, computed with the
 *                  mechanism's current variant.  PYRO_F32: they are float and
 *                  the arithmetic is float, always in the log-space form
 *                  (params stay double and are rounded to float); a rate
 *                  beyond the float range gives an infinite or NaN omega
 *                  (counted by the caller), a smaller one never overflows.
 *                  PYRO_E_UNSUPPORTED where the log-space form cannot run.
 */
PYRO_API int pyro_production_rates(const pyro_mech* mech, int64_t n, int64_t ld,
                          int dtype, const void* rho, const void* T,
                          const void* Y, void* wdot, const double* params,
                          void* stream);

/*
 * Reverse-mode product of the net production rates.  With
 * L = sum_cells sum_k wbar_k(cell) omega_k(cell) at fixed density, returns
 * the per-cell gradients dL/dY and dL/dT and the gradients with respect to
 * every Arrhenius triple summed over the cells (reverse sweep of the
 * equations named for pyro_production_rates; third-body efficiencies and
 * Troe shape parameters get no gradient).
 *
 *   rho[n], T[n], Y[S*ld]  the state (as for pyro_production_rates)
 *   wbar[S*ld]             dL/d omega
 *   Ybar[S*ld]             output dL/dY (zero where Y_k <= 0)
 *   Tbar[n]                output dL/dT
 *   params_bar             device array of 3*n_params doubles, overwritten
 *                          with dL/d(ln A, b, Ea) in the row order of params
 *                          (Ea per J/mol); deterministic (fixed-order sums)
 *   wdot[S*ld]             optional output (NULL to skip): the net production
 *                          rates of the same state, from the forward
 *                          recomputation the reverse sweep performs anyway
 *                          (equal to pyro_production_rates up to rounding order)
 *   params                 Arrhenius triples to differentiate at, or NULL
 * The call allocates a temporary workspace on the stream (stream-ordered).
 * FP64 only.  PYRO_E_UNSUPPORTED for mechanisms whose tables exceed the
 * kernel's LDS tile or with more than 16 species per wavefront.
 */
PYRO_API int pyro_production_rates_vjp(const pyro_mech* mech, int64_t n, int64_t ld,
                                       const double* rho, const double* T,
                                       const double* Y, const double* wbar,
                                       double* Ybar, double* Tbar, double* params_bar,
                                       double* wdot, const double* params, void* stream);

/*
 * pyro_production_rates_vjp without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results (bitwise) and
 * errors as pyro_production_rates_vjp, except: the per-workgroup parameter
 * partials live in a fixed device array of 2^19 doubles (4 MiB) that each
 * device holds from the first mechanism load on it until the process ends,
 * so the call returns PYRO_E_UNSUPPORTED when min(ceil(n/64), compute
 * units) x 3 (R + n_falloff) exceeds 2^19 (about 680 Arrhenius triples on a
 * 256-CU device), and it makes no hipMalloc, hipFree or memset (n == 0 zeroes
 * params_bar with a kernel).  Every call on one device shares that array:
 * calls that overlap in time on one device (other streams, other threads)
 * race and give wrong parameter gradients; calls on one stream are ordered.
 */
PYRO_API int pyro_production_rates_vjp_noalloc(const pyro_mech* mech, int64_t n, int64_t ld,
                                               const double* rho, const double* T,
                                               const double* Y, const double* wbar,
                                               double* Ybar, double* Tbar, double* params_bar,
                                               double* wdot, const double* params,
                                               void* stream);

/*
 * Chemical Jacobian J = dS/dY of the source terms S_j = W_j omega_j
 * (eq. jacobian and eq. chem_jacobian, Sec. "Automatic Differentiation
 * Enables Implicit Time Marching"; eq. massfrac_ode defines S), per cell, at
 * fixed density.
 *
 *   rho[n], T[n], Y[S*ld]  the state (as for pyro_production_rates); with
 *                  fixed_energy = 1, T must be the temperature of the state's
 *                  internal energy (as pyro_temperature returns it)
 *   fixed_energy   1: T follows Y at fixed internal energy (the paper's
 *                  source-term function, whose temperature comes from the
 *                  Newton inversion of eq. delta_temp), so that
 *                  J_jk = dS_j/dY_k|_T - dS_j/dT e_k/c_v with
 *                  e_k = (h_k - R T)/W_k and c_v = sum_i Y_i c_v,i;
 *                  0: the partial derivative at fixed T
 *   J[S*S*ld]      output, J[(j*S + k)*ld + i] = dS_j/dY_k of cell i (rows of
 *                  S*ld doubles, each species-major like Y); the entries of a
 *                  column k with Y_k <= 0 have no concentration part
 *   dSdT           optional output [S*ld], dS_j/dT at fixed Y, or NULL
 *   params         Arrhenius triples as for pyro_production_rates, or NULL
 * Asynchronous; S reverse sweeps with a unit cotangent per row (the
 * reactions without the row's species are skipped).  FP64 only.
 * PYRO_E_UNSUPPORTED for mechanisms the reverse sweep cannot run.
 */
PYRO_API int pyro_chemical_jacobian(const pyro_mech* mech, int64_t n, int64_t ld,
                                    const double* rho, const double* T, const double* Y,
                                    int fixed_energy, double* J, double* dSdT,
                                    const double* params, void* stream);

/*
 * Temperature from the mass-specific internal energy by Newton iteration
 * (Appendix A.3.1: eq. int_energy, eq. delta_temp, eq. cv):
 * T <- T - (Y.e(T) - e)/c_v(T), per cell, until the first update with
 * |dT| <= rtol*|T| or max_iter updates.
 *
 *   e[n]           internal energy (J/kg)
 *   Y[S*ld]        mass fractions (used as given)
 *   T_guess        device array of n initial guesses, or NULL to start every
 *                  cell from T_guess_value
 *   T_out[n]       result
 *   status[n]      number of updates taken, negated when rtol was not met
 *   max_iter       >= 1; rtol >= 0
 */
PYRO_API int pyro_temperature(const pyro_mech* mech, int64_t n, int64_t ld,
                     const double* e, const double* Y, const double* T_guess,
                     double T_guess_value, double* T_out, int32_t* status,
                     int max_iter, double rtol, void* stream);

/* Temperature from the mass-specific enthalpy h = sum_k Y_k h_k/W_k (J/kg)
 * by the same Newton iteration with c_p in place of c_v (the enthalpy
 * variant named at the end of Appendix A.3.1): T <- T - (Y.h(T) - h)/c_p(T).
 * Arguments, status and errors as for pyro_temperature. */
PYRO_API int pyro_temperature_from_enthalpy(const pyro_mech* mech, int64_t n, int64_t ld,
                                            const double* h, const double* Y,
                                            const double* T_guess, double T_guess_value,
                                            double* T_out, int32_t* status, int max_iter,
                                            double rtol, void* stream);

/*
 * Primitive from conserved variables, the per-cell equation-of-state routine
 * of the paper's flow solver (Sec. "Python Code Generation and Immediate
 * Execution using NumPy", in its order; eq. delta_temp and eq. eos):
 * rho = sum_k rho_k, Y_k = rho_k/rho, u = m/rho, e = E/rho - |u|^2/2,
 * T = Newton inversion of e (as pyro_temperature), p = rho R T/W.
 *
 *   dim                    0..3 velocity components
 *   partial_densities[S*ld] rho_k (kg/m^3), species-major
 *   momentum[dim*ld]       rho u_d, component-major (ignored if dim == 0)
 *   total_energy[n]        E = rho (e + |u|^2/2) (J/m^3)
 *   T_guess, T_guess_value, max_iter, rtol, status: as for pyro_temperature
 *   rho_out[n], Y_out[S*ld], u_out[dim*ld], T_out[n], p_out[n]: outputs
 * A cell with rho = 0 gives NaN/Inf results (no error).
 */
PYRO_API int pyro_primitive_from_conserved(const pyro_mech* mech, int64_t n, int64_t ld,
                                           int dim, const double* partial_densities,
                                           const double* momentum, const double* total_energy,
                                           const double* T_guess, double T_guess_value,
                                           double* rho_out, double* Y_out, double* u_out,
                                           double* T_out, double* p_out, int32_t* status,
                                           int max_iter, double rtol, void* stream);

/*
 * Mixture-averaged transport (appendix "Extensions to Flow & Transport":
 * eq. mixavg_viscosity, eq. mixavg_conductivity, eq. species_cond,
 * eq. diff_mix_rule and the binary-diffusivity fit).  With L = ln T (natural
 * logarithm) and X_k = W Y_k/W_k (W the mixture molar mass of the Y given,
 * not renormalised):
 *   mu_k = sqrt(T) (sum_m b_km L^m)^2, kappa_k = sqrt(T) sum_m c_km L^m,
 *   D_kj = sqrt(T) sum_m a_kjm L^m (no pressure factor),
 *   mu = sum_k X_k mu_k / sum_j Phi_kj X_j with
 *        Phi_kj = (1 + sqrt((mu_k/mu_j) sqrt(W_j/W_k)))^2 / sqrt(8 (1 + W_k/W_j)),
 *   kappa = (sum_k X_k kappa_k + (sum_k X_k/kappa_k)^-1)/2,
 *   D_k,m = (W - X_k W_k)/W (sum_{j != k} X_j/D_kj)^-1  (NaN/Inf for a pure
 *        species, left to IEEE arithmetic).
 *
 * pyro_transport_create copies host fits, visc[S][5] (b_km), cond[S][5]
 * (c_km) and diff[S][S][5] (a_kjm, index k first), into device tables of the
 * mechanism's device, with the per-pair constants of Phi formed once; *out
 * owns them until pyro_transport_free.  PYRO_E_ARG for non-finite
 * coefficients.  pyro_mixture_transport takes T[n], Y[S*ld] (device) and
 * writes mu[n] (Pa s), kappa[n] (W/(m K)) and D[S*ld] (m^2/s).
 */
typedef struct pyro_transport pyro_transport;
PYRO_API int pyro_transport_create(const pyro_mech* mech, const double* visc,
                                   const double* cond, const double* diff,
                                   pyro_transport** out);
PYRO_API void pyro_transport_free(pyro_transport* tr);
PYRO_API int pyro_mixture_transport(const pyro_mech* mech, const pyro_transport* tr, int64_t n,
                                    int64_t ld, const double* T, const double* Y, double* mu,
                                    double* kappa, double* D, void* stream);

/*
 * One time step of the homogeneous adiabatic isochoric reactor,
 * rho dY_k/dt = W_k omega_k (eq. massfrac_ode), at constant density and
 * internal energy; every evaluation takes T from the Newton inversion of the
 * energy (eq. delta_temp, rtol 1e-12, at most 50 updates).
 *
 *   PYRO_REACTOR_RK4  classical four-stage Runge-Kutta (the paper's explicit
 *                     autoignition marching);
 *   PYRO_REACTOR_CN   Crank-Nicolson, F = Y - Y^m - dt/(2 rho) (S + S^m) = 0
 *                     (eq. crank_nicol_rhs with the density of eq. massfrac_ode)
 *                     solved by Newton with the matrix I - dt/(2 rho) J
 *                     (eq. crank_nicol_jac; J = dS/dY at fixed density and
 *                     energy, as pyro_chemical_jacobian) from Y^m, per cell
 *                     until the first update with every |dY_k| <= tol (an
 *                     update holding a NaN never qualifies) or max_newton
 *                     updates; each update solves the S x S system of every
 *                     cell still iterating with partial pivoting
 *                     (Gauss-Jordan, one cell per wavefront, up to 64
 *                     species; Gaussian elimination past that).  The call
 *                     waits on the stream after each update to stop once
 *                     every cell has converged.
 *
 *   rho[n], e[n]      density and internal energy (constant over the step)
 *   Y[S*ld]           in: Y^m; out: the new mass fractions
 *   T[n]              in: guess for the first inversion; out: T of the new Y
 *   dt                device [n] step per cell, or NULL to use dt_value
 *   status[n]         out: RK4, the final inversion's count (0 if an inversion
 *                     failed on the way); CN, the Newton updates taken,
 *                     negated if tol was not met
 *   workspace         device, 256-byte aligned, at least
 *                     pyro_reactor_workspace_size(mech, n, ld, method) bytes
 *                     (CN holds one S x S matrix per cell)
 */
enum pyro_reactor_method { PYRO_REACTOR_RK4 = 0, PYRO_REACTOR_CN = 1 };
PYRO_API size_t pyro_reactor_workspace_size(const pyro_mech* mech, int64_t n, int64_t ld,
                                            int method);
PYRO_API int pyro_reactor_step(const pyro_mech* mech, int method, int64_t n, int64_t ld,
                               const double* rho, const double* e, double* Y, double* T,
                               const double* dt, double dt_value, double tol, int max_newton,
                               int32_t* status, void* workspace, size_t workspace_bytes,
                               void* stream);

/* Equation of state (Appendix A.1, eq. eos): rho = p W/(R T) and
 * p = rho R T/W with W = (sum_k Y_k/W_k)^-1.  FP64 cell arrays. */
PYRO_API int pyro_density(const pyro_mech* mech, int64_t n, int64_t ld, const double* p,
                 const double* T, const double* Y, double* rho_out, void* stream);
PYRO_API int pyro_pressure(const pyro_mech* mech, int64_t n, int64_t ld,
                  const double* rho, const double* T, const double* Y,
                  double* p_out, void* stream);

/* Mixture internal energy e = sum_k Y_k (h_k - R T)/W_k in J/kg
 * (Appendix A.3.1, eq. int_energy).  FP64 cell arrays. */
PYRO_API int pyro_internal_energy(const pyro_mech* mech, int64_t n, int64_t ld,
                         const double* T, const double* Y, double* e_out,
                         void* stream);

/*
 * Learned surrogate of the net production rates
 * ----------------------------------------------
 * Not part of the paper's method: an MLP that maps per-cell features to
 * omega, trained on states the exact kernel labels, with per-cell fallback
 * to the exact kernel where its error indicators trip.  BF16 weights and
 * activations, FP32 accumulation (v_mfma_f32_32x32x16_bf16).  BF16 values
 * are passed as raw 16-bit patterns (uint16_t).
 *
 * Network: 64 -> H -> H -> H -> 64 (SiLU after the three hidden layers).
 * Features (row of 64 per cell, see pyro_surrogate_features): T/1000,
 * log10 p, ln(max(Y_k, 0) + 1e-12) for the S species, shifted and scaled,
 * then a constant 1 and zeros.  Outputs: z_k = (asinh(omega_k/s_k) - mu_k)
 * / sigma_k in the first S columns.  One member's parameters are packed:
 * weights W1 [64][H], W2 [H][H], W3 [H][H], W4 [H][64] (row-major, input
 * index first), biases b1 [H], b2 [H], b3 [H], b4 [64].
 */
typedef struct pyro_surrogate {
    int32_t n_members;            /* ensemble size E, 1..4                    */
    int32_t hidden;               /* H, a multiple of 64                      */
    const uint16_t* weights;      /* device, E packed weight sets (BF16)      */
    const float* biases;          /* device, E packed bias sets               */
    const float* feat_shift;      /* device [64]                              */
    const float* feat_scale;      /* device [64]                              */
    const double* target_scale;   /* device [S]: s_k                          */
    const double* target_mean;    /* device [S]: mu_k                         */
    const double* target_std;     /* device [S]: sigma_k                      */
} pyro_surrogate;

/* Number of packed weights and biases of one member; returns the weights
 * count, 0 for an invalid hidden width. */
PYRO_API size_t pyro_mlp_param_counts(int hidden, int64_t* n_weights, int64_t* n_biases);

/* Forward pass of one member on a batch: X [batch][64] BF16 features,
 * acts a BF16 buffer of 6*batch*H receiving (pre-activation, activation) of
 * the three hidden layers, Z [batch][64] FP32 outputs. */
PYRO_API int pyro_mlp_forward(int hidden, int64_t batch, const uint16_t* X,
                              const uint16_t* W, const float* b, uint16_t* acts,
                              float* Z, void* stream);

/* Backward pass from dZ [batch][64] (BF16): gW and gb (FP32, packed like
 * the parameters) receive dLoss/dW and dLoss/db, summed over the batch in a
 * fixed order.  work: BF16 buffer of 2*batch*H; split_work: FP32 buffer of
 * splits*H*H (the batch is split into `splits` ranges for the weight
 * gradients). */
PYRO_API int pyro_mlp_backward(int hidden, int64_t batch, const uint16_t* X,
                               const uint16_t* W, const uint16_t* acts,
                               const uint16_t* dZ, float* gW, float* gb,
                               uint16_t* work, float* split_work, int splits,
                               void* stream);

/* Mean squared error over the first n_out of 64 output columns:
 * dZ = 2 (Z - Zt)/(batch n_out) (BF16) and per-block partial sums of the
 * squared errors in loss_partials[pyro_mlp_loss_partials(batch)]. */
PYRO_API int64_t pyro_mlp_loss_partials(int64_t batch);
PYRO_API int pyro_mlp_mse(int64_t batch, int n_out, const float* Z, const float* Zt,
                          uint16_t* dZ, float* loss_partials, void* stream);

/* AdamW with decoupled weight decay on FP32 master weights w (step >= 1);
 * w_bf16, if not NULL, receives the rounded copy. */
PYRO_API int pyro_adamw_step(int64_t n, float* w, uint16_t* w_bf16, const float* grad,
                             float* m1, float* m2, float lr, float beta1, float beta2,
                             float eps, float weight_decay, int step, void* stream);
PYRO_API int pyro_to_bf16(int64_t n, const float* x, uint16_t* y, void* stream);

/* Features X [n][64] (BF16) of the cells (rho, T, Y as for
 * pyro_production_rates); shift and scale are device [64] FP32. */
PYRO_API int pyro_surrogate_features(const pyro_mech* mech, int64_t n, int64_t ld,
                                     const double* rho, const double* T, const double* Y,
                                     const float* shift, const float* scale, uint16_t* X,
                                     void* stream);
/* Training targets Zt [n][64] (FP32) from omega [S*ld]. */
PYRO_API int pyro_surrogate_targets(const pyro_mech* mech, int64_t n, int64_t ld,
                                    const double* wdot, const double* scale,
                                    const double* mean, const double* std_dev, float* Zt,
                                    void* stream);

/* Bytes of device workspace pyro_surrogate_eval and pyro_surrogate_outputs
 * need for n cells (0 for an unsupported hidden width: evaluation supports
 * H = 64, 128, 256). */
PYRO_API size_t pyro_surrogate_workspace_size(const pyro_mech* mech, int64_t n, int hidden,
                                              int members);
/* Raw outputs Z [members][n][64] (FP32, device) of every member on the cells,
 * from the same fused kernel as pyro_surrogate_eval (before the ensemble mean
 * and the inverse transform).  workspace: device, 256-byte aligned. */
PYRO_API int pyro_surrogate_outputs(const pyro_mech* mech, const pyro_surrogate* sur,
                                    int64_t n, int64_t ld, const double* rho, const double* T,
                                    const double* Y, float* Z, void* workspace,
                                    size_t workspace_bytes, void* stream);
/*
 * Surrogate evaluation with fallback: wdot [S*ld] receives the prediction
 * omega_k = s_k sinh(mu_k + sigma_k zbar_k) from the ensemble-mean output
 * zbar, then the exact production rates for every cell that is not kept: a
 * cell is kept only if its prediction is finite, its ensemble spread
 * sqrt(sum_e ||omega^e - omega||^2 / E) / ||omega|| (omega^e from member e
 * alone) is below thr_spread and its element residual
 * ||A omega|| / || |A| |omega| || is below thr_resid (both strictly).  fell_back[n] (device u8) marks those
 * cells, *n_fallback (device int64) counts them; indicators, if not NULL,
 * receives the spread [n] then the residual [n].  thr = 0 sends every cell
 * to the exact kernel, +inf none; when a threshold admits no cell (<= 0 or
 * NaN) and indicators is NULL, the network is not run and the call is the
 * exact kernel on every cell (same wdot, flags and count).
 */
PYRO_API int pyro_surrogate_eval(const pyro_mech* mech, const pyro_surrogate* sur,
                                 int64_t n, int64_t ld, const double* rho, const double* T,
                                 const double* Y, double thr_spread, double thr_resid,
                                 double* wdot, uint8_t* fell_back, int64_t* n_fallback,
                                 double* indicators, void* workspace, size_t workspace_bytes,
                                 void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PYRO_H */
