// Internal declarations of libpyro: device tables of a loaded mechanism and
// the kernel launchers.  Not part of the public ABI (include/pyro.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "pyro.h"

namespace pyro {

// Universal gas constant (J mol^-1 K^-1) and the 1 atm reference pressure of
// the equilibrium constants (Appendix A.1, eq. equil_constants).
constexpr double kGasConstant = 8.314462618;
constexpr double kOneAtm = 101325.0;

// Cells per tile of the production-rate kernel (one cell per lane of a
// 64-wide wavefront) and waves per workgroup.
constexpr int kTile = 64;
constexpr int kWaves = 8;
// Reactions each wave evaluates per chunk; a chunk's rates of progress are
// parked in LDS before the species that own them gather their sums.
constexpr int kRxnPerWave = 2;
constexpr int kChunk = kWaves * kRxnPerWave;
// Max species a wave owns (accumulates) in the production-rate kernel.
constexpr int kMaxOwn = 64;
// Max third-body/falloff reactions a wave evaluates per tile; their [M]
// live in registers of that wave.
constexpr int kMaxPd = 16;
// Max molecules per reaction side.
constexpr int kMaxSide = 3;
// Max distinct T_mid values among the species (Newton kernel groups).
constexpr int kMaxTmidGroups = 4;
constexpr int kVjpWaves = 16;            // wavefronts of the reverse-sweep workgroup
constexpr int kVjpRow = kTile * 24;       // bytes per species row of the reverse sweep: C, G, wbar

// Reaction classes.
enum : int32_t { kElementary = 0, kThirdBody = 1, kLindemann = 2, kTroe = 3,
                 kNoReaction = -1 };

// One reaction as the production-rate kernel reads it: 64 bytes, read with a
// single scalar load because every lane of a wave handles the same reaction.
struct RxnRec {
    int32_t cls;          // class, or kNoReaction for an empty slot
    int32_t rev;          // 1 if reversible
    int32_t nr, np;       // molecules on each side (1..3)
    int32_t r[kMaxSide];  // byte offsets of the reactant slots in the C/G tile
    int32_t p[kMaxSide];  // byte offsets of the product slots
    int32_t dnu;          // sum of the net stoichiometric coefficients
    int32_t prow;         // row of the Arrhenius triple (the reaction index)
    int32_t pdw;          // position in the evaluating wave's [M] queue, -1 if none
    int32_t fo;           // falloff index, -1 if none
    int32_t qoff;         // byte offset of the rate-of-progress slot in a chunk
    int32_t pd;           // row of the efficiency table, -1 if none
};
static_assert(sizeof(RxnRec) == 64, "RxnRec must be 64 bytes");

// Species data of the species phase: g/RT coefficients for both NASA7
// ranges, with g/RT = c0 (1 - ln T) + c1 T + c2 T^2 + c3 T^3 + c4 T^4
// + c5 / T + c6, then T_mid and 1/W.
struct SpeciesRec {
    double lo[7];
    double hi[7];
    double t_mid;
    double inv_w;
};
static_assert(sizeof(SpeciesRec) == 128, "SpeciesRec must be 128 bytes");

// Troe data per falloff reaction: F_cent = (1-alpha) exp(T a3) + alpha
// exp(T a1) + exp(a2 / T) with a3 = -1/T***, a1 = -1/T*, a2 = -T**.
struct FalloffRec {
    double alpha, a3, a1, a2;
    int32_t troe;
    int32_t pad[7];
};
static_assert(sizeof(FalloffRec) == 64, "FalloffRec must be 64 bytes");

// Gathering entry: the byte offset of a rate-of-progress slot in its chunk
// buffer (bits 0-15) and the net coefficient nu as a signed 16-bit integer
// (bits 16-31).
using GatherEntry = uint32_t;

// Newton-kernel data: NASA7 coefficients a1..a6 of each range and 1/W.
struct NewtonSpecies {
    double lo[6];
    double hi[6];
    double inv_w;
    int32_t group;
    int32_t pad;
    double pad2[2];
};
static_assert(sizeof(NewtonSpecies) == 128, "NewtonSpecies must be 128 bytes");

// Device-side view of a mechanism, passed to kernels by value.
// Device-side view of a read-only table as constant-address-space memory:
// the tables never change while a kernel runs, and saying so lets the
// compiler read wave-uniform entries with scalar loads even inside loops that
// also store (which it cannot otherwise prove do not overwrite them).
// (the host pass only parses device code and sees a plain pointer)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
#else
template <typename T>
using cptr = const T*;
#endif
template <typename T>
__device__ inline cptr<T> cst(const T* p) {
    return (cptr<T>)(p);
}

// The double whose upper 16 bits are top (lower 48 bits zero).  Table
// coefficients stored this way reach the FMAs as scalar operands, with no
// conversion instruction.
__device__ inline double from_top16(uint32_t top) {
    return __builtin_bit_cast(double, uint64_t(top) << 48);
}

// The tables of one work schedule (see the loader): chunks of waves x rpw
// reaction slots, species owned per wave, gathering lists.
struct DevSched {
    int32_t n_chunks;
    int32_t n_pd_rows;                   // Jacobian rows: third-body rows of the row
    const RxnRec* rxn;                   // [n_chunks][waves][rpw]
    const double* effw;                  // [waves][S][MAXPD] efficiencies by queue slot
    const int32_t* n_pdw;                // [waves]
    const int32_t* own;                  // [waves][kMaxOwn]
    const int32_t* n_own;                // [waves]
    const int32_t* gptr;                 // [n_chunks][waves][kMaxOwn + 1]
    // reverse sweep: two words per entry, (slot offset | top16(nu') << 16,
    // top16(-nu'') | top16(nu' - nu'') << 16), top16(x) being the upper 16
    // bits of the double x (exact for small integers)
    const uint32_t* gent;
    const int32_t* pd_list;              // [waves][kMaxPd] third-body rows in chunk order
    const double* effo;                  // [waves][n_pd][MAXOWN] by owned species
    const int32_t* pd_rows;              // Jacobian rows: [n_pd_rows] third-body rows
};

struct DevMech {
    int32_t S, R, n_pd, n_fo;
    int32_t n_chunks;
    int32_t s_pad;                       // S rounded up to a multiple of 8
    int32_t n_groups;
    int32_t pad;
    double t_mid_group[kMaxTmidGroups];
    const SpeciesRec* species;           // [S]
    const RxnRec* rxn;                   // [n_chunks][waves][kRxnPerWave]
    const FalloffRec* falloff;           // [n_fo]
    const double* effw;                  // [waves][S][MAXPD] efficiencies by wave slot
    const int32_t* n_pdw;                // [waves] third-body/falloff reactions per wave
    const double* params;                // [R + n_fo][3] default triples
    const int32_t* own;                  // [waves][kMaxOwn] species owned
    const int32_t* n_own;                // [waves]
    const int32_t* gptr;                 // [n_chunks][waves][kMaxOwn + 1]
    const GatherEntry* gent;             // gathering entries
    const NewtonSpecies* newton;         // [S]
    const double* w;                     // [S] molar masses
    // reverse sweep (VJP): its own schedule over kVjpWaves wavefronts
    DevSched vjp;
    const double* eff_t;                 // [S][n_pd] efficiencies by species
    // reaction-equilibrium variant: per forward slot, the combined Gibbs
    // coefficients sum_k nu_kj c_k (low range [7], high range [7], T_mid, 0)
    const double* rxn_kc;                // [n_chunks][waves][kRxnPerWave][16]
    // MFMA third-body variant: B fragments of eps^T, [pd block][K-step][lane]
    // = eps[16 pb + l%16][4 kk + l/16] (zero outside n_pd x S)
    const double* eps_frag;
    // MFMA net-rate variant (S <= 64): B fragments of nu per chunk,
    // [chunk][species block 0..3][K-step 0..3][lane] = nu[16 sb + l%16][reaction
    // in slot 4 kk + l/16] (zero for empty slots and species past S)
    const double* nu_frag;
    // matrix-core log products (log-space FP64 variant): B fragments of nu'
    // (side 0) and nu'' (side 1) per chunk, [chunk][side][slot block][K-step]
    // [lane] = nu[4 kk + l/16][slot 16 sb + l%16] (zero for empty slots and
    // species past S); lp_nks K-steps of 4 species (0: table not built)
    const double* lp_frag;
    // Jacobian rows: per species j, the reverse-sweep schedule of the
    // reactions with a nonzero net coefficient of j ([S]; ownership tables
    // shared with vjp)
    const DevSched* jac_rows;
    // surrogate
    int32_t E;                           // elements
    int32_t lp_nks;
    const double* comp;                  // [E][S] atoms of element e in species k
};

// Device tables of a set of transport fits (see the transport kernel).
struct TransportTables {
    const double* inv_w;                 // [S] 1/W_k
    const double* visc;                  // [S][5] viscosity fit b_km
    const double* cond;                  // [S][5] conductivity fit c_km
    const double* pair;                  // [S (j)][S (k)][8]: w_kj, v_kj, a_kj0..4, 0
};

}  // namespace pyro

struct pyro_transport {
    int device = 0;
    int S = 0;
    pyro::TransportTables tt{};
    void* blob = nullptr;
};

struct pyro_mech {
    int device = 0;
    int S = 0, R = 0, E = 0, n_tb = 0, n_fo = 0;
    int nnz_f = 0, nnz_r = 0, nnz_net = 0;
    int max_own = 0;
    int max_pdw = 0;
    int vjp_max_own = 0;                 // the same for the reverse-sweep schedule
    int vjp_max_pdw = 0;
    bool kc_ok = false;                  // every reaction's species share one T_mid
    int wdot_variant = PYRO_WDOT_SPECIES_EQUILIBRIUM;
    // wavefronts of the production-rate workgroup: kWaves, or 2 kWaves for
    // mechanisms whose species rows leave room for only one workgroup per CU
    int fw_waves = pyro::kWaves;
    int n_cu = 0;                        // compute units of the device
    std::vector<double> W;               // host copy
    std::vector<double> params;          // host copy of the default triples
    pyro::DevMech dev{};
    void* blob = nullptr;                // one device allocation for all tables
    size_t blob_bytes = 0;
};

namespace pyro {

// Thread-local error message used by pyro_last_error().
void set_error(const std::string& msg);
void clear_error();
int fail(int code, const std::string& msg);
int hip_fail(hipError_t err, const char* what);

// Parses and validates a .pyromech file, builds the tables and uploads them.
int load_mechanism(const char* path, pyro_mech** out);

// Launchers (arguments already validated).
// n_dev: optional device-resident cell count (<= n) read by the kernel; the
// launch covers n cells and tiles past *n_dev exit at once.
hipError_t launch_production_rates(const pyro_mech* m, int64_t n, int64_t ld,
                                   int dtype, const void* rho, const void* T,
                                   const void* Y, void* wdot,
                                   const double* params, hipStream_t stream,
                                   const int64_t* n_dev = nullptr);
hipError_t launch_temperature(const pyro_mech* m, int64_t n, int64_t ld,
                              const double* e, const double* Y,
                              const double* T_guess, double T_guess_value,
                              double* T_out, int32_t* status, int max_iter,
                              double rtol, hipStream_t stream, bool enthalpy = false);
hipError_t launch_primitive(const pyro_mech* m, int64_t n, int64_t ld, int dim,
                            const double* rhok, const double* mom, const double* E,
                            const double* T_guess, double T_guess_value, double* rho_out,
                            double* Y_out, double* u_out, double* T_out, double* p_out,
                            int32_t* status, int max_iter, double rtol, hipStream_t stream);
hipError_t launch_eos(const pyro_mech* m, int64_t n, int64_t ld, int mode,
                      const double* a, const double* T, const double* Y,
                      double* out, hipStream_t stream);
hipError_t launch_internal_energy(const pyro_mech* m, int64_t n, int64_t ld,
                                  const double* T, const double* Y,
                                  double* e_out, hipStream_t stream);
// LDS bytes the production-rate kernel needs for this mechanism.
size_t production_rates_lds_bytes(const pyro_mech* m, bool reaction_equilibrium,
                                  bool mfma_third_body = false, bool log_space = false,
                                  int real_bytes = 8, bool log_products = false);
// The log-space form (FP64 variant, and every FP32 call) can run this
// mechanism: one T_mid per reaction and its rows fit the LDS tile.
bool log_space_supported(const pyro_mech* m, int real_bytes);
// The FP64 log-space form with its log products on the matrix cores fits.
bool log_products_supported(const pyro_mech* m);
// ln C floor of that form (0 * ln 0 would poison the dense contraction)
constexpr double kLnFloor = 1e30;
hipError_t prepare_production_rates(const pyro_mech* m);
hipError_t launch_production_rates_vjp(const pyro_mech* m, int64_t n, int64_t ld,
                                       const double* rho, const double* T, const double* Y,
                                       const double* wbar, double* Ybar, double* Tbar,
                                       double* params_bar, double* wdot,
                                       const double* params, hipStream_t stream);
// Rows of the chemical Jacobian J[j][k] = dS_j/dY_k (S_j = W_j omega_j),
// J laid out [S][S][ld]; dSdT ([S][ld]) optional.
hipError_t launch_chemical_jacobian(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                                    const double* T, const double* Y, int fixed_energy,
                                    double* J, double* dSdT, const double* params,
                                    hipStream_t stream);
// The same at fixed energy, J in 64-cell tiles of whole matrices: element
// (j, k) of cell c at J[((c / 64) S S + j S + k) 64 + c % 64], so that one
// cell's matrix spans one tile (S S 64 doubles) rather than S S cell rows.
hipError_t launch_chemical_jacobian_tiled(const pyro_mech* m, int64_t n, int64_t ld,
                                          const double* rho, const double* T, const double* Y,
                                          double* J, hipStream_t stream);
size_t vjp_lds_bytes(const pyro_mech* m);
// Fixed scratch of the allocation-free VJP (per-workgroup parameter partials).
constexpr size_t kVjpScratchDoubles = size_t(1) << 19;    // 4 MiB
hipError_t vjp_scratch_init(int device);
int vjp_scratch_blocks(const pyro_mech* m, int64_t n);
hipError_t launch_production_rates_vjp_noalloc(const pyro_mech* m, int64_t n, int64_t ld,
                                               const double* rho, const double* T,
                                               const double* Y, const double* wbar,
                                               double* Ybar, double* Tbar, double* params_bar,
                                               double* wdot, const double* params,
                                               hipStream_t stream);
// Reactor steps (method 0: Runge-Kutta, 1: Crank-Nicolson) and the bytes of
// workspace they carve.
size_t reactor_workspace_bytes(const pyro_mech* m, int64_t n, int64_t ld, int method);
hipError_t launch_rk4_step(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                           const double* e, double* Y, double* T, const double* dt,
                           double dt_value, int32_t* status, void* ws, hipStream_t s);
hipError_t launch_cn_step(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                          const double* e, double* Y, double* T, const double* dt,
                          double dt_value, double tol, int max_iter, int32_t* status, void* ws,
                          hipStream_t s);
hipError_t launch_transport(const pyro_mech* m, const TransportTables& tt, int64_t n,
                            int64_t ld, const double* T, const double* Y, double* mu,
                            double* kappa, double* D, hipStream_t stream);
bool nq_supported(const pyro_mech* m);
hipError_t prepare_vjp(const pyro_mech* m);

}  // namespace pyro
