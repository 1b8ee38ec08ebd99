// Internal declarations of the surrogate pipeline.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct pyro_mech;

namespace pyro {

constexpr int kFeatPad = 64;     // feature row: T, log10 p, S log-mass-fractions, 1, zeros
constexpr int kOutPad = 64;      // target row: S values, zeros
constexpr int kMaxElements = 16;
constexpr int kMaxMembers = 4;

hipError_t launch_features(const pyro_mech* m, int64_t n, int64_t ld, const double* rho,
                           const double* T, const double* Y, const float* shift,
                           const float* scale, uint16_t* X, hipStream_t stream);
hipError_t launch_targets(const pyro_mech* m, int64_t n, int64_t ld, const double* wdot,
                          const double* ts, const double* tmu, const double* tsig, float* Zt,
                          hipStream_t stream);
// fused inference (hidden widths 64, 128, 256)
bool fused_supported(int hidden);
int64_t packed_weight_elems(int hidden);
hipError_t launch_pack(int hidden, int members, int64_t w_total, int64_t b_total,
                       const uint16_t* W, const float* b, uint16_t* wp, float* bp,
                       hipStream_t stream);
// zout == nullptr: evaluation (wdot, flag, optional ind), the member outputs
// staged in zstage [members][S][n]; otherwise the raw member outputs
// [members][n][64] into zout
hipError_t launch_fused(const pyro_mech* m, int hidden, int members, int64_t n, int64_t ld,
                        const double* rho, const double* T, const double* Y,
                        const uint16_t* wp, const float* bp, int64_t w_stride, int64_t b_stride,
                        const float* shift, const float* scale, const double* ts,
                        const double* tmu, const double* tsig, double thr_spread,
                        double thr_resid, double* wdot, uint8_t* flag, double* ind, float* zout,
                        float* zstage, hipStream_t stream);
int64_t compaction_blocks(int64_t n);
hipError_t launch_compaction(int64_t n, const uint8_t* flag, int64_t* counts, int64_t* total,
                             int64_t* idx, hipStream_t stream);
hipError_t launch_fallback_all(int64_t n, uint8_t* flag, int64_t* total, hipStream_t stream);
hipError_t launch_gather(int S, int64_t n, int64_t ld, const int64_t* count, const int64_t* idx,
                         const double* rho, const double* T, const double* Y, double* rc,
                         double* Tc, double* Yc, hipStream_t stream);
hipError_t launch_scatter(int S, int64_t n, int64_t ld, const int64_t* count, const int64_t* idx,
                          const double* wc, double* wdot, hipStream_t stream);

}  // namespace pyro
