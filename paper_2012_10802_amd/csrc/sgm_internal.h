// Internal interface between the C-ABI layer (sgm_api.cpp) and the HIP
// kernels (sgm_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sgm {

// Launch configuration chosen at plan time.
struct KernelConfig {
    int vpl;        // disparities per lane; 16 lanes carry one scanline
    bool aligned;   // w % vpl == 0: vector loads/stores of a lane's values
    bool l8;        // per-path aggregated costs fit in uint8 (Cmax + P2 <= 255)
    int agg_block;  // threads per aggregation workgroup (multiple of 64)
};

struct Problem {
    int W, H, w, n, npaths, p1, p2, cmax;
};

// All launchers return hipSuccess or the launch error.
hipError_t launch_census(const Problem &pb, const uint8_t *img, int pitch, uint64_t *codes,
                         hipStream_t s);
hipError_t launch_cost(const Problem &pb, const KernelConfig &kc, const uint64_t *cl,
                       const uint64_t *cr, const int32_t *d_lo, uint8_t *cost, hipStream_t s);
// Aggregates the directions listed in paths[0..np) into np volumes at
// out + i * W*H*w elements (uint8 when l8, else uint16).
hipError_t launch_aggregate(const Problem &pb, const KernelConfig &kc, const uint8_t *cost,
                            const int *paths, int np, bool l8, void *out, hipStream_t s);
// S = sum of np volumes (uint8 when l8, else uint16) -> uint16.
hipError_t launch_sum(const Problem &pb, const KernelConfig &kc, const void *vols, int np,
                      bool l8, uint16_t *sum, hipStream_t s);
// Winner-take-all + sub-pixel on S (uint16) ...
hipError_t launch_wta_sum(const Problem &pb, const KernelConfig &kc, const uint16_t *sum,
                          const int32_t *d_lo, uint16_t *dint, float *dsub, hipStream_t s);
// ... or directly on np per-path volumes, summing on the fly.
hipError_t launch_wta_paths(const Problem &pb, const KernelConfig &kc, const void *vols, int np,
                            bool l8, const int32_t *d_lo, uint16_t *dint, float *dsub,
                            hipStream_t s);

}  // namespace sgm
