// Internal interface between the C-ABI layer (sgm_api.cpp) and the HIP
// kernels (sgm_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/sgm.h"

namespace sgm {

// thread-local text of the last failure (sgm_last_error)
constexpr int kErrorBufferSize = 512;
constexpr int kCensusTW = 64;  // census tile width in pixels (16 threads of 4 pixels)
constexpr int kCensusTH = 16;  // census tile height in rows (16 threads per row)
char *error_buffer();
// The aggregation addresses a volume with 32-bit byte offsets and drops a
// store by pointing it at byte 2^31, which must lie outside every volume:
// a uint16 volume therefore holds fewer than 2^30 values.
constexpr long long kMaxU16Volume = 1ll << 30;

// Lane mapping of the volume kernels: `lanes` lanes carry one scanline of
// the aggregation (one pixel of the selection), each holding `vpl`
// consecutive window values.  Compiled mappings: 16 lanes with vpl 2, 4, 8,
// 12 or 16 (any window width); 8 lanes with vpl 4 or 8 and 4 lanes with vpl
// 4, 8, 12 or 16, only for widths that are a multiple of vpl.
struct Mapping {
    int lanes, vpl;
};

// The mapping for window width w (1..256) and a requested lane count (4, 8
// or 16; 0 = 16).  A request that no compiled mapping serves at this width
// falls back to 16 lanes.
inline Mapping choose_mapping(int w, int lanes)
{
    if (lanes == 4 || lanes == 8) {
        static const int v8[] = {4, 8}, v4[] = {4, 8, 12, 16};
        const int *v = lanes == 8 ? v8 : v4;
        const int n = lanes == 8 ? 2 : 4;
        for (int i = 0; i < n; ++i)
            if (lanes * v[i] >= w && w % v[i] == 0) return Mapping{lanes, v[i]};
    }
    return Mapping{16, w <= 32 ? 2 : (w <= 64 ? 4 : (w <= 128 ? 8 : (w <= 192 ? 12 : 16)))};
}

// The selection's mapping: the fewest lanes per pixel that serve w (more
// pixels per wave, fewer idle lanes and cross-lane steps).
inline Mapping select_mapping(int w)
{
    Mapping m = choose_mapping(w, 4);
    if (m.lanes == 16) m = choose_mapping(w, 8);
    return m;
}

// Launch configuration chosen at plan time.
struct KernelConfig {
    int lanes;      // aggregation: lanes per scanline (4, 8 or 16)
    int vpl;        // aggregation: disparities per lane
    int wta_lanes;  // selection: lanes per pixel
    int wta_vpl;    // selection: disparities per lane
    bool aligned;   // vector loads/stores of a lane's values (w % vpl == 0
                    // and buffers aligned); false only with 16-lane mappings
    bool l8;        // per-path aggregated costs fit in uint8 (Cmax + P2 <= 255)
    int agg_block;  // threads per aggregation workgroup (multiple of 64)
    int agg_order;  // dispatch order of the aggregation's direction slots
                    // after the horizontal ones: 0 diagonal then vertical,
                    // 1 vertical then diagonal
};

struct Problem {
    int W, H, w, n, npaths, p1, p2, cmax;
};

// One-shot injected failures (see sgm_debug_inject_fault): true once for
// the armed kind, which is then disarmed.
enum { kFaultLaunch = 1, kFaultAlloc = 2 };
bool fault_take(int kind);

// All launchers return hipSuccess or the launch error.
hipError_t launch_census(const Problem &pb, const uint8_t *img, int pitch, uint64_t *codes,
                         hipStream_t s);
// both images of a pair in one launch
hipError_t launch_census_lr(const Problem &pb, const uint8_t *left, const uint8_t *right, int pitch, uint64_t *cl,
                            uint64_t *cr, hipStream_t s);
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

// ---------------------------------------------------------------------------
// per-pixel windows (w <= 16)

hipError_t launch_downsample4(const uint8_t *img, int W, int H, int pitch, long long img_stride, int nimg,
                              uint8_t *out, hipStream_t s);
hipError_t launch_cost_win(const Problem &pb, const uint64_t *cl, const uint64_t *cr, const int32_t *lo,
                           uint8_t *cost, hipStream_t s);
hipError_t launch_aggregate_win(const Problem &pb, const uint8_t *cost, const int32_t *lo, const int *paths, int np,
                                bool l8, void *out, long long vstride, hipStream_t s);
hipError_t launch_wta_win(const Problem &pb, const void *vols, long long vstride, int np, bool l8, const int32_t *lo,
                          uint16_t *dint, float *dsub, hipStream_t s);

// npairs pairs of one size, w = 16 and uint8 volumes: census, cost,
// aggregation (one launch, one scanline per lane) and selection.  Pair i's
// scratch (codes, cost, volumes) sits at i * ws_pair bytes from the first
// pair's pointers below.
struct WinPairs {
    const uint8_t *left, *right;
    int pitch;
    long long img_pair;  // bytes between the images of consecutive pairs
    const int32_t *lo;   // [npairs][H][W]
    int npairs;
    size_t ws_pair;      // bytes of workspace per pair
    uint8_t *lo8;        // the pair's window starts as bytes (in its workspace slice)
    uint64_t *codes_l, *codes_r;
    uint8_t *cost, *paths;
    long long vstride;   // bytes between direction volumes
    uint16_t *dint;      // [npairs][H][W]
    float *dsub;         // [npairs][H][W] or NULL
};
hipError_t launch_match_win_pairs(const Problem &pb, const WinPairs &b, hipStream_t s);

// ---------------------------------------------------------------------------
// batches

// Device descriptor of one pair.  Caller buffers are absolute pointers;
// scratch buffers are byte offsets into the run's workspace, so one table
// serves every workspace (and a captured graph keeps working).
struct PairDev {
    const uint8_t *left, *right;
    const int32_t *d_lo;
    uint16_t *dint;
    float *dsub;
    long long off_codes_l, off_codes_r, off_cost, off_vols;
    long long vstride;  // elements between per-direction volumes
    int32_t W, H, w, pitch, lanes, vpl, pad, wta_lanes, wta_vpl;
    int32_t h_vpl, h_pad;  // the horizontal directions' 16-lane mapping
    int32_t census_start, cost_start, wta_start;  // first block of the pair in each batched grid
    int32_t census_tx, census_ty, cost_tx;
};

struct BatchDev {
    uint8_t *ws;             // workspace base
    const PairDev *pairs;    // in the workspace
    const uint32_t *items;   // in the workspace: (pair << 8 | direction, group) per item
    uint32_t *counter;       // in the workspace
    int npairs, nitems;
    uint32_t p1x2, p2x2;
    int cmax, npaths;
};

// Workgroups of each batched grid (the last pair's start + its count).
struct BatchGrids {
    int census, cost, wta;
};

// ev (may be NULL, as may each entry): events recorded before the census,
// cost, aggregation and selection launches and after the selection.
hipError_t launch_batch(const BatchDev &b, const BatchGrids &g, int census_n, bool l8, int agg_waves,
                        hipStream_t s, const hipEvent_t *ev = nullptr);

// ---------------------------------------------------------------------------
// road model (fit, windows, disparity transformation)

size_t road_workspace_bytes(int W, int H, int nimg);
hipError_t launch_road_energy(const float *disp, const uint8_t *mask, int W, int H, int nimg, float min_disp,
                              double margin, const sgm_road_fit *prior, double tol, const double *phi, int nphi,
                              double *energy, void *ws, hipStream_t s);
hipError_t launch_road_fit(const float *disp, const uint8_t *mask, int W, int H, int nimg, float min_disp,
                           double margin, const sgm_road_fit *prior, double tol, sgm_road_fit *fit, void *ws,
                           hipStream_t s);
hipError_t launch_road_window(const sgm_road_fit *fit, int W, int H, int nimg, int w, int mode, double delta,
                              double scale, int32_t *d_lo, hipStream_t s);
hipError_t launch_disp_transform(const float *disp, const sgm_road_fit *fit, int W, int H, int nimg,
                                 double delta, float *out, hipStream_t s);

// ---------------------------------------------------------------------------
// pothole threshold and labelling

hipError_t launch_road_window_map(const sgm_road_fit *fit, int W, int H, int nimg, int w, double scale, int32_t *lo,
                                  hipStream_t s);
hipError_t launch_road_mask(const float *disp, const sgm_road_fit *fit, int W, int H, int nimg, double f_min,
                            double margin, uint8_t *mask, hipStream_t s);
size_t pothole_workspace_bytes(int nbins, int nimg);
constexpr int kSlicMaxRounds = 100;  // the most SLIC rounds one call runs
size_t slic_workspace_bytes(int W, int H, int S, int nimg);
hipError_t launch_slic(const float *d2, const uint8_t *mask, int W, int H, int nimg, int S, double m, int iters,
                       double tol, int32_t *rounds, int32_t *labels, float *d3, double *centres, void *ws,
                       hipStream_t s);
hipError_t launch_pothole_threshold(const float *d2, const uint8_t *mask, int W, int H, int nimg, double lo,
                                    double b, int nbins, double delta_pd, sgm_pothole_threshold *out,
                                    double *curve, void *ws, hipStream_t s);
hipError_t launch_pothole_prune(const int32_t *superpixels, int W, int H, int nimg, int32_t *labels, hipStream_t s);
hipError_t launch_pothole_label(const float *d2, const uint8_t *mask, int W, int H, int nimg,
                                const sgm_pothole_threshold *thr, int32_t *labels, hipStream_t s);

}  // namespace sgm
