// Host-only stand-in for the device side of libsgm, for the sanitizer run of
// the library's host code (test infrastructure, never part of the library).
//
// The C-ABI layer (sgm_api.cpp, sgm_batch_api.cpp) is compiled unchanged
// for the host with AddressSanitizer and UndefinedBehaviorSanitizer and
// linked against this file instead of the HIP runtime and the kernels:
//   * the HIP runtime calls it makes are answered on the host (device memory
//     is host memory, copies are memcpy, events and graphs are tokens);
//   * every kernel launcher checks the launch configuration the host chose
//     and touches the first and last byte of every buffer the kernel would
//     read or write, so a wrong size or offset in a workspace layout becomes
//     an AddressSanitizer report;
//   * the batch launcher also walks the descriptor table and the queue the
//     host uploaded and checks that every scanline group of every pair and
//     direction is queued exactly once and that the per-pair grids tile the
//     batched grids.
// A failed check prints its reason and aborts.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <set>
#include <tuple>

#include "../../paper_2012_10802_amd/csrc/sgm_internal.h"

#define CHECK(c)                                                                     \
    do {                                                                             \
        if (!(c)) {                                                                  \
            fprintf(stderr, "fake device: check failed at line %d: %s\n", __LINE__, #c); \
            abort();                                                                 \
        }                                                                            \
    } while (0)

namespace {

volatile unsigned char g_sink;

// read the first and last byte of [p, p + n)
void touch_r(const void *p, size_t n)
{
    if (!n) return;
    CHECK(p != nullptr);
    const unsigned char *b = static_cast<const unsigned char *>(p);
    g_sink = b[0];
    g_sink = b[n - 1];
}
// write the first and last byte of [p, p + n)
void touch_w(void *p, size_t n)
{
    if (!n) return;
    CHECK(p != nullptr);
    unsigned char *b = static_cast<unsigned char *>(p);
    b[0] = 0x5A;
    b[n - 1] = 0x5A;
}

size_t vol(const sgm::Problem &pb) { return (size_t)pb.W * pb.H * pb.w; }
size_t npix(const sgm::Problem &pb) { return (size_t)pb.W * pb.H; }

void check_mapping(int w, int lanes, int vpl, bool aligned)
{
    CHECK(lanes == 4 || lanes == 8 || lanes == 16);
    if (lanes == 16) CHECK(vpl == 2 || vpl == 4 || vpl == 8 || vpl == 12 || vpl == 16);
    if (lanes == 8) CHECK(vpl == 4 || vpl == 8);
    if (lanes == 4) CHECK(vpl == 4 || vpl == 8 || vpl == 12 || vpl == 16);
    CHECK(lanes * vpl >= w);
    if (lanes < 16) CHECK(aligned && w % vpl == 0);
    if (aligned) CHECK(w % vpl == 0);
}

long long vol_stride_elems(const sgm::Problem &pb, bool l8)
{
    const long long esz = l8 ? 1 : 2;
    return (((long long)vol(pb) * esz + 255) / 256 * 256) / esz;
}

int groups(int r, int W, int H, int lpi)
{
    if (r <= 1) return (H + lpi - 1) / lpi;
    if (r <= 3) return (W + lpi - 1) / lpi;
    return (W + H - 1 + lpi - 1) / lpi;
}

}  // namespace

// ---------------------------------------------------------------------------
// HIP runtime, answered on the host

extern "C" {

hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int)
{
    *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 0;
    return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600 *p, int)
{
    memset(p, 0, sizeof *p);
    snprintf(p->gcnArchName, sizeof p->gcnArchName, "gfx950:fake host");
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "fake device error"; }
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = reinterpret_cast<hipEvent_t>(new int(0));
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e)
{
    delete reinterpret_cast<int *>(e);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t)
{
    CHECK(e != nullptr);
    ++*reinterpret_cast<int *>(e);
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e)
{
    CHECK(e != nullptr);
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    CHECK(a && b);
    *ms = 1.0f;
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned)
{
    *p = malloc(n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void *p)
{
    free(p);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t)
{
    if (n) memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g)
{
    *g = reinterpret_cast<hipGraph_t>(new int(1));
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *, char *, size_t)
{
    CHECK(g != nullptr);
    *x = reinterpret_cast<hipGraphExec_t>(new int(2));
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t)
{
    CHECK(x != nullptr);
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g)
{
    delete reinterpret_cast<int *>(g);
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x)
{
    delete reinterpret_cast<int *>(x);
    return hipSuccess;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// kernel launchers: configuration checks and buffer extents

namespace sgm {

hipError_t launch_census(const Problem &pb, const uint8_t *img, int pitch, uint64_t *codes, hipStream_t)
{
    CHECK(pitch >= pb.W && (pb.n == 3 || pb.n == 5 || pb.n == 7));
    touch_r(img, (size_t)(pb.H - 1) * pitch + pb.W);
    touch_w(codes, npix(pb) * 8);
    return hipSuccess;
}

hipError_t launch_census_lr(const Problem &pb, const uint8_t *left, const uint8_t *right, int pitch, uint64_t *cl,
                            uint64_t *cr, hipStream_t s)
{
    launch_census(pb, left, pitch, cl, s);
    return launch_census(pb, right, pitch, cr, s);
}

hipError_t launch_cost(const Problem &pb, const KernelConfig &, const uint64_t *cl, const uint64_t *cr,
                       const int32_t *d_lo, uint8_t *cost, hipStream_t)
{
    touch_r(cl, npix(pb) * 8);
    touch_r(cr, npix(pb) * 8);
    if (d_lo) touch_r(d_lo, (size_t)pb.H * 4);
    touch_w(cost, vol(pb));
    return hipSuccess;
}

hipError_t launch_aggregate(const Problem &pb, const KernelConfig &kc, const uint8_t *cost, const int *paths,
                            int np, bool l8, void *out, hipStream_t)
{
    check_mapping(pb.w, kc.lanes, kc.vpl, kc.aligned);
    CHECK(kc.agg_block % 64 == 0 && kc.agg_block >= kc.lanes);
    CHECK(np >= 1 && np <= 8);
    std::set<int> seen;
    for (int i = 0; i < np; ++i) {
        CHECK(paths[i] >= 0 && paths[i] < 8);
        CHECK(seen.insert(paths[i]).second);
    }
    touch_r(cost, vol(pb));
    const size_t esz = l8 ? 1 : 2;
    uint8_t *o = static_cast<uint8_t *>(out);
    touch_w(o, ((size_t)(np - 1) * vol_stride_elems(pb, l8) + vol(pb)) * esz);
    return hipSuccess;
}

hipError_t launch_sum(const Problem &pb, const KernelConfig &, const void *vols, int np, bool l8, uint16_t *sum,
                      hipStream_t)
{
    const size_t esz = l8 ? 1 : 2;
    touch_r(vols, ((size_t)(np - 1) * vol_stride_elems(pb, l8) + vol(pb)) * esz);
    touch_w(sum, vol(pb) * 2);
    return hipSuccess;
}

hipError_t launch_wta_sum(const Problem &pb, const KernelConfig &kc, const uint16_t *sum, const int32_t *d_lo,
                          uint16_t *dint, float *dsub, hipStream_t)
{
    CHECK(kc.vpl * 16 >= pb.w);
    touch_r(sum, vol(pb) * 2);
    if (d_lo) touch_r(d_lo, (size_t)pb.H * 4);
    touch_w(dint, npix(pb) * 2);
    if (dsub) touch_w(dsub, npix(pb) * 4);
    return hipSuccess;
}

hipError_t launch_wta_paths(const Problem &pb, const KernelConfig &kc, const void *vols, int np, bool l8,
                            const int32_t *d_lo, uint16_t *dint, float *dsub, hipStream_t)
{
    check_mapping(pb.w, kc.wta_lanes, kc.wta_vpl, kc.aligned);
    const size_t esz = l8 ? 1 : 2;
    touch_r(vols, ((size_t)(np - 1) * vol_stride_elems(pb, l8) + vol(pb)) * esz);
    if (d_lo) touch_r(d_lo, (size_t)pb.H * 4);
    touch_w(dint, npix(pb) * 2);
    if (dsub) touch_w(dsub, npix(pb) * 4);
    return hipSuccess;
}

hipError_t launch_downsample4(const uint8_t *img, int W, int H, int pitch, long long img_stride, int nimg,
                              uint8_t *out, hipStream_t)
{
    CHECK(W >= 4 && H >= 4 && pitch >= W && nimg >= 1);
    touch_r(img, (size_t)(nimg - 1) * img_stride + (size_t)(H - 1) * pitch + W);
    touch_w(out, (size_t)nimg * (W / 4) * (H / 4));
    return hipSuccess;
}

hipError_t launch_cost_win(const Problem &pb, const uint64_t *cl, const uint64_t *cr, const int32_t *lo,
                           uint8_t *cost, hipStream_t)
{
    touch_r(cl, npix(pb) * 8);
    touch_r(cr, npix(pb) * 8);
    touch_r(lo, npix(pb) * 4);
    touch_w(cost, npix(pb) * 16);
    return hipSuccess;
}

hipError_t launch_aggregate_win(const Problem &pb, const uint8_t *cost, const int32_t *lo, const int *paths, int np,
                                bool l8, void *out, long long vstride, hipStream_t)
{
    CHECK(np >= 1 && np <= 8 && pb.w <= 16);
    for (int i = 0; i < np; ++i) CHECK(paths[i] >= 0 && paths[i] < 8);
    touch_r(cost, vol(pb));
    touch_r(lo, npix(pb) * 4);
    const size_t esz = l8 ? 1 : 2;
    touch_w(out, ((size_t)(np - 1) * vstride + vol(pb)) * esz);
    return hipSuccess;
}

hipError_t launch_wta_win(const Problem &pb, const void *vols, long long vstride, int np, bool l8, const int32_t *lo,
                          uint16_t *dint, float *dsub, hipStream_t)
{
    const size_t esz = l8 ? 1 : 2;
    touch_r(vols, ((size_t)(np - 1) * vstride + vol(pb)) * esz);
    touch_r(lo, npix(pb) * 4);
    touch_w(dint, npix(pb) * 2);
    if (dsub) touch_w(dsub, npix(pb) * 4);
    return hipSuccess;
}

hipError_t launch_match_win_pairs(const Problem &pb, const WinPairs &b, hipStream_t)
{
    CHECK(b.npairs >= 1 && pb.w == 16);
    const size_t last = (size_t)(b.npairs - 1);
    touch_r(b.left, last * b.img_pair + (size_t)(pb.H - 1) * b.pitch + pb.W);
    touch_r(b.right, last * b.img_pair + (size_t)(pb.H - 1) * b.pitch + pb.W);
    touch_r(b.lo, (size_t)b.npairs * npix(pb) * 4);
    touch_w(b.codes_l, last * b.ws_pair + npix(pb) * 8);
    touch_w(b.codes_r, last * b.ws_pair + npix(pb) * 8);
    touch_w(b.cost, last * b.ws_pair + vol(pb));
    if (b.lo8) touch_w(b.lo8, last * b.ws_pair + npix(pb));
    touch_w(b.paths, last * b.ws_pair + (size_t)(pb.npaths - 1) * b.vstride + vol(pb));
    touch_w(b.dint, (size_t)b.npairs * npix(pb) * 2);
    if (b.dsub) touch_w(b.dsub, (size_t)b.npairs * npix(pb) * 4);
    return hipSuccess;
}

// The batch: the uploaded descriptor table and queue must describe every
// pair's buffers inside the workspace, tile the batched grids and queue
// every scanline group once.
hipError_t launch_batch(const BatchDev &b, const BatchGrids &g, int census_n, bool l8, int agg_waves, hipStream_t,
                        const hipEvent_t *ev)
{
    CHECK(census_n == 3 || census_n == 5 || census_n == 7);
    CHECK(b.npairs >= 1 && agg_waves >= 1 && agg_waves <= b.nitems);
    touch_w(b.counter, 4);
    const size_t esz = l8 ? 1 : 2;
    int census_next = 0, cost_next = 0, wta_next = 0;
    std::set<std::tuple<int, int, int>> want;
    for (int i = 0; i < b.npairs; ++i) {
        const PairDev &P = b.pairs[i];
        CHECK(P.W >= 1 && P.H >= 1 && P.pitch >= P.W && P.w >= 1 && P.w <= 256);
        check_mapping(P.w, P.lanes, P.vpl, true);
        check_mapping(P.w, P.wta_lanes, P.wta_vpl, true);
        CHECK(P.pad == (P.w < P.lanes * P.vpl ? 1 : 0));
        const size_t np = (size_t)P.W * P.H, nv = np * P.w;
        touch_r(P.left, (size_t)(P.H - 1) * P.pitch + P.W);
        touch_r(P.right, (size_t)(P.H - 1) * P.pitch + P.W);
        if (P.d_lo) touch_r(P.d_lo, (size_t)P.H * 4);
        touch_w(P.dint, np * 2);
        if (P.dsub) touch_w(P.dsub, np * 4);
        for (int k = 0; k < 2; ++k) touch_w(b.ws + (k ? P.off_codes_r : P.off_codes_l), np * 8);
        touch_w(b.ws + P.off_cost, nv);
        CHECK(P.off_codes_l % 256 == 0 && P.off_codes_r % 256 == 0 && P.off_cost % 256 == 0 && P.off_vols % 256 == 0);
        touch_w(b.ws + P.off_vols, ((size_t)(b.npaths - 1) * P.vstride + nv) * esz);
        CHECK(P.census_start == census_next && P.cost_start == cost_next && P.wta_start == wta_next);
        CHECK(P.census_tx == (P.W + kCensusTW - 1) / kCensusTW && P.census_ty == (P.H + kCensusTH - 1) / kCensusTH);
        census_next += 2 * P.census_tx * P.census_ty;
        cost_next += P.cost_tx * P.H;
        const long long ppb = 256 / P.wta_lanes;
        wta_next += (int)(((long long)np + ppb - 1) / ppb);
        // horizontal directions: the 16-lane mapping, four scanlines per item
        check_mapping(P.w, 16, P.h_vpl, true);
        CHECK(P.h_pad == (P.w < 16 * P.h_vpl ? 1 : 0));
        for (int r = 0; r < b.npaths; ++r) {
            const int lpi = 64 / (r <= 1 ? 16 : P.lanes);
            for (int q = 0, n = groups(r, P.W, P.H, lpi); q < n; ++q) want.insert(std::make_tuple(i, r, q));
        }
    }
    CHECK(g.census == census_next && g.cost == cost_next && g.wta == wta_next);
    CHECK((size_t)b.nitems == want.size());
    std::set<std::tuple<int, int, int>> got;
    for (int it = 0; it < b.nitems; ++it) {
        const uint32_t w0 = b.items[2 * it], q = b.items[2 * it + 1];
        CHECK(got.insert(std::make_tuple((int)(w0 >> 8), (int)(w0 & 0xFF), (int)q)).second);
    }
    CHECK(got == want);
    for (int i = 0; ev && i < 5; ++i)
        if (ev[i]) hipEventRecord(ev[i], nullptr);
    return hipSuccess;
}

// road model, pothole threshold, superpixels: sizes of this stand-in's own
// workspaces, and the extents of the buffers each launcher names
size_t road_workspace_bytes(int W, int H, int nimg) { return (size_t)nimg * (4096 + (size_t)(W + H) * 8); }
size_t pothole_workspace_bytes(int nbins, int nimg) { return (size_t)nimg * (size_t)nbins * 64 + 256; }
size_t slic_workspace_bytes(int W, int H, int S, int nimg)
{
    return (size_t)nimg * ((size_t)(W / S + 1) * (H / S + 1) * 96 + 256);
}

hipError_t launch_road_energy(const float *disp, const uint8_t *mask, int W, int H, int nimg, float, double,
                              const sgm_road_fit *prior, double, const double *phi, int nphi, double *energy,
                              void *ws, hipStream_t)
{
    touch_r(disp, (size_t)nimg * W * H * 4);
    if (mask) touch_r(mask, (size_t)nimg * W * H);
    if (prior) touch_r(prior, (size_t)nimg * sizeof(sgm_road_fit));
    touch_r(phi, (size_t)nphi * 8);
    touch_w(energy, (size_t)nimg * nphi * 8);
    touch_w(ws, road_workspace_bytes(W, H, nimg));
    return hipSuccess;
}

hipError_t launch_road_fit(const float *disp, const uint8_t *mask, int W, int H, int nimg, float, double,
                           const sgm_road_fit *prior, double, sgm_road_fit *fit, void *ws, hipStream_t)
{
    touch_r(disp, (size_t)nimg * W * H * 4);
    if (mask) touch_r(mask, (size_t)nimg * W * H);
    if (prior) touch_r(prior, (size_t)nimg * sizeof(sgm_road_fit));
    touch_w(fit, (size_t)nimg * sizeof(sgm_road_fit));
    touch_w(ws, road_workspace_bytes(W, H, nimg));
    return hipSuccess;
}

hipError_t launch_road_window(const sgm_road_fit *fit, int, int H, int nimg, int, int, double, double, int32_t *d_lo,
                              hipStream_t)
{
    touch_r(fit, (size_t)nimg * sizeof(sgm_road_fit));
    touch_w(d_lo, (size_t)nimg * H * 4);
    return hipSuccess;
}

hipError_t launch_disp_transform(const float *disp, const sgm_road_fit *fit, int W, int H, int nimg, double,
                                 float *out, hipStream_t)
{
    touch_r(disp, (size_t)nimg * W * H * 4);
    touch_r(fit, (size_t)nimg * sizeof(sgm_road_fit));
    touch_w(out, (size_t)nimg * W * H * 4);
    return hipSuccess;
}

hipError_t launch_road_window_map(const sgm_road_fit *fit, int W, int H, int nimg, int, double, int32_t *lo,
                                  hipStream_t)
{
    touch_r(fit, (size_t)nimg * sizeof(sgm_road_fit));
    touch_w(lo, (size_t)nimg * W * H * 4);
    return hipSuccess;
}

hipError_t launch_road_mask(const float *disp, const sgm_road_fit *fit, int W, int H, int nimg, double, double,
                            uint8_t *mask, hipStream_t)
{
    touch_r(disp, (size_t)nimg * W * H * 4);
    touch_r(fit, (size_t)nimg * sizeof(sgm_road_fit));
    touch_w(mask, (size_t)nimg * W * H);
    return hipSuccess;
}

hipError_t launch_slic(const float *d2, const uint8_t *mask, int W, int H, int nimg, int S, double, int iters, double,
                       int32_t *rounds, int32_t *labels, float *d3, double *centres, void *ws, hipStream_t)
{
    CHECK(S >= 1 && iters >= 0 && iters <= kSlicMaxRounds);
    const size_t np = (size_t)nimg * W * H;
    touch_r(d2, np * 4);
    if (mask) touch_r(mask, np);
    if (rounds) touch_w(rounds, (size_t)nimg * 4);
    touch_w(labels, np * 4);
    if (d3) touch_w(d3, np * 4);
    touch_w(centres, (size_t)nimg * ((W + S - 1) / S) * ((H + S - 1) / S) * 3 * 8);
    touch_w(ws, slic_workspace_bytes(W, H, S, nimg));
    return hipSuccess;
}

hipError_t launch_pothole_threshold(const float *d2, const uint8_t *mask, int W, int H, int nimg, double, double,
                                    int nbins, double, sgm_pothole_threshold *out, double *curve, void *ws,
                                    hipStream_t)
{
    touch_r(d2, (size_t)nimg * W * H * 4);
    if (mask) touch_r(mask, (size_t)nimg * W * H);
    touch_w(out, (size_t)nimg * sizeof(sgm_pothole_threshold));
    if (curve) touch_w(curve, (size_t)nimg * nbins * 8);
    touch_w(ws, pothole_workspace_bytes(nbins, nimg));
    return hipSuccess;
}

hipError_t launch_pothole_prune(const int32_t *superpixels, int W, int H, int nimg, int32_t *labels, hipStream_t)
{
    touch_r(superpixels, (size_t)nimg * W * H * 4);
    touch_w(labels, (size_t)nimg * W * H * 4);
    return hipSuccess;
}

hipError_t launch_pothole_label(const float *d2, const uint8_t *mask, int W, int H, int nimg,
                                const sgm_pothole_threshold *thr, int32_t *labels, hipStream_t)
{
    touch_r(d2, (size_t)nimg * W * H * 4);
    if (mask) touch_r(mask, (size_t)nimg * W * H);
    touch_r(thr, (size_t)nimg * sizeof(sgm_pothole_threshold));
    touch_w(labels, (size_t)nimg * W * H * 4);
    return hipSuccess;
}

}  // namespace sgm
