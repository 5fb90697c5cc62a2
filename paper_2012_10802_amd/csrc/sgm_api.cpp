// C-ABI layer of the SGM library: plans, argument validation, workspace
// layout and the calls declared in include/sgm.h.  Every check happens on
// the host before anything is enqueued; kernels live in sgm_kernels.hip.

#include "../../include/sgm.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <cstdlib>
#include <new>

#include "sgm_internal.h"

struct sgm_plan_s {
    sgm_params params;
    sgm::Problem pb;
    sgm::KernelConfig kc;
    int paths[8];
    size_t n_pix, n_vol;      // W*H, W*H*w
    size_t off_codes_l, off_codes_r, off_cost, off_paths, ws_bytes;
};

namespace {

sgm_status fail(sgm_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(sgm::error_buffer(), sgm::kErrorBufferSize, fmt, ap);
    va_end(ap);
    return st;
}

sgm_status hip_fail(hipError_t e, const char *what)
{
    return fail(SGM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// One-shot fault injection (failure-handling tests): armed by
// sgm_debug_inject_fault() or, at first use, by the environment variable
// SGM_FAULT_INJECT=launch|alloc.  The next call that would launch (or
// allocate pinned memory) returns SGM_ERR_HIP instead, enqueueing nothing.
std::atomic<int> g_fault{-1};  // -1: environment not read yet

}  // namespace
namespace sgm {
bool fault_take(int kind)
{
    int cur = g_fault.load();
    if (cur < 0) {
        const char *e = getenv("SGM_FAULT_INJECT");
        const int k = !e ? 0 : (!strcmp(e, "launch") ? kFaultLaunch : (!strcmp(e, "alloc") ? kFaultAlloc : 0));
        int expected = -1;
        g_fault.compare_exchange_strong(expected, k);
        cur = g_fault.load();
    }
    if (cur != kind) return false;
    int expected = kind;
    return g_fault.compare_exchange_strong(expected, 0);
}
}  // namespace sgm
namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool is_aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

sgm_status check_plan(sgm_plan_t plan)
{
    if (!plan) return fail(SGM_ERR_INVALID, "plan is NULL");
    return SGM_OK;
}

sgm_status check_ws(const sgm_plan_s *p, void *ws, size_t bytes)
{
    if (!ws) return fail(SGM_ERR_INVALID, "workspace is NULL");
    if (!is_aligned(ws, 256)) return fail(SGM_ERR_INVALID, "workspace must be 256-byte aligned");
    if (bytes < p->ws_bytes)
        return fail(SGM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", bytes,
                    p->ws_bytes);
    return SGM_OK;
}

// Effective kernel configuration for given buffer pointers: vector access of
// a lane's values needs w % vpl == 0 and buffers aligned to a lane's bytes;
// misaligned buffers take the 16-lane mapping's element-wise form.
sgm::KernelConfig config_for(const sgm_plan_s *p, const void *a, const void *b)
{
    sgm::KernelConfig kc = p->kc;
    // widest access: a lane's values as uint16 (2*vpl bytes), issued as
    // power-of-two sized pieces
    const size_t bytes = (size_t)(kc.vpl > kc.wta_vpl ? kc.vpl : kc.wta_vpl) * 2;
    const size_t need = bytes & (~bytes + 1);
    if (kc.aligned && ((a && !is_aligned(a, need)) || (b && !is_aligned(b, need)))) {
        const sgm::Mapping m = sgm::choose_mapping(p->pb.w, 16);
        kc.lanes = kc.wta_lanes = m.lanes;
        kc.vpl = kc.wta_vpl = m.vpl;
        kc.aligned = false;
    }
    return kc;
}

sgm_status make_plan(const sgm_params *pr, int lanes, int order, sgm_plan_t *out);

}  // namespace

namespace sgm {
char *error_buffer()
{
    static thread_local char buf[kErrorBufferSize] = "";
    return buf;
}
}  // namespace sgm

extern "C" {

const char *sgm_status_str(sgm_status s)
{
    switch (s) {
    case SGM_OK: return "SGM_OK";
    case SGM_ERR_INVALID: return "SGM_ERR_INVALID";
    case SGM_ERR_UNSUPPORTED: return "SGM_ERR_UNSUPPORTED";
    case SGM_ERR_HIP: return "SGM_ERR_HIP";
    case SGM_ERR_WORKSPACE: return "SGM_ERR_WORKSPACE";
    }
    return "unknown sgm_status";
}

const char *sgm_last_error(void) { return sgm::error_buffer(); }

sgm_status sgm_plan(const sgm_params *pr, sgm_plan_t *out) { return make_plan(pr, 0, 0, out); }

sgm_status sgm_plan_tuned(const sgm_params *pr, const sgm_tuning *tuning, sgm_plan_t *out)
{
    if (!tuning) return fail(SGM_ERR_INVALID, "tuning is NULL");
    if (tuning->lanes != 0 && tuning->lanes != 4 && tuning->lanes != 8 && tuning->lanes != 16)
        return fail(SGM_ERR_INVALID, "lanes %d not in {0, 4, 8, 16}", tuning->lanes);
    if (tuning->order != 0 && tuning->order != 1)
        return fail(SGM_ERR_INVALID, "order %d not in {0, 1} for a plan", tuning->order);
    return make_plan(pr, tuning->lanes, tuning->order, out);
}

sgm_status sgm_plan_get_tuning(sgm_plan_t plan, sgm_tuning *tuning)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!tuning) return fail(SGM_ERR_INVALID, "tuning is NULL");
    *tuning = sgm_tuning{0, plan->kc.agg_order, plan->kc.lanes};
    return SGM_OK;
}

}  // extern "C"

namespace {

sgm_status make_plan(const sgm_params *pr, int lanes, int order, sgm_plan_t *out)
{
    if (!pr || !out) return fail(SGM_ERR_INVALID, "params and out must not be NULL");
    *out = nullptr;
    const sgm_params &q = *pr;
    if (q.width < 1 || q.height < 1) return fail(SGM_ERR_INVALID, "width and height must be >= 1");
    if (q.census != 3 && q.census != 5 && q.census != 7)
        return fail(SGM_ERR_UNSUPPORTED, "census window %d not in {3, 5, 7}", q.census);
    if (q.ndisp < 1 || q.ndisp > 256) return fail(SGM_ERR_INVALID, "ndisp %d not in [1, 256]", q.ndisp);
    if (q.npaths != 4 && q.npaths != 8) return fail(SGM_ERR_UNSUPPORTED, "npaths %d not in {4, 8}", q.npaths);
    if (q.p1 < 0 || q.p2 < q.p1) return fail(SGM_ERR_INVALID, "need 0 <= P1 <= P2 (got %d, %d)", q.p1, q.p2);
    const int cmax = q.census * q.census - 1;
    // window indices beyond w carry the cost 0x3FFF; they never win a
    // minimum while 2*Cmax + 3*P2 < 0x3FFF
    if (2 * cmax + 3 * q.p2 >= 0x3FFF)
        return fail(SGM_ERR_INVALID, "need 2*Cmax + 3*P2 < 16383 (Cmax %d, P2 %d)", cmax, q.p2);
    if ((long long)q.npaths * (cmax + q.p2) > 0xFFFF)
        return fail(SGM_ERR_INVALID, "summed cost would exceed 16 bits");
    if ((long long)q.width * q.height * q.ndisp >= (1ll << 31))
        return fail(SGM_ERR_UNSUPPORTED, "W*H*ndisp must be < 2^31");
    if (q.flags != 0) return fail(SGM_ERR_INVALID, "flags must be 0");

    sgm_plan_s *p = new (std::nothrow) sgm_plan_s();
    if (!p) return fail(SGM_ERR_INVALID, "out of host memory");
    p->params = q;
    p->pb = {q.width, q.height, q.ndisp, q.census, q.npaths, q.p1, q.p2, cmax};
    const sgm::Mapping mp = sgm::choose_mapping(q.ndisp, lanes);
    p->kc.lanes = mp.lanes;
    p->kc.vpl = mp.vpl;
    const sgm::Mapping ms = sgm::select_mapping(q.ndisp);
    p->kc.wta_lanes = ms.lanes;
    p->kc.wta_vpl = ms.vpl;
    // (narrower mappings exist only for widths that are a multiple of vpl)
    p->kc.aligned = (q.ndisp % sgm::choose_mapping(q.ndisp, 16).vpl) == 0;
    p->kc.l8 = cmax + q.p2 <= 255;
    if (!p->kc.l8 && (long long)q.width * q.height * q.ndisp >= sgm::kMaxU16Volume) {
        delete p;
        return fail(SGM_ERR_UNSUPPORTED,
                    "uint16 per-path volumes (Cmax + P2 > 255) need W*H*ndisp < 2^30 (got %lld)",
                    (long long)q.width * q.height * q.ndisp);
    }
    p->kc.agg_block = 256;
    p->kc.agg_order = order;
    for (int i = 0; i < 8; ++i) p->paths[i] = i;
    p->n_pix = (size_t)q.width * q.height;
    p->n_vol = p->n_pix * (size_t)q.ndisp;
    const size_t esz = p->kc.l8 ? 1 : 2;
    const size_t vstride = align256(p->n_vol * esz);
    size_t off = 0;
    p->off_codes_l = off;
    off += align256(p->n_pix * 8);
    p->off_codes_r = off;
    off += align256(p->n_pix * 8);
    p->off_cost = off;
    off += align256(p->n_vol);
    p->off_paths = off;
    off += vstride * (size_t)q.npaths;
    p->ws_bytes = off;
    *out = p;
    return SGM_OK;
}

}  // namespace

extern "C" {

void sgm_plan_free(sgm_plan_t plan) { delete plan; }

sgm_status sgm_workspace_size(sgm_plan_t plan, size_t *bytes)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!bytes) return fail(SGM_ERR_INVALID, "bytes is NULL");
    *bytes = plan->ws_bytes;
    return SGM_OK;
}

sgm_status sgm_census(sgm_plan_t plan, const uint8_t *image, int32_t pitch, uint64_t *codes, void *stream)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!image || !codes) return fail(SGM_ERR_INVALID, "image and codes must not be NULL");
    if (pitch < plan->pb.W) return fail(SGM_ERR_INVALID, "pitch %d < width %d", pitch, plan->pb.W);
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_census(plan->pb, image, pitch, codes, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "census launch");
}

sgm_status sgm_cost(sgm_plan_t plan, const uint8_t *left, const uint8_t *right, int32_t pitch, const int32_t *d_lo,
                    uint8_t *cost, void *ws, size_t ws_bytes, void *stream)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!left || !right || !cost) return fail(SGM_ERR_INVALID, "left, right and cost must not be NULL");
    if (pitch < plan->pb.W) return fail(SGM_ERR_INVALID, "pitch %d < width %d", pitch, plan->pb.W);
    if (sgm_status s = check_ws(plan, ws, ws_bytes)) return s;
    uint8_t *base = static_cast<uint8_t *>(ws);
    uint64_t *cl = reinterpret_cast<uint64_t *>(base + plan->off_codes_l);
    uint64_t *cr = reinterpret_cast<uint64_t *>(base + plan->off_codes_r);
    hipStream_t st = (hipStream_t)stream;
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_census_lr(plan->pb, left, right, pitch, cl, cr, st);
    if (e == hipSuccess) e = sgm::launch_cost(plan->pb, config_for(plan, cost, nullptr), cl, cr, d_lo, cost, st);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "cost launch");
}

sgm_status sgm_aggregate(sgm_plan_t plan, const uint8_t *cost, uint16_t *sum, void *ws, size_t ws_bytes,
                         void *stream)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!cost || !sum) return fail(SGM_ERR_INVALID, "cost and sum must not be NULL");
    if (sgm_status s = check_ws(plan, ws, ws_bytes)) return s;
    void *vols = static_cast<uint8_t *>(ws) + plan->off_paths;
    hipStream_t st = (hipStream_t)stream;
    const sgm::KernelConfig kc = config_for(plan, cost, nullptr);
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_aggregate(plan->pb, kc, cost, plan->paths, plan->pb.npaths, kc.l8, vols, st);
    if (e == hipSuccess) e = sgm::launch_sum(plan->pb, kc, vols, plan->pb.npaths, kc.l8, sum, st);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "aggregate launch");
}

sgm_status sgm_aggregate_path(sgm_plan_t plan, const uint8_t *cost, int32_t path, uint16_t *L, void *stream)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!cost || !L) return fail(SGM_ERR_INVALID, "cost and L must not be NULL");
    if (path < 0 || path > 7) return fail(SGM_ERR_INVALID, "path %d not in [0, 7]", path);
    if ((long long)plan->n_vol >= sgm::kMaxU16Volume)
        return fail(SGM_ERR_UNSUPPORTED, "sgm_aggregate_path writes uint16: W*H*ndisp must be < 2^30");
    const sgm::KernelConfig kc = config_for(plan, cost, L);
    const int paths[1] = {path};
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_aggregate(plan->pb, kc, cost, paths, 1, false, L, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "aggregate_path launch");
}

sgm_status sgm_wta(sgm_plan_t plan, const uint16_t *sum, const int32_t *d_lo, uint16_t *disp_int, float *disp_sub,
                   void *stream)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!sum || !disp_int) return fail(SGM_ERR_INVALID, "sum and disp_int must not be NULL");
    const sgm::KernelConfig kc = config_for(plan, sum, nullptr);
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_wta_sum(plan->pb, kc, sum, d_lo, disp_int, disp_sub, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "wta launch");
}

sgm_status sgm_aggregate_wta(sgm_plan_t plan, const uint8_t *cost, const int32_t *d_lo, uint16_t *disp_int,
                             float *disp_sub, void *ws, size_t ws_bytes, void *stream)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!cost || !disp_int) return fail(SGM_ERR_INVALID, "cost and disp_int must not be NULL");
    if (sgm_status s = check_ws(plan, ws, ws_bytes)) return s;
    void *vols = static_cast<uint8_t *>(ws) + plan->off_paths;
    hipStream_t st = (hipStream_t)stream;
    const sgm::KernelConfig kc = config_for(plan, cost, nullptr);
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_aggregate(plan->pb, kc, cost, plan->paths, plan->pb.npaths, kc.l8, vols, st);
    if (e == hipSuccess)
        e = sgm::launch_wta_paths(plan->pb, kc, vols, plan->pb.npaths, kc.l8, d_lo, disp_int, disp_sub, st);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "aggregate_wta launch");
}

sgm_status sgm_path_volumes(sgm_plan_t plan, int32_t *elem_bytes, size_t *volume_stride, size_t *total_bytes)
{
    if (sgm_status s = check_plan(plan)) return s;
    const size_t esz = plan->kc.l8 ? 1 : 2;
    const size_t vs = align256(plan->n_vol * esz);
    if (elem_bytes) *elem_bytes = (int32_t)esz;
    if (volume_stride) *volume_stride = vs;
    if (total_bytes) *total_bytes = vs * (size_t)plan->pb.npaths;
    return SGM_OK;
}

sgm_status sgm_aggregate_paths(sgm_plan_t plan, const uint8_t *cost, void *paths, size_t paths_bytes, void *stream)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!cost || !paths) return fail(SGM_ERR_INVALID, "cost and paths must not be NULL");
    if (!is_aligned(paths, 256)) return fail(SGM_ERR_INVALID, "paths must be 256-byte aligned");
    size_t total = 0;
    sgm_path_volumes(plan, nullptr, nullptr, &total);
    if (paths_bytes < total)
        return fail(SGM_ERR_WORKSPACE, "paths buffer of %zu bytes is smaller than the %zu required", paths_bytes,
                    total);
    const sgm::KernelConfig kc = config_for(plan, cost, nullptr);
    hipError_t e =
        sgm::launch_aggregate(plan->pb, kc, cost, plan->paths, plan->pb.npaths, kc.l8, paths, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "aggregate_paths launch");
}

sgm_status sgm_wta_paths(sgm_plan_t plan, const void *paths, const int32_t *d_lo, uint16_t *disp_int,
                         float *disp_sub, void *stream)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!paths || !disp_int) return fail(SGM_ERR_INVALID, "paths and disp_int must not be NULL");
    if (!is_aligned(paths, 256)) return fail(SGM_ERR_INVALID, "paths must be 256-byte aligned");
    const sgm::KernelConfig kc = config_for(plan, nullptr, nullptr);
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_wta_paths(plan->pb, kc, paths, plan->pb.npaths, kc.l8, d_lo, disp_int, disp_sub,
                                         (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "wta_paths launch");
}

sgm_status sgm_match(sgm_plan_t plan, const uint8_t *left, const uint8_t *right, int32_t pitch, const int32_t *d_lo,
                     uint16_t *disp_int, float *disp_sub, void *ws, size_t ws_bytes, void *stream)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!disp_int) return fail(SGM_ERR_INVALID, "disp_int must not be NULL");
    if (sgm_status s = check_ws(plan, ws, ws_bytes)) return s;
    uint8_t *cost = static_cast<uint8_t *>(ws) + plan->off_cost;
    if (sgm_status s = sgm_cost(plan, left, right, pitch, d_lo, cost, ws, ws_bytes, stream)) return s;
    return sgm_aggregate_wta(plan, cost, d_lo, disp_int, disp_sub, ws, ws_bytes, stream);
}

sgm_status sgm_autotune(const sgm_params *params, const uint8_t *left, const uint8_t *right, int32_t pitch,
                        const int32_t *d_lo, uint16_t *disp_int, float *disp_sub, void *ws, size_t ws_bytes,
                        void *stream, const char *cache_path, sgm_tuning *chosen)
{
    if (!params) return fail(SGM_ERR_INVALID, "params is NULL");
    sgm_plan_t base = nullptr;
    if (sgm_status s = make_plan(params, 0, 0, &base)) return s;
    const sgm_params q = base->params;
    const int deflt = base->kc.lanes;
    sgm_plan_free(base);
    // cache key: device architecture and the problem's shape and parameters
    // (h16: horizontal directions on 16 lanes, so entries timed with another
    // schedule are not reused)
    char key[256];
    {
        int dev = 0;
        hipDeviceProp_t prop;
        char arch[64] = "unknown";
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
        for (char *c = arch; *c; ++c)
            if (*c == ' ' || *c == ':') *c = '_';
        snprintf(key, sizeof key, "single|h16|%s|%dx%dx%d|n%d|R%d|P%d,%d", arch, q.width, q.height, q.ndisp, q.census,
                 q.npaths, q.p1, q.p2);
    }
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "r")) {
            char line[512], k[300];
            int lanes = -1, order = -1, found = -1, found_order = 0;
            double ms = 0;
            while (fgets(line, sizeof line, f))
                if (sscanf(line, "%299s %d %d %lf", k, &lanes, &order, &ms) == 4 && !strcmp(k, key) &&
                    (lanes == 4 || lanes == 8 || lanes == 16) && (order == 0 || order == 1)) {
                    found = lanes;
                    found_order = order;
                }
            fclose(f);
            if (found > 0) {
                if (chosen) *chosen = sgm_tuning{0, found_order, found};
                return SGM_OK;
            }
        }
    }
    // time each distinct (lane mapping, slot order): one warm-up run, then
    // the best of three
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return fail(SGM_ERR_HIP, "autotune: event creation failed");
    }
    int best = deflt, best_order = 0, seen[6] = {0, 0, 0, 0, 0, 0}, nseen = 0;
    float best_ms = 1e30f;
    sgm_status rs = SGM_OK;
    static const int kTrials[6][2] = {{16, 0}, {16, 1}, {8, 0}, {8, 1}, {4, 0}, {4, 1}};  // (lanes, order)
    for (const auto &trial : kTrials) {
        sgm_plan_t p = nullptr;
        if ((rs = make_plan(params, trial[0], trial[1], &p)) != SGM_OK) break;
        const int eff = p->kc.lanes, key2 = eff * 2 + trial[1];
        bool dup = false;
        for (int i = 0; i < nseen; ++i) dup = dup || seen[i] == key2;
        if (dup) {
            sgm_plan_free(p);
            continue;
        }
        seen[nseen++] = key2;
        float ms = 1e30f;
        for (int rep = 0; rep < 4 && rs == SGM_OK; ++rep) {
            if (hipEventRecord(e0, st) != hipSuccess) rs = fail(SGM_ERR_HIP, "autotune: event record failed");
            if (rs == SGM_OK) rs = sgm_match(p, left, right, pitch, d_lo, disp_int, disp_sub, ws, ws_bytes, stream);
            if (rs == SGM_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                rs = fail(SGM_ERR_HIP, "autotune: event wait failed");
            float t = 0;
            if (rs == SGM_OK && rep > 0 && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms = t < ms ? t : ms;
        }
        sgm_plan_free(p);
        if (rs != SGM_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            best = eff;
            best_order = trial[1];
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rs != SGM_OK) return rs;
    if (cache_path)
        if (FILE *f = fopen(cache_path, "a")) {
            fprintf(f, "%s %d %d %.5f\n", key, best, best_order, best_ms);
            fclose(f);
        }
    if (chosen) *chosen = sgm_tuning{0, best_order, best};
    return SGM_OK;
}

// ---------------------------------------------------------------------------
// per-pixel windows

namespace {

sgm_status check_win_plan(sgm_plan_t plan)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (plan->pb.w > 16) return fail(SGM_ERR_UNSUPPORTED, "per-pixel windows need ndisp <= 16 (got %d)", plan->pb.w);
    return SGM_OK;
}

}  // namespace

sgm_status sgm_downsample4(const uint8_t *img, int32_t width, int32_t height, int32_t pitch, uint8_t *out,
                           void *stream)
{
    if (!img || !out) return fail(SGM_ERR_INVALID, "img and out must not be NULL");
    if (width < 4 || height < 4 || pitch < width) return fail(SGM_ERR_INVALID, "need width, height >= 4, pitch >= width");
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_downsample4(img, width, height, pitch, 0, 1, out, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "downsample launch");
}

sgm_status sgm_downsample4_batch(const uint8_t *images, int32_t width, int32_t height, int32_t pitch,
                                 int64_t image_stride, int32_t nimg, uint8_t *out, void *stream)
{
    if (!images || !out) return fail(SGM_ERR_INVALID, "images and out must not be NULL");
    if (width < 4 || height < 4 || pitch < width) return fail(SGM_ERR_INVALID, "need width, height >= 4, pitch >= width");
    if (nimg < 1 || nimg > 65535) return fail(SGM_ERR_INVALID, "nimg must be in [1, 65535]");
    if (image_stride < (int64_t)pitch * height) return fail(SGM_ERR_INVALID, "image_stride < pitch * height");
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_downsample4(images, width, height, pitch, (long long)image_stride, nimg, out,
                                           (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "downsample4 launch");
}

sgm_status sgm_cost_win(sgm_plan_t plan, const uint8_t *left, const uint8_t *right, int32_t pitch, const int32_t *lo,
                        uint8_t *cost, void *ws, size_t ws_bytes, void *stream)
{
    if (sgm_status s = check_win_plan(plan)) return s;
    if (!left || !right || !lo || !cost) return fail(SGM_ERR_INVALID, "left, right, lo and cost must not be NULL");
    if (pitch < plan->pb.W) return fail(SGM_ERR_INVALID, "pitch %d < width %d", pitch, plan->pb.W);
    if (!is_aligned(cost, 16)) return fail(SGM_ERR_INVALID, "cost must be 16-byte aligned");
    if (sgm_status s = check_ws(plan, ws, ws_bytes)) return s;
    uint8_t *base = static_cast<uint8_t *>(ws);
    uint64_t *cl = reinterpret_cast<uint64_t *>(base + plan->off_codes_l);
    uint64_t *cr = reinterpret_cast<uint64_t *>(base + plan->off_codes_r);
    hipStream_t st = (hipStream_t)stream;
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_census_lr(plan->pb, left, right, pitch, cl, cr, st);
    if (e == hipSuccess) e = sgm::launch_cost_win(plan->pb, cl, cr, lo, cost, st);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "cost_win launch");
}

sgm_status sgm_aggregate_win_paths(sgm_plan_t plan, const uint8_t *cost, const int32_t *lo, void *paths,
                                   size_t paths_bytes, void *stream)
{
    if (sgm_status s = check_win_plan(plan)) return s;
    if (!cost || !lo || !paths) return fail(SGM_ERR_INVALID, "cost, lo and paths must not be NULL");
    if (!is_aligned(paths, 256)) return fail(SGM_ERR_INVALID, "paths must be 256-byte aligned");
    size_t total = 0, vs = 0;
    sgm_path_volumes(plan, nullptr, &vs, &total);
    if (paths_bytes < total)
        return fail(SGM_ERR_WORKSPACE, "paths buffer of %zu bytes is smaller than the %zu required", paths_bytes,
                    total);
    const long long vstride = (long long)(vs / (plan->kc.l8 ? 1 : 2));
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_aggregate_win(plan->pb, cost, lo, plan->paths, plan->pb.npaths, plan->kc.l8, paths,
                                             vstride, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "aggregate_win launch");
}

sgm_status sgm_wta_win_paths(sgm_plan_t plan, const void *paths, const int32_t *lo, uint16_t *disp_int,
                             float *disp_sub, void *stream)
{
    if (sgm_status s = check_win_plan(plan)) return s;
    if (!paths || !lo || !disp_int) return fail(SGM_ERR_INVALID, "paths, lo and disp_int must not be NULL");
    if (!is_aligned(paths, 256)) return fail(SGM_ERR_INVALID, "paths must be 256-byte aligned");
    size_t vs = 0;
    sgm_path_volumes(plan, nullptr, &vs, nullptr);
    const long long vstride = (long long)(vs / (plan->kc.l8 ? 1 : 2));
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_wta_win(plan->pb, paths, vstride, plan->pb.npaths, plan->kc.l8, lo, disp_int,
                                       disp_sub, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "wta_win launch");
}

sgm_status sgm_match_win(sgm_plan_t plan, const uint8_t *left, const uint8_t *right, int32_t pitch, const int32_t *lo,
                         uint16_t *disp_int, float *disp_sub, void *ws, size_t ws_bytes, void *stream)
{
    if (sgm_status s = check_win_plan(plan)) return s;
    if (sgm_status s = check_ws(plan, ws, ws_bytes)) return s;
    uint8_t *base = static_cast<uint8_t *>(ws);
    if (sgm_status s = sgm_cost_win(plan, left, right, pitch, lo, base + plan->off_cost, ws, ws_bytes, stream))
        return s;
    size_t total = 0;
    sgm_path_volumes(plan, nullptr, nullptr, &total);
    if (sgm_status s = sgm_aggregate_win_paths(plan, base + plan->off_cost, lo, base + plan->off_paths, total, stream))
        return s;
    return sgm_wta_win_paths(plan, base + plan->off_paths, lo, disp_int, disp_sub, stream);
}

}  // extern "C"

namespace {
// workspace slice of one pair in a windowed batch: the plan's workspace,
// then the window starts as bytes
size_t win_pair_bytes(const sgm_plan_s *p) { return p->ws_bytes + align256(p->n_pix); }
}  // namespace

extern "C" {

sgm_status sgm_workspace_size_win_batch(sgm_plan_t plan, int32_t nimg, size_t *bytes)
{
    if (sgm_status s = check_plan(plan)) return s;
    if (!bytes) return fail(SGM_ERR_INVALID, "bytes is NULL");
    if (nimg < 1) return fail(SGM_ERR_INVALID, "nimg must be >= 1 (got %d)", nimg);
    *bytes = win_pair_bytes(plan) * (size_t)nimg;
    return SGM_OK;
}

sgm_status sgm_match_win_batch(sgm_plan_t plan, const uint8_t *left, const uint8_t *right, int32_t pitch,
                               int64_t image_stride, const int32_t *lo, int32_t nimg, uint16_t *disp_int,
                               float *disp_sub, void *ws, size_t ws_bytes, void *stream)
{
    if (sgm_status s = check_win_plan(plan)) return s;
    if (plan->pb.w != 16 || !plan->kc.l8)
        return fail(SGM_ERR_UNSUPPORTED, "batched windows need ndisp = 16 and Cmax + P2 <= 255");
    if (!left || !right || !lo || !disp_int || !ws)
        return fail(SGM_ERR_INVALID, "left, right, lo, disp_int and workspace must not be NULL");
    if (nimg < 1) return fail(SGM_ERR_INVALID, "nimg must be >= 1 (got %d)", nimg);
    if (pitch < plan->pb.W) return fail(SGM_ERR_INVALID, "pitch %d < width %d", pitch, plan->pb.W);
    if (image_stride < (int64_t)pitch * plan->pb.H)
        return fail(SGM_ERR_INVALID, "image_stride %lld < pitch * height", (long long)image_stride);
    if (!is_aligned(ws, 256)) return fail(SGM_ERR_INVALID, "workspace must be 256-byte aligned");
    const size_t pair_bytes = win_pair_bytes(plan);
    if (ws_bytes / (size_t)nimg < pair_bytes)
        return fail(SGM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                    pair_bytes * (size_t)nimg);
    uint8_t *base = static_cast<uint8_t *>(ws);
    size_t vs = 0;
    sgm_path_volumes(plan, nullptr, &vs, nullptr);
    sgm::WinPairs b{};
    b.left = left;
    b.right = right;
    b.pitch = pitch;
    b.img_pair = (long long)image_stride;
    b.lo = lo;
    b.npairs = nimg;
    b.ws_pair = pair_bytes;
    b.lo8 = base + plan->ws_bytes;
    b.codes_l = reinterpret_cast<uint64_t *>(base + plan->off_codes_l);
    b.codes_r = reinterpret_cast<uint64_t *>(base + plan->off_codes_r);
    b.cost = base + plan->off_cost;
    b.paths = base + plan->off_paths;
    b.vstride = (long long)vs;
    b.dint = disp_int;
    b.dsub = disp_sub;
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_match_win_pairs(plan->pb, b, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "match_win_batch launch");
}

sgm_status sgm_debug_inject_fault(int32_t kind)
{
    if (kind < 0 || kind > 2) return fail(SGM_ERR_INVALID, "fault kind %d not in {0, 1, 2}", kind);
    g_fault.store(kind);
    return SGM_OK;
}

static sgm_status check_maps(int32_t W, int32_t H, int32_t nimg)
{
    if (W < 1 || H < 1 || nimg < 1) return fail(SGM_ERR_INVALID, "width, height and nimg must be >= 1");
    if (nimg > 65535) return fail(SGM_ERR_UNSUPPORTED, "nimg %d > 65535", nimg);
    if ((long long)W * H > (1LL << 30)) return fail(SGM_ERR_UNSUPPORTED, "W*H must be <= 2^30");
    return SGM_OK;
}

sgm_status sgm_road_workspace_size(int32_t W, int32_t H, int32_t nimg, size_t *bytes)
{
    if (!bytes) return fail(SGM_ERR_INVALID, "bytes is NULL");
    sgm_status st = check_maps(W, H, nimg);
    if (st != SGM_OK) return st;
    *bytes = sgm::road_workspace_bytes(W, H, nimg);
    return SGM_OK;
}

sgm_status sgm_road_fit_batch(const float *disp, const uint8_t *mask, int32_t W, int32_t H, int32_t nimg,
                              float min_disp, double margin, const sgm_road_fit *prior, double tol,
                              sgm_road_fit *fit, void *ws, size_t ws_bytes, void *stream)
{
    if (!disp || !fit) return fail(SGM_ERR_INVALID, "disp and fit must not be NULL");
    sgm_status st = check_maps(W, H, nimg);
    if (st != SGM_OK) return st;
    if (isnan(min_disp) || isnan(margin)) return fail(SGM_ERR_INVALID, "min_disp and margin must not be NaN");
    if (!(tol >= 0.0)) return fail(SGM_ERR_INVALID, "tol must be >= 0 (or +INFINITY)");
    if (prior && !is_aligned(prior, 8)) return fail(SGM_ERR_INVALID, "prior misaligned");
    if (!ws) return fail(SGM_ERR_INVALID, "workspace is NULL");
    if (!is_aligned(ws, 256)) return fail(SGM_ERR_INVALID, "workspace must be 256-byte aligned");
    if (!is_aligned(disp, 4) || !is_aligned(fit, 8)) return fail(SGM_ERR_INVALID, "disp or fit misaligned");
    const size_t need = sgm::road_workspace_bytes(W, H, nimg);
    if (ws_bytes < need)
        return fail(SGM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_road_fit(disp, mask, W, H, nimg, min_disp, margin, prior, tol, fit, ws,
                                           (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "road fit launch");
}

sgm_status sgm_road_energy_batch(const float *disp, const uint8_t *mask, int32_t W, int32_t H, int32_t nimg,
                                 float min_disp, double margin, const sgm_road_fit *prior, double tol,
                                 const double *phi, int32_t nphi, double *energy, void *ws, size_t ws_bytes,
                                 void *stream)
{
    if (!disp || !phi || !energy) return fail(SGM_ERR_INVALID, "disp, phi and energy must not be NULL");
    sgm_status st = check_maps(W, H, nimg);
    if (st != SGM_OK) return st;
    if (nphi < 1 || nphi > 65536) return fail(SGM_ERR_INVALID, "nphi %d not in [1, 65536]", nphi);
    if (isnan(min_disp) || isnan(margin)) return fail(SGM_ERR_INVALID, "min_disp and margin must not be NaN");
    if (!(tol >= 0.0)) return fail(SGM_ERR_INVALID, "tol must be >= 0 (or +INFINITY)");
    if (prior && !is_aligned(prior, 8)) return fail(SGM_ERR_INVALID, "prior misaligned");
    if (!ws) return fail(SGM_ERR_INVALID, "workspace is NULL");
    if (!is_aligned(ws, 256)) return fail(SGM_ERR_INVALID, "workspace must be 256-byte aligned");
    if (!is_aligned(disp, 4) || !is_aligned(phi, 8) || !is_aligned(energy, 8))
        return fail(SGM_ERR_INVALID, "disp, phi or energy misaligned");
    const size_t need = sgm::road_workspace_bytes(W, H, nimg);
    if (ws_bytes < need)
        return fail(SGM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_road_energy(disp, mask, W, H, nimg, min_disp, margin, prior, tol, phi, nphi, energy,
                                           ws, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "road energy launch");
}

sgm_status sgm_road_window_batch(const sgm_road_fit *fit, int32_t W, int32_t H, int32_t nimg, int32_t w,
                                 int32_t mode, double delta, double scale, int32_t *d_lo, void *stream)
{
    if (!fit || !d_lo) return fail(SGM_ERR_INVALID, "fit and d_lo must not be NULL");
    sgm_status st = check_maps(W, H, nimg);
    if (st != SGM_OK) return st;
    if (w < 1) return fail(SGM_ERR_INVALID, "w must be >= 1");
    if (mode != 0 && mode != 1) return fail(SGM_ERR_INVALID, "mode %d not in {0, 1}", mode);
    if (!isfinite(delta)) return fail(SGM_ERR_INVALID, "delta must be finite");
    if (!(scale > 0.0) || !isfinite(scale)) return fail(SGM_ERR_INVALID, "scale must be finite and > 0");
    if (!is_aligned(fit, 8) || !is_aligned(d_lo, 4)) return fail(SGM_ERR_INVALID, "fit or d_lo misaligned");
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_road_window(fit, W, H, nimg, w, mode, delta, scale, d_lo, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "road window launch");
}

sgm_status sgm_disparity_transform_batch(const float *disp, const sgm_road_fit *fit, int32_t W, int32_t H,
                                         int32_t nimg, double delta_dt, float *out, void *stream)
{
    if (!disp || !fit || !out) return fail(SGM_ERR_INVALID, "disp, fit and out must not be NULL");
    sgm_status st = check_maps(W, H, nimg);
    if (st != SGM_OK) return st;
    if (!isfinite(delta_dt)) return fail(SGM_ERR_INVALID, "delta_dt must be finite");
    if (!is_aligned(disp, 4) || !is_aligned(out, 4) || !is_aligned(fit, 8))
        return fail(SGM_ERR_INVALID, "disp, out or fit misaligned");
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_disp_transform(disp, fit, W, H, nimg, delta_dt, out, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "disparity transform launch");
}

sgm_status sgm_pothole_workspace_size(int32_t nbins, int32_t nimg, size_t *bytes)
{
    if (!bytes) return fail(SGM_ERR_INVALID, "bytes is NULL");
    if (nbins < 2 || nbins > 512) return fail(SGM_ERR_INVALID, "nbins %d not in [2, 512]", nbins);
    if (nimg < 1 || nimg > 65535) return fail(SGM_ERR_INVALID, "nimg %d not in [1, 65535]", nimg);
    *bytes = sgm::pothole_workspace_bytes(nbins, nimg);
    return SGM_OK;
}

sgm_status sgm_pothole_threshold_batch(const float *d2, const uint8_t *mask, int32_t W, int32_t H, int32_t nimg,
                                       double lo, double hi, int32_t nbins, double delta_pd,
                                       sgm_pothole_threshold *result, double *e2_curve, void *ws, size_t ws_bytes,
                                       void *stream)
{
    if (!d2 || !result) return fail(SGM_ERR_INVALID, "d2 and result must not be NULL");
    sgm_status st = check_maps(W, H, nimg);
    if (st != SGM_OK) return st;
    if (nbins < 2 || nbins > 512) return fail(SGM_ERR_INVALID, "nbins %d not in [2, 512]", nbins);
    if (!isfinite(lo) || !isfinite(hi) || !(lo < hi)) return fail(SGM_ERR_INVALID, "need finite lo < hi");
    if (!isfinite(delta_pd)) return fail(SGM_ERR_INVALID, "delta_pd must be finite");
    const double b = (hi - lo) / nbins;
    if (!(b > 0.0) || !isfinite(8.0 * b) || !isfinite(8.0 * lo))
        return fail(SGM_ERR_INVALID, "bin width out of range");
    if (!ws) return fail(SGM_ERR_INVALID, "workspace is NULL");
    if (!is_aligned(ws, 256)) return fail(SGM_ERR_INVALID, "workspace must be 256-byte aligned");
    if (!is_aligned(d2, 4) || !is_aligned(result, 8) || !is_aligned(e2_curve, 8))
        return fail(SGM_ERR_INVALID, "d2, result or e2_curve misaligned");
    const size_t need = sgm::pothole_workspace_bytes(nbins, nimg);
    if (ws_bytes < need)
        return fail(SGM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_pothole_threshold(d2, mask, W, H, nimg, lo, b, nbins, delta_pd, result, e2_curve, ws,
                                                 (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "pothole threshold launch");
}

sgm_status sgm_pothole_label_batch(const float *d2, const uint8_t *mask, int32_t W, int32_t H, int32_t nimg,
                                   const sgm_pothole_threshold *result, int32_t *labels, void *stream)
{
    if (!d2 || !result || !labels) return fail(SGM_ERR_INVALID, "d2, result and labels must not be NULL");
    sgm_status st = check_maps(W, H, nimg);
    if (st != SGM_OK) return st;
    if (!is_aligned(d2, 4) || !is_aligned(result, 8) || !is_aligned(labels, 4))
        return fail(SGM_ERR_INVALID, "d2, result or labels misaligned");
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_pothole_label(d2, mask, W, H, nimg, result, labels, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "pothole label launch");
}

sgm_status sgm_pothole_prune_batch(const int32_t *superpixels, int32_t W, int32_t H, int32_t nimg, int32_t *labels,
                                   void *stream)
{
    if (!superpixels || !labels) return fail(SGM_ERR_INVALID, "superpixels and labels must not be NULL");
    sgm_status st = check_maps(W, H, nimg);
    if (st != SGM_OK) return st;
    if (!is_aligned(superpixels, 4) || !is_aligned(labels, 4))
        return fail(SGM_ERR_INVALID, "superpixels or labels misaligned");
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_pothole_prune(superpixels, W, H, nimg, labels, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "pothole prune launch");
}

sgm_status sgm_road_window_map_batch(const sgm_road_fit *fit, int32_t W, int32_t H, int32_t nimg, int32_t w,
                                     double scale, int32_t *lo, void *stream)
{
    if (!fit || !lo) return fail(SGM_ERR_INVALID, "fit and lo must not be NULL");
    sgm_status st = check_maps(W, H, nimg);
    if (st != SGM_OK) return st;
    if (w < 1) return fail(SGM_ERR_INVALID, "w must be >= 1");
    if (!(scale > 0.0) || !isfinite(scale)) return fail(SGM_ERR_INVALID, "scale must be finite and > 0");
    if (!is_aligned(fit, 8) || !is_aligned(lo, 4)) return fail(SGM_ERR_INVALID, "fit or lo misaligned");
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_road_window_map(fit, W, H, nimg, w, scale, lo, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "road window map launch");
}

sgm_status sgm_road_mask_batch(const float *disp, const sgm_road_fit *fit, int32_t W, int32_t H, int32_t nimg,
                               double f_min, double margin, uint8_t *mask, void *stream)
{
    if (!disp || !fit || !mask) return fail(SGM_ERR_INVALID, "disp, fit and mask must not be NULL");
    sgm_status st = check_maps(W, H, nimg);
    if (st != SGM_OK) return st;
    if (isnan(f_min) || isnan(margin)) return fail(SGM_ERR_INVALID, "f_min and margin must not be NaN");
    if (!is_aligned(disp, 4) || !is_aligned(fit, 8)) return fail(SGM_ERR_INVALID, "disp or fit misaligned");
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_road_mask(disp, fit, W, H, nimg, f_min, margin, mask, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "road mask launch");
}

static sgm_status check_slic(int32_t W, int32_t H, int32_t S, int32_t nimg)
{
    sgm_status st = check_maps(W, H, nimg);
    if (st != SGM_OK) return st;
    if (S < 2 || S > 256) return fail(SGM_ERR_INVALID, "S %d not in [2, 256]", S);
    if ((H + S - 1) / S > 65535) return fail(SGM_ERR_UNSUPPORTED, "more than 65535 rows of grid cells");
    return SGM_OK;
}

sgm_status sgm_slic_workspace_size(int32_t W, int32_t H, int32_t S, int32_t nimg, size_t *bytes)
{
    if (!bytes) return fail(SGM_ERR_INVALID, "bytes is NULL");
    sgm_status st = check_slic(W, H, S, nimg);
    if (st != SGM_OK) return st;
    *bytes = sgm::slic_workspace_bytes(W, H, S, nimg);
    return SGM_OK;
}

sgm_status sgm_slic_batch(const float *d2, const uint8_t *mask, int32_t W, int32_t H, int32_t nimg, int32_t S,
                          double m, int32_t iters, double tol, int32_t *rounds, int32_t *labels, float *d3,
                          double *centres, void *ws, size_t ws_bytes, void *stream)
{
    if (!d2 || !labels || !d3 || !centres) return fail(SGM_ERR_INVALID, "d2, labels, d3 and centres must not be NULL");
    sgm_status st = check_slic(W, H, S, nimg);
    if (st != SGM_OK) return st;
    if (!isfinite(m) || m < 0.0) return fail(SGM_ERR_INVALID, "m must be finite and >= 0");
    if (iters < 1 || iters > sgm::kSlicMaxRounds)
        return fail(SGM_ERR_INVALID, "iters %d not in [1, %d]", iters, sgm::kSlicMaxRounds);
    if (!(tol >= 0.0) || !isfinite(tol)) return fail(SGM_ERR_INVALID, "tol must be finite and >= 0");
    if (rounds && !is_aligned(rounds, 4)) return fail(SGM_ERR_INVALID, "rounds misaligned");
    if (!ws) return fail(SGM_ERR_INVALID, "workspace is NULL");
    if (!is_aligned(ws, 256)) return fail(SGM_ERR_INVALID, "workspace must be 256-byte aligned");
    if (!is_aligned(d2, 4) || !is_aligned(labels, 4) || !is_aligned(d3, 4) || !is_aligned(centres, 8))
        return fail(SGM_ERR_INVALID, "d2, labels, d3 or centres misaligned");
    const size_t need = sgm::slic_workspace_bytes(W, H, S, nimg);
    if (ws_bytes < need)
        return fail(SGM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    if (sgm::fault_take(sgm::kFaultLaunch)) return fail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = sgm::launch_slic(d2, mask, W, H, nimg, S, m, iters, tol, rounds, labels, d3, centres, ws,
                                    (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "slic launch");
}

sgm_status sgm_window_from_road(double a0, double a1, double phi, int32_t W, int32_t H, int32_t w, int32_t mode,
                                double delta, int32_t *d_lo)
{
    if (!d_lo) return fail(SGM_ERR_INVALID, "d_lo_host is NULL");
    if (W < 1 || H < 1 || w < 1) return fail(SGM_ERR_INVALID, "sizes must be >= 1");
    if (mode != 0 && mode != 1) return fail(SGM_ERR_INVALID, "mode %d not in {0, 1}", mode);
    if (!isfinite(a0) || !isfinite(a1) || !isfinite(phi) || !isfinite(delta))
        return fail(SGM_ERR_INVALID, "road parameters must be finite");
    const double cx = (W - 1) * 0.5, cy = (H - 1) * 0.5;
    const double c = cos(phi), s = sin(phi);
    // the road disparity is linear in x along a row, so its minimum over
    // x = 0..W-1 sits at x = 0 or x = W-1
    const double xmin = s > 0.0 ? (double)(W - 1) : 0.0;
    for (int v = 0; v < H; ++v) {
        double lo;
        if (mode == 0) {
            lo = floor(a0 + a1 * c * (v - cy) + 0.5) - (double)(w / 2);
        } else {
            lo = floor(a0 + a1 * (c * (v - cy) - s * (xmin - cx)) - delta);
        }
        if (lo > 32767.0) return fail(SGM_ERR_INVALID, "window start out of range on row %d", v);
        d_lo[v] = lo > 0.0 ? (int32_t)lo : 0;
    }
    return SGM_OK;
}

}  // extern "C"
