// C-ABI layer of batches: validation, workspace layout, the per-pair
// descriptor table and the aggregation queue, runs, graph capture and the
// autotuner.  Kernels live in sgm_batch.hip.

#include "../../include/sgm.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "sgm_internal.h"

namespace {

sgm_status bfail(sgm_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(sgm::error_buffer(), sgm::kErrorBufferSize, fmt, ap);
    va_end(ap);
    return st;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// values per lane of the 16-lane mapping (every window width has one); a
// pair's ndisp must be a multiple of it
int lane_width(int w) { return sgm::choose_mapping(w, 16).vpl; }

// Step range of scanline group g (lpi lines) of direction r; same geometry
// as the kernels (horizontal: rows, vertical: columns, diagonal: sheared
// index).
int group_length(int r, int g, int W, int H, int lpi)
{
    static const int DU[8] = {1, -1, 0, 0, 1, -1, 1, -1};
    static const int DV[8] = {0, 0, 1, -1, 1, 1, -1, -1};
    const int du = DU[r], dv = DV[r];
    if (dv == 0) return W;
    if (du == 0) return H;
    int i0 = 1 << 30, i1 = 0;
    for (int l = 0; l < lpi; ++l) {
        const int idx = lpi * g + l;
        if (idx >= W + H - 1) break;
        const int ell = du > 0 ? idx - (H - 1) : idx;
        int a, b;
        if (du > 0) {
            a = std::max(0, -ell);
            b = std::min(H, W - ell);
        } else {
            a = std::max(0, ell - (W - 1));
            b = std::min(H, ell + 1);
        }
        if (b > a) {
            i0 = std::min(i0, a);
            i1 = std::max(i1, b);
        }
    }
    return i1 > i0 ? i1 - i0 : 0;
}

// scanline groups of direction r: one wave (64 lanes) carries lpi lines
int groups_of(int r, int W, int H, int lpi)
{
    if (r <= 1) return (H + lpi - 1) / lpi;
    if (r <= 3) return (W + lpi - 1) / lpi;
    return (W + H - 1 + lpi - 1) / lpi;
}

struct Item {
    uint32_t w0, g;
    int len, pair, kind;
};

}  // namespace

struct sgm_batch_s {
    sgm_batch_params prm;
    std::vector<sgm_pair> pairs;
    int cmax = 0;
    bool l8 = true;
    sgm_tuning tuning{8, 0, 0};
    size_t off_pairs = 0, off_items = 0, off_counter = 0, ws_bytes = 0;
    std::vector<sgm::PairDev> dev;  // offsets, host copy
    sgm::BatchGrids grids{0, 0, 0};
    std::vector<Item> items;
    sgm::PairDev *pin_pairs = nullptr;  // pinned host copies uploaded by every run
    uint32_t *pin_items = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // recorded after every enqueued run or graph replay: the pinned tables
    // and the graph stay untouched until the device has passed it
    hipEvent_t inflight = nullptr;
    bool capturing = false;
    int num_cu = 0;
    ~sgm_batch_s()
    {
        if (inflight) {
            hipEventSynchronize(inflight);
            hipEventDestroy(inflight);
        }
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (pin_pairs) hipHostFree(pin_pairs);
        if (pin_items) hipHostFree(pin_items);
    }
};

namespace {

// Block until the device has finished every run and replay enqueued so far
// (they read the pinned tables through their uploads, and replays run the
// graph).
void wait_inflight(sgm_batch_s *b)
{
    if (b->inflight) hipEventSynchronize(b->inflight);
}

// Mark the end of the work just enqueued on `st` (not while capturing: the
// graph's own replays are marked when launched).
hipError_t mark_inflight(sgm_batch_s *b, hipStream_t st)
{
    if (b->capturing) return hipSuccess;
    if (!b->inflight) {
        hipError_t e = hipEventCreateWithFlags(&b->inflight, hipEventDisableTiming);
        if (e != hipSuccess) {
            b->inflight = nullptr;
            return e;
        }
    }
    return hipEventRecord(b->inflight, st);
}

void drop_graph(sgm_batch_s *b)
{
    wait_inflight(b);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Lane mapping of every pair, the selection grid and the aggregation queue
// for the current tuning's lane count (the caller has waited for enqueued
// runs, which read the pinned tables).  Items are built in pair and
// direction order; order_items then sorts them.
void layout_queue(sgm_batch_s *b)
{
    b->items.clear();
    int wta_blk = 0;
    const int np = (int)b->pairs.size();
    for (int i = 0; i < np; ++i) {
        const sgm_pair &p = b->pairs[i];
        sgm::PairDev &d = b->dev[i];
        const sgm::Mapping m = sgm::choose_mapping(p.ndisp, b->tuning.lanes);
        d.lanes = m.lanes;
        d.vpl = m.vpl;
        d.pad = p.ndisp < m.lanes * m.vpl ? 1 : 0;
        // the horizontal directions always take 16 lanes per scanline
        const sgm::Mapping mh = sgm::choose_mapping(p.ndisp, 16);
        d.h_vpl = mh.vpl;
        d.h_pad = p.ndisp < 16 * mh.vpl ? 1 : 0;
        const sgm::Mapping ms = sgm::select_mapping(p.ndisp);
        d.wta_lanes = ms.lanes;
        d.wta_vpl = ms.vpl;
        const long long npix = (long long)p.width * p.height, ppb = 256 / ms.lanes;
        d.wta_start = wta_blk;
        wta_blk += (int)((npix + ppb - 1) / ppb);
        for (int r = 0; r < b->prm.npaths; ++r) {
            const int kind = r <= 1 ? 0 : (r >= 4 ? 1 : 2);  // horizontal, diagonal, vertical
            const int lpi = 64 / (kind == 0 ? 16 : m.lanes);  // scanlines per item
            for (int g = 0, n = groups_of(r, p.width, p.height, lpi); g < n; ++g)
                b->items.push_back(Item{(uint32_t)(i << 8 | r), (uint32_t)g,
                                        group_length(r, g, p.width, p.height, lpi), i, kind});
        }
    }
    b->grids.wta = wta_blk;
    memcpy(b->pin_pairs, b->dev.data(), b->dev.size() * sizeof(sgm::PairDev));
}

// Queue order of the aggregation items for the current tuning.
void order_items(sgm_batch_s *b)
{
    wait_inflight(b);  // a pending upload may still read the pinned queue
    std::vector<Item> &it = b->items;
    switch (b->tuning.order) {
    case 1:  // pair by pair, horizontal then diagonal then vertical inside a pair
        std::stable_sort(it.begin(), it.end(), [](const Item &x, const Item &y) {
            return x.pair != y.pair ? x.pair < y.pair : x.kind < y.kind;
        });
        break;
    case 2:  // direction kind by kind over all pairs
        std::stable_sort(it.begin(), it.end(), [](const Item &x, const Item &y) {
            return x.kind != y.kind ? x.kind < y.kind : x.pair < y.pair;
        });
        break;
    default:  // longest scanline group first
        std::stable_sort(it.begin(), it.end(), [](const Item &x, const Item &y) { return x.len > y.len; });
        break;
    }
    for (size_t i = 0; i < it.size(); ++i) {
        b->pin_items[2 * i] = it[i].w0;
        b->pin_items[2 * i + 1] = it[i].g;
    }
}

sgm_status check_batch_ws(const sgm_batch_s *b, void *ws, size_t bytes)
{
    if (!ws) return bfail(SGM_ERR_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return bfail(SGM_ERR_INVALID, "workspace must be 256-byte aligned");
    if (bytes < b->ws_bytes)
        return bfail(SGM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", bytes,
                     b->ws_bytes);
    return SGM_OK;
}

int agg_waves(sgm_batch_s *b)
{
    if (b->num_cu <= 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        b->num_cu = n;
    }
    const long long want = (long long)b->num_cu * b->tuning.waves_per_cu;
    return (int)std::max(1ll, std::min(want, (long long)b->items.size()));
}

sgm_status enqueue_run(sgm_batch_s *b, void *ws, hipStream_t st, const hipEvent_t *ev = nullptr)
{
    if (sgm::fault_take(sgm::kFaultLaunch)) return bfail(SGM_ERR_HIP, "injected launch failure");
    uint8_t *base = static_cast<uint8_t *>(ws);
    const size_t np = b->pairs.size();
    hipError_t e = hipMemcpyAsync(base + b->off_pairs, b->pin_pairs, np * sizeof(sgm::PairDev),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + b->off_items, b->pin_items, b->items.size() * 2 * sizeof(uint32_t),
                           hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return bfail(SGM_ERR_HIP, "descriptor upload: %s", hipGetErrorString(e));
    sgm::BatchDev d;
    d.ws = base;
    d.pairs = reinterpret_cast<const sgm::PairDev *>(base + b->off_pairs);
    d.items = reinterpret_cast<const uint32_t *>(base + b->off_items);
    d.counter = reinterpret_cast<uint32_t *>(base + b->off_counter);
    d.npairs = (int)np;
    d.nitems = (int)b->items.size();
    d.p1x2 = (uint32_t)b->prm.p1 * 0x10001u;
    d.p2x2 = (uint32_t)b->prm.p2 * 0x10001u;
    d.cmax = b->cmax;
    d.npaths = b->prm.npaths;
    e = sgm::launch_batch(d, b->grids, b->prm.census, b->l8, agg_waves(b), st, ev);
    if (e == hipSuccess) e = mark_inflight(b, st);
    return e == hipSuccess ? SGM_OK : bfail(SGM_ERR_HIP, "batch launch: %s", hipGetErrorString(e));
}

std::string tuning_key(const sgm_batch_s *b)
{
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    for (char &c : arch)
        if (c == ' ' || c == ':') c = '_';
    std::vector<std::string> shapes;
    for (const sgm_pair &p : b->pairs)
        shapes.push_back(std::to_string(p.width) + "x" + std::to_string(p.height) + "x" + std::to_string(p.ndisp));
    std::sort(shapes.begin(), shapes.end());
    // (h16: horizontal directions on 16 lanes, so entries timed with another
    // schedule are not reused)
    std::string key = "batch|h16|" + arch + "|n" + std::to_string(b->prm.census) + "|R" + std::to_string(b->prm.npaths) + "|P" +
                      std::to_string(b->prm.p1) + "," + std::to_string(b->prm.p2) + "|";
    for (size_t i = 0; i < shapes.size();) {
        size_t j = i;
        while (j < shapes.size() && shapes[j] == shapes[i]) ++j;
        key += shapes[i] + "*" + std::to_string(j - i) + ";";
        i = j;
    }
    return key;
}

bool valid_tuning(const sgm_tuning &t)
{
    return t.waves_per_cu >= 1 && t.waves_per_cu <= 32 && t.order >= 0 && t.order <= 2 &&
           (t.lanes == 0 || t.lanes == 4 || t.lanes == 8 || t.lanes == 16);
}

bool read_cache(const char *path, const std::string &key, sgm_tuning *out)
{
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[4096];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char k[3500];
        int wv = 0, ord = 0, lanes = -1;
        double ms = 0;
        if (sscanf(line, "%3499s %d %d %d %lf", k, &wv, &ord, &lanes, &ms) == 5 && key == k) {
            sgm_tuning t{wv, ord, lanes};
            if (valid_tuning(t)) {
                *out = t;
                found = true;
            }
        }
    }
    fclose(f);
    return found;
}

}  // namespace

extern "C" {

sgm_status sgm_batch_plan(const sgm_batch_params *prm, const sgm_pair *pairs, int32_t npairs, sgm_batch_t *out)
{
    if (!prm || !pairs || !out) return bfail(SGM_ERR_INVALID, "params, pairs and out must not be NULL");
    *out = nullptr;
    if (npairs < 1 || npairs > (1 << 23)) return bfail(SGM_ERR_INVALID, "npairs %d out of range", npairs);
    const sgm_batch_params &q = *prm;
    if (q.census != 3 && q.census != 5 && q.census != 7)
        return bfail(SGM_ERR_UNSUPPORTED, "census window %d not in {3, 5, 7}", q.census);
    if (q.npaths != 4 && q.npaths != 8) return bfail(SGM_ERR_UNSUPPORTED, "npaths %d not in {4, 8}", q.npaths);
    if (q.p1 < 0 || q.p2 < q.p1) return bfail(SGM_ERR_INVALID, "need 0 <= P1 <= P2");
    const int cmax = q.census * q.census - 1;
    if (2 * cmax + 3 * q.p2 >= 0x3FFF) return bfail(SGM_ERR_INVALID, "need 2*Cmax + 3*P2 < 16383");
    if ((long long)q.npaths * (cmax + q.p2) > 0xFFFF) return bfail(SGM_ERR_INVALID, "summed cost exceeds 16 bits");
    if (q.flags != 0) return bfail(SGM_ERR_INVALID, "flags must be 0");
    for (int i = 0; i < npairs; ++i) {
        const sgm_pair &p = pairs[i];
        if (p.width < 1 || p.height < 1 || p.pitch < p.width)
            return bfail(SGM_ERR_INVALID, "pair %d: bad size or pitch", i);
        if (p.ndisp < 1 || p.ndisp > 256) return bfail(SGM_ERR_INVALID, "pair %d: ndisp not in [1, 256]", i);
        if (p.ndisp % lane_width(p.ndisp))
            return bfail(SGM_ERR_UNSUPPORTED, "pair %d: ndisp %d is not a multiple of its lane width %d", i,
                         p.ndisp, lane_width(p.ndisp));
        if ((long long)p.width * p.height * p.ndisp >= (1ll << 31))
            return bfail(SGM_ERR_UNSUPPORTED, "pair %d: W*H*ndisp must be < 2^31", i);
        if (cmax + q.p2 > 255 && (long long)p.width * p.height * p.ndisp >= sgm::kMaxU16Volume)
            return bfail(SGM_ERR_UNSUPPORTED, "pair %d: uint16 per-path volumes need W*H*ndisp < 2^30", i);
        if (!p.left || !p.right || !p.disp_int) return bfail(SGM_ERR_INVALID, "pair %d: NULL buffer", i);
    }
    sgm_batch_s *b = new (std::nothrow) sgm_batch_s();
    if (!b) return bfail(SGM_ERR_INVALID, "out of host memory");
    b->prm = q;
    b->pairs.assign(pairs, pairs + npairs);
    b->cmax = cmax;
    b->l8 = cmax + q.p2 <= 255;
    const size_t esz = b->l8 ? 1 : 2;

    // workspace: descriptor table, queue, counter, then each pair's scratch
    size_t off = 0;
    b->off_pairs = off;
    off += align256((size_t)npairs * sizeof(sgm::PairDev));
    // queue capacity: the most items any lane count gives (16 lanes, four
    // scanlines per item)
    size_t nitems = 0;
    for (int i = 0; i < npairs; ++i)
        for (int r = 0; r < q.npaths; ++r) nitems += groups_of(r, pairs[i].width, pairs[i].height, 4);
    if (nitems >= (1u << 31)) {
        delete b;
        return bfail(SGM_ERR_UNSUPPORTED, "too many scanline groups");
    }
    b->off_items = off;
    off += align256(nitems * 2 * sizeof(uint32_t));
    b->off_counter = off;
    off += 256;
    b->dev.resize(npairs);
    int census_blk = 0, cost_blk = 0;
    for (int i = 0; i < npairs; ++i) {
        const sgm_pair &p = pairs[i];
        sgm::PairDev &d = b->dev[i];
        memset(&d, 0, sizeof d);
        const size_t npix = (size_t)p.width * p.height, nvol = npix * (size_t)p.ndisp;
        d.left = p.left;
        d.right = p.right;
        d.d_lo = p.d_lo;
        d.dint = p.disp_int;
        d.dsub = p.disp_sub;
        d.off_codes_l = (long long)off;
        off += align256(npix * 8);
        d.off_codes_r = (long long)off;
        off += align256(npix * 8);
        d.off_cost = (long long)off;
        off += align256(nvol);
        d.off_vols = (long long)off;
        const size_t vs = align256(nvol * esz);
        off += vs * (size_t)q.npaths;
        d.vstride = (long long)(vs / esz);
        d.W = p.width;
        d.H = p.height;
        d.w = p.ndisp;
        d.pitch = p.pitch;
        d.census_tx = (p.width + sgm::kCensusTW - 1) / sgm::kCensusTW;
        d.census_ty = (p.height + sgm::kCensusTH - 1) / sgm::kCensusTH;
        d.cost_tx = (p.width + 63) / 64;
        d.census_start = census_blk;
        census_blk += 2 * d.census_tx * d.census_ty;
        d.cost_start = cost_blk;
        cost_blk += d.cost_tx * p.height;
    }
    b->ws_bytes = off;
    b->grids = {census_blk, cost_blk, 0};
    b->items.reserve(nitems);
    if (sgm::fault_take(sgm::kFaultAlloc)) {
        delete b;
        return bfail(SGM_ERR_HIP, "injected allocation failure");
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&b->pin_pairs), npairs * sizeof(sgm::PairDev)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&b->pin_items), std::max<size_t>(1, nitems) * 2 * sizeof(uint32_t)) !=
            hipSuccess) {
        delete b;
        return bfail(SGM_ERR_HIP, "pinned host allocation failed");
    }
    layout_queue(b);
    order_items(b);
    *out = b;
    return SGM_OK;
}

void sgm_batch_free(sgm_batch_t b) { delete b; }

sgm_status sgm_batch_workspace_size(sgm_batch_t b, size_t *bytes)
{
    if (!b || !bytes) return bfail(SGM_ERR_INVALID, "batch and bytes must not be NULL");
    *bytes = b->ws_bytes;
    return SGM_OK;
}

sgm_status sgm_batch_set_tuning(sgm_batch_t b, const sgm_tuning *t)
{
    if (!b || !t) return bfail(SGM_ERR_INVALID, "batch and tuning must not be NULL");
    if (!valid_tuning(*t)) return bfail(SGM_ERR_INVALID, "tuning out of range");
    if (t->order != b->tuning.order || t->waves_per_cu != b->tuning.waves_per_cu || t->lanes != b->tuning.lanes) {
        drop_graph(b);  // also waits for every enqueued run
        const bool relayout = t->lanes != b->tuning.lanes;
        const bool reorder = relayout || t->order != b->tuning.order;
        b->tuning = *t;
        if (relayout) layout_queue(b);
        if (reorder) order_items(b);
    }
    return SGM_OK;
}

sgm_status sgm_batch_get_tuning(sgm_batch_t b, sgm_tuning *t)
{
    if (!b || !t) return bfail(SGM_ERR_INVALID, "batch and tuning must not be NULL");
    *t = b->tuning;
    return SGM_OK;
}

sgm_status sgm_batch_run(sgm_batch_t b, void *ws, size_t bytes, void *stream)
{
    if (!b) return bfail(SGM_ERR_INVALID, "batch is NULL");
    if (sgm_status s = check_batch_ws(b, ws, bytes)) return s;
    return enqueue_run(b, ws, (hipStream_t)stream);
}

sgm_status sgm_batch_capture(sgm_batch_t b, void *ws, size_t bytes, void *stream)
{
    if (!b) return bfail(SGM_ERR_INVALID, "batch is NULL");
    if (!stream) return bfail(SGM_ERR_INVALID, "capture needs a stream other than the null stream");
    if (sgm_status s = check_batch_ws(b, ws, bytes)) return s;
    drop_graph(b);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(SGM_ERR_HIP, "begin capture: %s", hipGetErrorString(e));
    b->capturing = true;
    sgm_status rs = enqueue_run(b, ws, st);
    b->capturing = false;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (rs != SGM_OK) {
        if (g) hipGraphDestroy(g);
        return rs;
    }
    if (e != hipSuccess) return bfail(SGM_ERR_HIP, "end capture: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        return bfail(SGM_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    b->graph = g;
    b->exec = x;
    return SGM_OK;
}

sgm_status sgm_batch_launch(sgm_batch_t b, void *stream)
{
    if (!b) return bfail(SGM_ERR_INVALID, "batch is NULL");
    if (!b->exec) return bfail(SGM_ERR_INVALID, "no captured graph (call sgm_batch_capture first)");
    if (sgm::fault_take(sgm::kFaultLaunch)) return bfail(SGM_ERR_HIP, "injected launch failure");
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e == hipSuccess) e = mark_inflight(b, (hipStream_t)stream);
    return e == hipSuccess ? SGM_OK : bfail(SGM_ERR_HIP, "graph launch: %s", hipGetErrorString(e));
}

sgm_status sgm_batch_run_timed(sgm_batch_t b, void *ws, size_t bytes, void *stream, float *ms)
{
    if (!b || !ms) return bfail(SGM_ERR_INVALID, "batch and ms must not be NULL");
    if (sgm_status s = check_batch_ws(b, ws, bytes)) return s;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    sgm_status rs = SGM_OK;
    for (int i = 0; i < 5 && rs == SGM_OK; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) {
            ev[i] = nullptr;
            rs = bfail(SGM_ERR_HIP, "event creation failed");
        }
    if (rs == SGM_OK) rs = enqueue_run(b, ws, (hipStream_t)stream, ev);
    if (rs == SGM_OK) {
        hipError_t e = hipEventSynchronize(ev[4]);
        for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]);
        if (e != hipSuccess) rs = bfail(SGM_ERR_HIP, "stage timing: %s", hipGetErrorString(e));
    }
    for (hipEvent_t x : ev)
        if (x) hipEventDestroy(x);
    return rs;
}

sgm_status sgm_batch_autotune(sgm_batch_t b, void *ws, size_t bytes, void *stream, const char *cache_path,
                              sgm_tuning *chosen)
{
    if (!b) return bfail(SGM_ERR_INVALID, "batch is NULL");
    if (sgm_status s = check_batch_ws(b, ws, bytes)) return s;
    const std::string key = tuning_key(b);
    sgm_tuning t;
    if (read_cache(cache_path, key, &t)) {
        sgm_status s = sgm_batch_set_tuning(b, &t);
        if (chosen) *chosen = b->tuning;
        return s;
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        if (chosen) *chosen = b->tuning;
        return bfail(SGM_ERR_HIP, "event creation failed; default tuning kept");
    }
    const sgm_tuning start = b->tuning;
    sgm_tuning best = start;
    float best_ms = 1e30f;
    bool ok = true;
    auto trial = [&](const sgm_tuning &c) {
        sgm_batch_set_tuning(b, &c);
        float ms = 1e30f;
        for (int rep = 0; rep < 3 && ok; ++rep) {
            ok = hipEventRecord(e0, st) == hipSuccess && enqueue_run(b, ws, st) == SGM_OK &&
                 hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float t_ms = 0;
            if (ok && rep > 0 && hipEventElapsedTime(&t_ms, e0, e1) == hipSuccess) ms = std::min(ms, t_ms);
        }
        if (ok && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    };
    // every lane mapping x waves per CU x queue order (the best lane count
    // moves with the waves per CU: on 16 quarter-scale 480x270x48 pairs 4
    // lanes at 4 waves beat the best 8-lane choice by 10 %)
    const int waves[] = {4, 8, 12, 16, 24};
    for (int lanes : {16, 8, 4})
        for (int order = 0; order <= 2 && ok; ++order)
            for (int wv : waves)
                if (ok) trial(sgm_tuning{wv, order, lanes});
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (!ok) {
        sgm_batch_set_tuning(b, &start);
        if (chosen) *chosen = b->tuning;
        return bfail(SGM_ERR_HIP, "autotune run failed; previous tuning kept");
    }
    sgm_batch_set_tuning(b, &best);
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s %d %d %d %.4f\n", key.c_str(), best.waves_per_cu, best.order, best.lanes, best_ms);
            fclose(f);
        }
    }
    if (chosen) *chosen = b->tuning;
    return SGM_OK;
}

}  // extern "C"
