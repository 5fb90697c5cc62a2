// Sanitizer run of libsgm's host code (test infrastructure): the C-ABI layer
// compiled for the host with AddressSanitizer and UndefinedBehaviorSanitizer,
// linked against tests/sanitize/fake_device.cpp instead of the GPU, and
// driven through every call of include/sgm.h with valid and invalid
// arguments.  Every buffer is allocated with exactly the size the ABI
// documents, so a layout or size error in the host code shows up as an
// AddressSanitizer report in the stand-in launchers.  Prints "clean" at the
// end; any failed expectation exits non-zero.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/sgm.h"

static int g_failures = 0;
#define EXPECT(c)                                                           \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "driver: expectation failed at line %d: %s (%s)\n", __LINE__, #c, \
                    sgm_last_error());                                      \
            ++g_failures;                                                   \
        }                                                                   \
    } while (0)

namespace {

// an exactly sized, 256-byte aligned heap block (the ABI's alignment)
struct Buf {
    void *p = nullptr;
    size_t n = 0;
    explicit Buf(size_t bytes) : n(bytes)
    {
        p = aligned_alloc(256, ((bytes ? bytes : 1) + 255) / 256 * 256);
        memset(p, 0, ((bytes ? bytes : 1) + 255) / 256 * 256);
    }
    ~Buf() { free(p); }
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
    template <typename T> T *as() { return static_cast<T *>(p); }
};

sgm_params params(int W, int H, int n, int w, int R, int p1 = 10, int p2 = 120)
{
    sgm_params q;
    q.width = W;
    q.height = H;
    q.census = n;
    q.ndisp = w;
    q.npaths = R;
    q.p1 = p1;
    q.p2 = p2;
    q.flags = 0;
    return q;
}

// every single-pair call on one plan with exactly sized buffers
void single_pair(int W, int H, int n, int w, int R, int p2, int lanes, bool with_dlo)
{
    sgm_params q = params(W, H, n, w, R, 10, p2);
    sgm_plan_t plan = nullptr;
    sgm_tuning t{0, 0, lanes};
    EXPECT(sgm_plan_tuned(&q, &t, &plan) == SGM_OK);
    if (!plan) return;
    sgm_tuning got{};
    EXPECT(sgm_plan_get_tuning(plan, &got) == SGM_OK);
    EXPECT(got.lanes == 4 || got.lanes == 8 || got.lanes == 16);
    size_t ws = 0, vstride = 0, total = 0;
    int32_t esz = 0;
    EXPECT(sgm_workspace_size(plan, &ws) == SGM_OK);
    EXPECT(sgm_path_volumes(plan, &esz, &vstride, &total) == SGM_OK);
    const int pitch = W + (W % 3);
    const size_t npix = (size_t)W * H, nvol = npix * w;
    Buf left((size_t)H * pitch), right((size_t)H * pitch), dlo((size_t)H * 4), work(ws), cost(nvol),
        sum(nvol * 2), L(nvol * 2), paths(total), dint(npix * 2), dsub(npix * 4), codes(npix * 8);
    const int32_t *d_lo = with_dlo ? dlo.as<int32_t>() : nullptr;
    EXPECT(sgm_census(plan, left.as<uint8_t>(), pitch, codes.as<uint64_t>(), nullptr) == SGM_OK);
    EXPECT(sgm_cost(plan, left.as<uint8_t>(), right.as<uint8_t>(), pitch, d_lo, cost.as<uint8_t>(), work.p, ws,
                    nullptr) == SGM_OK);
    EXPECT(sgm_aggregate(plan, cost.as<uint8_t>(), sum.as<uint16_t>(), work.p, ws, nullptr) == SGM_OK);
    if ((long long)nvol < (1ll << 30))
        for (int r = 0; r < R; ++r)
            EXPECT(sgm_aggregate_path(plan, cost.as<uint8_t>(), r, L.as<uint16_t>(), nullptr) == SGM_OK);
    EXPECT(sgm_wta(plan, sum.as<uint16_t>(), d_lo, dint.as<uint16_t>(), dsub.as<float>(), nullptr) == SGM_OK);
    EXPECT(sgm_aggregate_wta(plan, cost.as<uint8_t>(), d_lo, dint.as<uint16_t>(), nullptr, work.p, ws, nullptr) ==
           SGM_OK);
    EXPECT(sgm_aggregate_paths(plan, cost.as<uint8_t>(), paths.p, total, nullptr) == SGM_OK);
    EXPECT(sgm_wta_paths(plan, paths.p, d_lo, dint.as<uint16_t>(), dsub.as<float>(), nullptr) == SGM_OK);
    EXPECT(sgm_match(plan, left.as<uint8_t>(), right.as<uint8_t>(), pitch, d_lo, dint.as<uint16_t>(),
                     dsub.as<float>(), work.p, ws, nullptr) == SGM_OK);
    // a cost volume one byte off its alignment: the element-wise mapping
    if (nvol > 1) {
        Buf odd(nvol + 1);
        EXPECT(sgm_cost(plan, left.as<uint8_t>(), right.as<uint8_t>(), pitch, d_lo, odd.as<uint8_t>() + 1, work.p,
                        ws, nullptr) == SGM_OK);
        EXPECT(sgm_aggregate_wta(plan, odd.as<uint8_t>() + 1, d_lo, dint.as<uint16_t>(), dsub.as<float>(), work.p,
                                 ws, nullptr) == SGM_OK);
    }
    // refused before anything is enqueued
    EXPECT(sgm_match(plan, left.as<uint8_t>(), right.as<uint8_t>(), pitch, d_lo, dint.as<uint16_t>(),
                     dsub.as<float>(), work.p, ws - 1, nullptr) == SGM_ERR_WORKSPACE);
    EXPECT(sgm_aggregate_paths(plan, cost.as<uint8_t>(), paths.p, total - 1, nullptr) == SGM_ERR_WORKSPACE);
    EXPECT(sgm_cost(plan, left.as<uint8_t>(), right.as<uint8_t>(), W - 1, d_lo, cost.as<uint8_t>(), work.p, ws,
                    nullptr) == SGM_ERR_INVALID);
    EXPECT(sgm_aggregate_path(plan, cost.as<uint8_t>(), 8, L.as<uint16_t>(), nullptr) == SGM_ERR_INVALID);
    sgm_plan_free(plan);
}

void plans()
{
    // widths around every lane mapping, ragged sizes, both volume types
    const int widths[] = {1, 2, 3, 4, 7, 8, 12, 16, 20, 24, 32, 40, 48, 56, 64, 65, 96, 100, 128, 129, 192, 256};
    for (int w : widths)
        for (int lanes : {0, 4, 8, 16}) {
            single_pair(19, 7, 7, w, 8, 120, lanes, true);
            single_pair(5, 13, 5, w, 4, 220, lanes, false);
        }
    single_pair(1, 1, 3, 1, 4, 20, 0, false);
    single_pair(64, 1, 7, 64, 8, 120, 4, true);
    single_pair(1, 64, 7, 24, 8, 120, 8, true);
    // parameter validation
    sgm_plan_t p = nullptr;
    sgm_params bad[] = {params(0, 5, 7, 8, 8), params(5, 5, 9, 8, 8),  params(5, 5, 7, 0, 8),
                        params(5, 5, 7, 257, 8), params(5, 5, 7, 8, 6), params(5, 5, 7, 8, 8, 11, 10),
                        params(5, 5, 7, 8, 8, 10, 8200), params(40000, 40000, 7, 8, 8),
                        params(4096, 2304, 7, 128, 8, 10, 220)};
    for (const sgm_params &q : bad) {
        EXPECT(sgm_plan(&q, &p) != SGM_OK);
        EXPECT(p == nullptr);
    }
    sgm_params ok = params(8, 8, 7, 16, 8);
    sgm_tuning t{0, 0, 5};
    EXPECT(sgm_plan_tuned(&ok, &t, &p) == SGM_ERR_INVALID);
    EXPECT(sgm_plan_tuned(&ok, nullptr, &p) == SGM_ERR_INVALID);
    EXPECT(sgm_plan(nullptr, &p) == SGM_ERR_INVALID);
    EXPECT(sgm_plan_get_tuning(nullptr, &t) == SGM_ERR_INVALID);
    size_t n = 0;
    EXPECT(sgm_workspace_size(nullptr, &n) == SGM_ERR_INVALID);
    for (int s = -5; s <= 1; ++s) EXPECT(sgm_status_str((sgm_status)s) != nullptr);
}

void autotune()
{
    const char *cache = "sanitize_tune_cache.txt";
    remove(cache);
    const int W = 23, H = 9, w = 24;
    sgm_params q = params(W, H, 7, w, 8);
    sgm_plan_t plan = nullptr;
    EXPECT(sgm_plan(&q, &plan) == SGM_OK);
    size_t ws = 0;
    sgm_workspace_size(plan, &ws);
    Buf left((size_t)W * H), right((size_t)W * H), work(ws), dint((size_t)W * H * 2), dsub((size_t)W * H * 4);
    sgm_tuning a{}, b{};
    EXPECT(sgm_autotune(&q, left.as<uint8_t>(), right.as<uint8_t>(), W, nullptr, dint.as<uint16_t>(),
                        dsub.as<float>(), work.p, ws, nullptr, cache, &a) == SGM_OK);
    EXPECT(sgm_autotune(&q, left.as<uint8_t>(), right.as<uint8_t>(), W, nullptr, dint.as<uint16_t>(),
                        dsub.as<float>(), work.p, ws, nullptr, cache, &b) == SGM_OK);
    EXPECT(a.lanes == b.lanes);
    // a corrupt cache falls back to timing
    FILE *f = fopen(cache, "w");
    fputs("\xff\xfe garbage without fields\nsingle|x 1\n", f);
    fclose(f);
    EXPECT(sgm_autotune(&q, left.as<uint8_t>(), right.as<uint8_t>(), W, nullptr, dint.as<uint16_t>(),
                        dsub.as<float>(), work.p, ws, nullptr, cache, &b) == SGM_OK);
    EXPECT(sgm_autotune(&q, left.as<uint8_t>(), right.as<uint8_t>(), W, nullptr, dint.as<uint16_t>(),
                        dsub.as<float>(), work.p, ws - 1, nullptr, nullptr, &b) == SGM_ERR_WORKSPACE);
    remove(cache);
    sgm_plan_free(plan);
}

void batches()
{
    struct Shape {
        int W, H, w, pitch;
        bool rows;
    };
    const Shape shapes[] = {{97, 61, 24, 97, true}, {160, 120, 64, 160, false}, {200, 150, 128, 256, false},
                            {45, 33, 16, 45, true},  {64, 40, 192, 64, false},  {70, 9, 256, 80, false},
                            {33, 70, 32, 33, false}, {51, 47, 48, 64, true},    {1, 1, 4, 1, false}};
    const int np = sizeof shapes / sizeof shapes[0];
    std::vector<Buf *> bufs;
    std::vector<sgm_pair> pairs(np);
    for (int i = 0; i < np; ++i) {
        const Shape &s = shapes[i];
        Buf *l = new Buf((size_t)s.pitch * s.H), *r = new Buf((size_t)s.pitch * s.H);
        Buf *d = new Buf((size_t)s.H * 4), *di = new Buf((size_t)s.W * s.H * 2), *ds = new Buf((size_t)s.W * s.H * 4);
        bufs.insert(bufs.end(), {l, r, d, di, ds});
        pairs[i] = sgm_pair{s.W, s.H, s.w, s.pitch, l->as<uint8_t>(), r->as<uint8_t>(),
                            s.rows ? d->as<int32_t>() : nullptr, di->as<uint16_t>(), i % 2 ? ds->as<float>() : nullptr};
    }
    for (int R : {4, 8}) {
        sgm_batch_params bp{7, R, 10, R == 8 ? 120 : 220, 0};
        sgm_batch_t b = nullptr;
        EXPECT(sgm_batch_plan(&bp, pairs.data(), np, &b) == SGM_OK);
        if (!b) continue;
        size_t ws = 0;
        EXPECT(sgm_batch_workspace_size(b, &ws) == SGM_OK);
        Buf work(ws);
        EXPECT(sgm_batch_run(b, work.p, ws, nullptr) == SGM_OK);
        for (int lanes : {0, 4, 8, 16})
            for (int order = 0; order <= 2; ++order)
                for (int wv : {1, 8, 32}) {
                    sgm_tuning t{wv, order, lanes}, back{};
                    EXPECT(sgm_batch_set_tuning(b, &t) == SGM_OK);
                    EXPECT(sgm_batch_get_tuning(b, &back) == SGM_OK);
                    EXPECT(back.lanes == lanes && back.order == order && back.waves_per_cu == wv);
                    EXPECT(sgm_batch_run(b, work.p, ws, nullptr) == SGM_OK);
                }
        int dummy_stream = 0;
        void *stream = &dummy_stream;  // capture needs a non-null stream token
        EXPECT(sgm_batch_capture(b, work.p, ws, stream) == SGM_OK);
        EXPECT(sgm_batch_launch(b, stream) == SGM_OK);
        sgm_tuning t2{4, 1, 4};
        EXPECT(sgm_batch_set_tuning(b, &t2) == SGM_OK);  // drops the graph
        EXPECT(sgm_batch_launch(b, stream) == SGM_ERR_INVALID);
        EXPECT(sgm_batch_capture(b, work.p, ws, nullptr) == SGM_ERR_INVALID);
        float ms[4];
        EXPECT(sgm_batch_run_timed(b, work.p, ws, nullptr, ms) == SGM_OK);
        const char *cache = "sanitize_batch_cache.txt";
        remove(cache);
        sgm_tuning c1{}, c2{};
        EXPECT(sgm_batch_autotune(b, work.p, ws, nullptr, cache, &c1) == SGM_OK);
        EXPECT(sgm_batch_autotune(b, work.p, ws, nullptr, cache, &c2) == SGM_OK);
        EXPECT(c1.lanes == c2.lanes && c1.order == c2.order && c1.waves_per_cu == c2.waves_per_cu);
        remove(cache);
        EXPECT(sgm_batch_run(b, work.p, ws - 1, nullptr) == SGM_ERR_WORKSPACE);
        sgm_tuning badt{0, 0, 0};
        EXPECT(sgm_batch_set_tuning(b, &badt) == SGM_ERR_INVALID);
        badt = sgm_tuning{8, 3, 0};
        EXPECT(sgm_batch_set_tuning(b, &badt) == SGM_ERR_INVALID);
        badt = sgm_tuning{8, 0, 12};
        EXPECT(sgm_batch_set_tuning(b, &badt) == SGM_ERR_INVALID);
        // injected failures enqueue nothing
        EXPECT(sgm_debug_inject_fault(1) == SGM_OK);
        EXPECT(sgm_batch_run(b, work.p, ws, nullptr) == SGM_ERR_HIP);
        EXPECT(sgm_batch_run(b, work.p, ws, nullptr) == SGM_OK);
        sgm_batch_free(b);
    }
    // invalid batches
    sgm_batch_params bp{7, 8, 10, 120, 0};
    sgm_batch_t b = nullptr;
    sgm_pair bad = pairs[0];
    bad.ndisp = 25;  // not a multiple of its lane width
    EXPECT(sgm_batch_plan(&bp, &bad, 1, &b) == SGM_ERR_UNSUPPORTED);
    bad = pairs[0];
    bad.pitch = bad.width - 1;
    EXPECT(sgm_batch_plan(&bp, &bad, 1, &b) == SGM_ERR_INVALID);
    EXPECT(sgm_batch_plan(&bp, pairs.data(), 0, &b) == SGM_ERR_INVALID);
    EXPECT(sgm_debug_inject_fault(2) == SGM_OK);
    EXPECT(sgm_batch_plan(&bp, pairs.data(), np, &b) == SGM_ERR_HIP);
    EXPECT(b == nullptr);
    for (Buf *x : bufs) delete x;
}

void windows()
{
    const int W = 37, H = 11, n = 7;
    sgm_params q = params(W, H, n, 16, 8);
    sgm_plan_t plan = nullptr;
    EXPECT(sgm_plan(&q, &plan) == SGM_OK);
    size_t ws = 0, total = 0;
    sgm_workspace_size(plan, &ws);
    sgm_path_volumes(plan, nullptr, nullptr, &total);
    const size_t npix = (size_t)W * H;
    Buf left(npix), right(npix), lo(npix * 4), work(ws), cost(npix * 16), paths(total), dint(npix * 2),
        dsub(npix * 4);
    EXPECT(sgm_cost_win(plan, left.as<uint8_t>(), right.as<uint8_t>(), W, lo.as<int32_t>(), cost.as<uint8_t>(),
                        work.p, ws, nullptr) == SGM_OK);
    EXPECT(sgm_aggregate_win_paths(plan, cost.as<uint8_t>(), lo.as<int32_t>(), paths.p, total, nullptr) == SGM_OK);
    EXPECT(sgm_wta_win_paths(plan, paths.p, lo.as<int32_t>(), dint.as<uint16_t>(), dsub.as<float>(), nullptr) ==
           SGM_OK);
    EXPECT(sgm_match_win(plan, left.as<uint8_t>(), right.as<uint8_t>(), W, lo.as<int32_t>(), dint.as<uint16_t>(),
                         nullptr, work.p, ws, nullptr) == SGM_OK);
    const int nimg = 3, pitch = W + 5;
    size_t wsb = 0;
    EXPECT(sgm_workspace_size_win_batch(plan, nimg, &wsb) == SGM_OK);
    Buf bl((size_t)nimg * pitch * H), br((size_t)nimg * pitch * H), blo(npix * 4 * nimg), bws(wsb),
        bdi(npix * 2 * nimg), bds(npix * 4 * nimg);
    EXPECT(sgm_match_win_batch(plan, bl.as<uint8_t>(), br.as<uint8_t>(), pitch, (int64_t)pitch * H,
                               blo.as<int32_t>(), nimg, bdi.as<uint16_t>(), bds.as<float>(), bws.p, wsb,
                               nullptr) == SGM_OK);
    EXPECT(sgm_match_win_batch(plan, bl.as<uint8_t>(), br.as<uint8_t>(), pitch, (int64_t)pitch * H,
                               blo.as<int32_t>(), nimg, bdi.as<uint16_t>(), bds.as<float>(), bws.p, wsb - 1,
                               nullptr) == SGM_ERR_WORKSPACE);
    Buf small((size_t)(W / 4) * (H / 4) * nimg);
    EXPECT(sgm_downsample4(left.as<uint8_t>(), W, H, W, small.as<uint8_t>(), nullptr) == SGM_OK);
    EXPECT(sgm_downsample4_batch(bl.as<uint8_t>(), W, H, pitch, (int64_t)pitch * H, nimg, small.as<uint8_t>(),
                                 nullptr) == SGM_OK);
    EXPECT(sgm_downsample4(left.as<uint8_t>(), 3, H, W, small.as<uint8_t>(), nullptr) == SGM_ERR_INVALID);
    sgm_plan_free(plan);
    // window helper (host, fp64)
    std::vector<int32_t> dl(H);
    EXPECT(sgm_window_from_road(7.8, 0.0996, 0.03, W, H, 24, 0, 0.0, dl.data()) == SGM_OK);
    EXPECT(sgm_window_from_road(7.8, 0.0996, 0.05, W, H, 24, 1, 3.0, dl.data()) == SGM_OK);
    EXPECT(sgm_window_from_road(NAN, 0.0996, 0.05, W, H, 24, 1, 3.0, dl.data()) != SGM_OK);
}

void road_pothole_slic()
{
    const int W = 41, H = 23, nimg = 2;
    const size_t np = (size_t)W * H * nimg;
    size_t rws = 0, pws = 0, sws = 0;
    EXPECT(sgm_road_workspace_size(W, H, nimg, &rws) == SGM_OK);
    Buf disp(np * 4), mask(np), fit(sizeof(sgm_road_fit) * nimg), work(rws), dlo((size_t)H * nimg * 4),
        lo(np * 4), out(np * 4), phi(8 * 5), energy(8 * 5 * nimg);
    EXPECT(sgm_road_fit_batch(disp.as<float>(), mask.as<uint8_t>(), W, H, nimg, 0.5f, -INFINITY, nullptr,
                              INFINITY, fit.as<sgm_road_fit>(), work.p, rws, nullptr) == SGM_OK);
    EXPECT(sgm_road_fit_batch(disp.as<float>(), nullptr, W, H, nimg, 0.5f, 4.0, fit.as<sgm_road_fit>(), 2.0,
                              fit.as<sgm_road_fit>(), work.p, rws, nullptr) == SGM_OK);
    EXPECT(sgm_road_fit_batch(disp.as<float>(), nullptr, W, H, nimg, 0.5f, 4.0, nullptr, INFINITY,
                              fit.as<sgm_road_fit>(), work.p, rws - 1, nullptr) == SGM_ERR_WORKSPACE);
    EXPECT(sgm_road_energy_batch(disp.as<float>(), mask.as<uint8_t>(), W, H, nimg, 0.5f, -INFINITY, nullptr,
                                 INFINITY, phi.as<double>(), 5, energy.as<double>(), work.p, rws, nullptr) == SGM_OK);
    EXPECT(sgm_road_window_batch(fit.as<sgm_road_fit>(), W, H, nimg, 24, 1, 2.0, 1.0, dlo.as<int32_t>(), nullptr) ==
           SGM_OK);
    EXPECT(sgm_road_window_map_batch(fit.as<sgm_road_fit>(), W, H, nimg, 16, 4.0, lo.as<int32_t>(), nullptr) ==
           SGM_OK);
    EXPECT(sgm_disparity_transform_batch(disp.as<float>(), fit.as<sgm_road_fit>(), W, H, nimg, 10.0,
                                         out.as<float>(), nullptr) == SGM_OK);
    EXPECT(sgm_road_mask_batch(disp.as<float>(), fit.as<sgm_road_fit>(), W, H, nimg, 2.0, 4.0, mask.as<uint8_t>(),
                               nullptr) == SGM_OK);
    const int nbins = 64;
    EXPECT(sgm_pothole_workspace_size(nbins, nimg, &pws) == SGM_OK);
    Buf pw(pws), res(sizeof(sgm_pothole_threshold) * nimg), curve(8 * nbins * nimg), labels(np * 4), sp(np * 4);
    EXPECT(sgm_pothole_threshold_batch(out.as<float>(), mask.as<uint8_t>(), W, H, nimg, 2.0, 18.0, nbins, 2.36,
                                       res.as<sgm_pothole_threshold>(), curve.as<double>(), pw.p, pws,
                                       nullptr) == SGM_OK);
    EXPECT(sgm_pothole_threshold_batch(out.as<float>(), nullptr, W, H, nimg, 18.0, 2.0, nbins, 2.36,
                                       res.as<sgm_pothole_threshold>(), nullptr, pw.p, pws, nullptr) == SGM_ERR_INVALID);
    EXPECT(sgm_pothole_label_batch(out.as<float>(), mask.as<uint8_t>(), W, H, nimg, res.as<sgm_pothole_threshold>(),
                                   labels.as<int32_t>(), nullptr) == SGM_OK);
    EXPECT(sgm_pothole_prune_batch(sp.as<int32_t>(), W, H, nimg, labels.as<int32_t>(), nullptr) == SGM_OK);
    const int S = 8;
    EXPECT(sgm_slic_workspace_size(W, H, S, nimg, &sws) == SGM_OK);
    const size_t K = (size_t)((W + S - 1) / S) * ((H + S - 1) / S);
    Buf sw(sws), rounds(4 * nimg), d3(np * 4), centres(K * 3 * 8 * nimg);
    EXPECT(sgm_slic_batch(out.as<float>(), mask.as<uint8_t>(), W, H, nimg, S, 4.0, 10, 0.25, rounds.as<int32_t>(),
                          sp.as<int32_t>(), d3.as<float>(), centres.as<double>(), sw.p, sws, nullptr) == SGM_OK);
    EXPECT(sgm_slic_batch(out.as<float>(), mask.as<uint8_t>(), W, H, nimg, 1, 4.0, 10, 0.25, rounds.as<int32_t>(),
                          sp.as<int32_t>(), d3.as<float>(), centres.as<double>(), sw.p, sws, nullptr) == SGM_ERR_INVALID);
}

}  // namespace

int main()
{
    plans();
    autotune();
    batches();
    windows();
    road_pothole_slic();
    if (g_failures) {
        fprintf(stderr, "driver: %d expectation(s) failed\n", g_failures);
        return 1;
    }
    printf("clean\n");
    return 0;
}
