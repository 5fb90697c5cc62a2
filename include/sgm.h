/*
 * sgm.h -- C ABI of the MI355X (gfx950) semi-global matching library.
 *
 * The library computes the dense-stereo stage of the road-disparity
 * pipeline of Fan et al., "Rethinking Road Surface 3D Reconstruction and
 * Pothole Detection: From Perspective Transformation to Disparity Map
 * Segmentation":
 *   - per-pixel matching cost c(p,d) (Sec. II-B, eq. (7); the paper leaves
 *     the cost open, the library uses an n x n census transform with the
 *     Hamming distance);
 *   - path aggregation along 4 or 8 image directions (Sec. II-B, eq. (8)),
 *     in the normalised form
 *       L_r(p,k) = C(p,k) + min(L_r(q,k), L_r(q,k-1)+P1, L_r(q,k+1)+P1,
 *                               m_q+P2) - m_q,   q = p - r,
 *                  m_q = min_i L_r(q,i);
 *   - the summed cost S(p,k) = sum_r L_r(p,k) and the winner-take-all
 *     disparity (eq. (9), read as the smallest k minimising S);
 *   - parabola sub-pixel refinement (Sec. I names sub-pixel disparities,
 *     the method is not given);
 *   - the perspective-transformation window (Sec. II-A, eq. (6)) as a
 *     per-row integer window start d_lo(v): window index k of row v means
 *     disparity d_lo(v) + k, and outputs are returned in disparities of
 *     the original pair (eq. (10)).
 *
 * Conventions common to every call
 *   - Images are uint8 grayscale, row-major, H rows of W pixels, with a
 *     row pitch in bytes (pitch >= W).  The left image is the reference.
 *   - Volumes are row-major [H][W][w] with the window index k fastest:
 *     element (u, v, k) is at ((v * W + u) * w + k).
 *   - Path indices r = 0..7 are the directions (du, dv) = (+1,0), (-1,0),
 *     (0,+1), (0,-1), (+1,+1), (-1,+1), (+1,-1), (-1,-1); the predecessor
 *     of pixel p on path r is p - r.  4-path runs use r = 0..3.
 *   - Every pointer marked "device" is device memory owned by the caller;
 *     the library never allocates, frees or synchronises on the compute
 *     calls.  Work is enqueued asynchronously on `stream` (a hipStream_t;
 *     NULL is the null stream).  Outputs are valid once the stream has
 *     reached the enqueued work.
 *   - Argument checks happen before anything is enqueued; a failing call
 *     enqueues nothing.  A failed launch returns SGM_ERR_HIP.  Device faults
 *     surface at the caller's next synchronisation.  sgm_last_error()
 *     returns a thread-local description of the last failure.
 *   - A plan is immutable after sgm_plan() and may be used from several
 *     threads and streams at once, each with its own workspace.
 */
#ifndef SGM_H
#define SGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGM_OK = 0,
    SGM_ERR_INVALID = -1,     /* null pointer, size or parameter out of range */
    SGM_ERR_UNSUPPORTED = -2, /* well-formed request the library does not handle */
    SGM_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed */
    SGM_ERR_WORKSPACE = -4    /* the workspace passed is smaller than required */
} sgm_status;

/* Parameters of one matching problem (Sec. II-B, eq. (7)-(8)). */
typedef struct {
    int32_t width, height; /* W, H >= 1, W * H * ndisp < 2^31, and < 2^30
                              when Cmax + P2 > 255 (uint16 per-path volumes;
                              larger ones give SGM_ERR_UNSUPPORTED)        */
    int32_t census;        /* census window side n: 3, 5 or 7 (Cmax = n*n-1) */
    int32_t ndisp;         /* window width w, 1..256                       */
    int32_t npaths;        /* 4 or 8                                       */
    int32_t p1, p2;        /* 0 <= P1 <= P2, 2*Cmax + 3*P2 < 16383 and
                              npaths * (Cmax + P2) <= 65535                 */
    uint32_t flags;        /* reserved, must be 0                          */
} sgm_params;

typedef struct sgm_plan_s *sgm_plan_t;

/* Launch choices (picked by sgm_autotune / sgm_batch_autotune or set by
 * hand; none of them changes results).
 *   lanes: lanes that carry one scanline of the aggregation's vertical
 *          and diagonal directions, each holding w / lanes (rounded up to a
 *          compiled count) consecutive window values, so that a wave of 64
 *          lanes advances 64 / lanes scanlines: 16 serves every window
 *          width; 8 and 4 serve widths up to 64 that are a multiple of the
 *          per-lane count (8: 4 or 8 values; 4: 4, 8, 12 or 16).  0 means
 *          16; a count that does not serve a width falls back to 16 (for
 *          the plan, or for that pair of a batch).  The horizontal
 *          directions always take 16 lanes per scanline, and the selection
 *          the fewest lanes per pixel that serve the width.
 *   order: plans: dispatch order of the aggregation's direction slots
 *          after the horizontal ones (0 diagonal then vertical, 1 vertical
 *          then diagonal); batches: queue order of the scanline groups (0
 *          longest first, 1 pair by pair, 2 direction by direction).
 *   waves_per_cu: batches only (ignored by plans): resident aggregation
 *          waves per compute unit, 1..32. */
typedef struct {
    int32_t waves_per_cu;
    int32_t order;
    int32_t lanes;
} sgm_tuning;

/* Validate `params` and build a plan (host only, touches no device).
 * On success *out owns host memory released by sgm_plan_free(). */
sgm_status sgm_plan(const sgm_params *params, sgm_plan_t *out);
void sgm_plan_free(sgm_plan_t plan);

/* sgm_plan with the launch choices tuning->lanes (0, 4, 8 or 16) and
 * tuning->order (0 or 1; other values: SGM_ERR_INVALID); the plan's results
 * are those of sgm_plan.  sgm_plan_get_tuning reports the lane count and
 * slot order the plan uses (waves_per_cu reads 0). */
sgm_status sgm_plan_tuned(const sgm_params *params, const sgm_tuning *tuning, sgm_plan_t *out);
sgm_status sgm_plan_get_tuning(sgm_plan_t plan, sgm_tuning *tuning);

/* Bytes of device workspace that sgm_cost, sgm_aggregate,
 * sgm_aggregate_wta and sgm_match need (one figure covers all of them).
 * The workspace must be 256-byte aligned; its contents need not persist
 * between calls. */
sgm_status sgm_workspace_size(sgm_plan_t plan, size_t *bytes);

/* Census codes of one image: codes[v * W + u] (device, uint64), bit b set
 * iff the b-th neighbour of the n x n window (row by row, centre skipped,
 * coordinates clamped to the image) is strictly darker than the centre. */
sgm_status sgm_census(sgm_plan_t plan, const uint8_t *image, int32_t pitch,
                      uint64_t *codes, void *stream);

/* Matching cost volume (device, uint8 [H][W][w]):
 *   C(u,v,k) = popcount(cL(u,v) XOR cR(u - d_lo[v] - k, v)),
 *   or Cmax where u - d_lo[v] - k < 0  (Sec. II-B with eq. (6)).
 * d_lo: device int32 [H] window starts, each >= 0, or NULL for all 0. */
sgm_status sgm_cost(sgm_plan_t plan, const uint8_t *left, const uint8_t *right,
                    int32_t pitch, const int32_t *d_lo, uint8_t *cost,
                    void *workspace, size_t workspace_bytes, void *stream);

/* Summed aggregated cost (device, uint16 [H][W][w]): S = sum_r L_r over the
 * plan's npaths directions (eq. (8), eq. (9)). */
sgm_status sgm_aggregate(sgm_plan_t plan, const uint8_t *cost, uint16_t *sum,
                         void *workspace, size_t workspace_bytes, void *stream);

/* One direction's aggregated cost L_r (device, uint16 [H][W][w]), for
 * testing and inspection; path in 0..7 (see the direction table above).
 * Being uint16, it needs W * H * ndisp < 2^30 (else SGM_ERR_UNSUPPORTED). */
sgm_status sgm_aggregate_path(sgm_plan_t plan, const uint8_t *cost, int32_t path,
                              uint16_t *L, void *stream);

/* Winner-take-all and sub-pixel step on a summed cost volume (eq. (9),
 * eq. (10)).  k* is the smallest k minimising S(p,k); disp_int[v*W+u] =
 * d_lo[v] + k* (device uint16 [H][W]).  If disp_sub is not NULL it receives
 * (float)(d_lo[v] + k*) + delta (device float [H][W]), where for
 * 0 < k* < w-1, delta = (S(k*-1) - S(k*+1)) / (2 (S(k*-1) - 2 S(k*) +
 * S(k*+1))) computed as one IEEE fp32 division of exact integers, and
 * delta = 0 otherwise.  d_lo may be NULL (all 0). */
sgm_status sgm_wta(sgm_plan_t plan, const uint16_t *sum, const int32_t *d_lo,
                   uint16_t *disp_int, float *disp_sub, void *stream);

/* sgm_aggregate followed by sgm_wta without materialising S: identical
 * outputs, less memory traffic. */
sgm_status sgm_aggregate_wta(sgm_plan_t plan, const uint8_t *cost,
                             const int32_t *d_lo, uint16_t *disp_int,
                             float *disp_sub, void *workspace,
                             size_t workspace_bytes, void *stream);

/* Layout of the per-direction aggregated costs that sgm_aggregate_paths
 * writes: npaths volumes [H][W][w] of elem_bytes each (1 when Cmax + P2 <=
 * 255, else 2), volume r starting volume_stride bytes after volume r-1
 * (a multiple of 256); total_bytes covers all of them. */
sgm_status sgm_path_volumes(sgm_plan_t plan, int32_t *elem_bytes, size_t *volume_stride,
                            size_t *total_bytes);

/* The aggregation step alone (eq. (8)): every direction's L_r in one
 * launch, written to `paths` (device, 256-byte aligned, layout from
 * sgm_path_volumes; volume r holds direction r). */
sgm_status sgm_aggregate_paths(sgm_plan_t plan, const uint8_t *cost, void *paths,
                               size_t paths_bytes, void *stream);

/* Selection on per-direction volumes (eq. (9), eq. (10)): S is summed on
 * the fly and never stored; outputs as for sgm_wta. */
sgm_status sgm_wta_paths(sgm_plan_t plan, const void *paths, const int32_t *d_lo,
                         uint16_t *disp_int, float *disp_sub, void *stream);

/* The whole path on one pair: census, cost, aggregation, selection and
 * sub-pixel step.  Identical outputs to sgm_cost + sgm_aggregate_wta; the
 * cost volume lives in the workspace. */
sgm_status sgm_match(sgm_plan_t plan, const uint8_t *left, const uint8_t *right,
                     int32_t pitch, const int32_t *d_lo, uint16_t *disp_int,
                     float *disp_sub, void *workspace, size_t workspace_bytes,
                     void *stream);

/* Pick the lane count and slot order for `params`: reuse the entry for
 * this device architecture and problem (W, H, w, census, paths, P1, P2)
 * from the text file `cache_path` (may be NULL) if it holds one, else run
 * sgm_match with every distinct (lane mapping, order) on the given buffers
 * (as for sgm_match; the outputs are overwritten), time each on `stream`
 * (one warm-up, best of three; the host waits), keep the fastest and
 * append it to the file.  *chosen (may be NULL) receives the result, for
 * sgm_plan_tuned. */
sgm_status sgm_autotune(const sgm_params *params, const uint8_t *left, const uint8_t *right,
                        int32_t pitch, const int32_t *d_lo, uint16_t *disp_int, float *disp_sub,
                        void *workspace, size_t workspace_bytes, void *stream,
                        const char *cache_path, sgm_tuning *chosen);

/* For callers that cannot allocate device memory (work under stream
 * capture, serving loops, harnesses that forbid hipMalloc): sgm_match with
 * its workspace in a library-owned device array of
 * SGM_NOALLOC_SCRATCH_BYTES bytes, so plans whose sgm_workspace_size() is at
 * most that (e.g. 320x240, 32 disparities, 4 paths: 13.5 MB) need no
 * workspace argument.  Same arguments and identical outputs as sgm_match.
 *   - Allocates nothing: no hipMalloc / hipFree, no memset, no copy; only
 *     the kernels of sgm_match are enqueued on `stream`.
 *   - Every device the library runs on holds its own copy of the array
 *     from the code object's load until the process ends; its device
 *     address is looked up on the first call made with that device current.
 *   - Every call on one device shares that device's array: calls that
 *     overlap on one device (several streams or threads) race and give
 *     undefined results; serialise them.  Nothing in the array needs to
 *     start at zero, and each call overwrites what the previous one left.
 *   - A plan needing more than SGM_NOALLOC_SCRATCH_BYTES of workspace gives
 *     SGM_ERR_WORKSPACE before anything is enqueued. */
#define SGM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sgm_status sgm_match_noalloc(sgm_plan_t plan, const uint8_t *left, const uint8_t *right,
                             int32_t pitch, const int32_t *d_lo, uint16_t *disp_int,
                             float *disp_sub, void *stream);

/* ------------------------------------------------------------------------
 * Per-pixel search windows in absolute disparity (the learned-window form).
 *
 * Pixel p searches the w disparities [lo(p), lo(p) + w), w = the plan's
 * ndisp, which must be <= 16; lo is a device int32 [H][W] map with
 * 0 <= lo(p) <= 256 - w (values outside give unspecified but memory-safe
 * results).  Volumes are [H][W][w] by window index j = d - lo(p).
 *   cost:        C(u,v,j) = popcount(cL(u,v) XOR cR(u - lo(u,v) - j, v)),
 *                Cmax where that column is < 0 (Sec. II-B).
 *   aggregation: eq. (8) in absolute disparity: with q = p - r,
 *                L(p,j) = C(p,j) + min(Lq(d), Lq(d-1)+P1, Lq(d+1)+P1,
 *                m_q+P2) - m_q at d = lo(p) + j, where Lq(d) is q's value at
 *                window index d - lo(q) and counts as infinite outside q's
 *                window, and m_q is the minimum over q's window.
 *   selection:   as sgm_wta on window indices; outputs lo(p) + k* (+ the
 *                parabola offset).
 * The workspace and path-volume layout are those of the plan.
 */
sgm_status sgm_cost_win(sgm_plan_t plan, const uint8_t *left, const uint8_t *right,
                        int32_t pitch, const int32_t *lo, uint8_t *cost /* 16-byte aligned */,
                        void *workspace, size_t workspace_bytes, void *stream);
sgm_status sgm_aggregate_win_paths(sgm_plan_t plan, const uint8_t *cost, const int32_t *lo,
                                   void *paths, size_t paths_bytes, void *stream);
sgm_status sgm_wta_win_paths(sgm_plan_t plan, const void *paths, const int32_t *lo,
                             uint16_t *disp_int, float *disp_sub, void *stream);
sgm_status sgm_match_win(sgm_plan_t plan, const uint8_t *left, const uint8_t *right,
                         int32_t pitch, const int32_t *lo, uint16_t *disp_int, float *disp_sub,
                         void *workspace, size_t workspace_bytes, void *stream);

/* Per-pixel-window SGM of nimg pairs of one size (the plan's) together:
 * census and cost of every pair, the aggregation of every pair and
 * direction in ONE launch (one scanline per lane, 16 window values in
 * registers), and the selection of every pair.  Results equal sgm_match_win
 * on each pair.  Needs ndisp = 16 and Cmax + P2 <= 255 (uint8 volumes),
 * else SGM_ERR_UNSUPPORTED.
 *   left, right   device uint8; pair i at + i * image_stride bytes, rows of
 *                 `pitch` bytes (image_stride >= pitch * H)
 *   lo            device int32 [nimg][H][W] window starts
 *   disp_int      device uint16 [nimg][H][W]; disp_sub float32 [nimg][H][W]
 *                 or NULL
 *   workspace     device, 256-byte aligned, sgm_workspace_size_win_batch()
 *                 bytes (pair i uses the i-th of nimg equal slices: the
 *                 plan's workspace, then its window starts as bytes, which
 *                 the aggregation reads instead of the int32 map).
 * Library-owned state: the horizontal directions are aggregated on a second
 * stream per device, created (non-blocking, default priority) on the first
 * call on that device and kept until the process ends; `stream` forks to it
 * and joins back through two library-owned events, so the call stays
 * ordered on `stream` like every other call.  The fork and join are
 * serialised by a process-wide mutex: concurrent callers (any thread, any
 * stream) run this call's enqueue one at a time, and their horizontal
 * passes queue on the one side stream. */
sgm_status sgm_workspace_size_win_batch(sgm_plan_t plan, int32_t nimg, size_t *bytes);
sgm_status sgm_match_win_batch(sgm_plan_t plan, const uint8_t *left, const uint8_t *right,
                               int32_t pitch, int64_t image_stride, const int32_t *lo,
                               int32_t nimg, uint16_t *disp_int, float *disp_sub, void *workspace,
                               size_t workspace_bytes, void *stream);

/* 4 x 4 box reduction of an 8-bit image (the coarse level of the
 * learned-window form): out is floor(H/4) x floor(W/4), row-major, each
 * value (sum of its 16 pixels + 8) / 16.  Device buffers; needs W, H >= 4. */
sgm_status sgm_downsample4(const uint8_t *image, int32_t width, int32_t height, int32_t pitch,
                           uint8_t *out, void *stream);
/* The same for nimg images image_stride bytes apart (>= pitch * height);
 * out holds the nimg results packed, [nimg][H/4][W/4]. */
sgm_status sgm_downsample4_batch(const uint8_t *images, int32_t width, int32_t height,
                                 int32_t pitch, int64_t image_stride, int32_t nimg, uint8_t *out,
                                 void *stream);

/* ------------------------------------------------------------------------
 * The search-window network (learned-window form) and its training.
 *
 * Four 3x3 convolutions with 16 channels, zero padding, ReLU after the
 * first three; bfloat16 weights and activations, float32 accumulation on
 * the matrix cores.  It runs on the quarter-resolution level: input channel
 * 0 = coarse disparity / 16, channel 1 = coarse left intensity / 255 - 1/2,
 * channel 2 = min(column - coarse disparity, 16) / 16 (distance of the
 * coarse match from the left border), channels 3..15 zero; output channel
 * 0 = window-centre offset (coarse pixels), channel 1 = confidence logit.
 * Where the confidence sigmoid(logit) exceeds the threshold tau the window
 * of a full-resolution pixel is centred on 4 * (coarse + offset); elsewhere
 * the pixel falls back to full-range SGM (its window, still needed by the
 * windowed aggregation of its neighbours, is centred on 4 * coarse).
 *
 * The network has no counterpart in the paper, whose windows come from the
 * road model of Sec. II-A (eq. (3), (6)); it predicts the same quantity
 * (a search window per pixel instead of per row) from the quarter-scale
 * full-range SGM result.
 *
 * Buffers (all device, caller-owned; n images of W x H at a time):
 *   params  float32 [sgm_cnn_num_params()]: per layer W[tap][co][ci], b[co],
 *           tap = (dy + 1) * 3 + (dx + 1)
 *   wf, wb  bfloat16 [4][9][16][16]: weights as [tap][co][ci] and
 *           [tap][ci][co] (written by sgm_cnn_pack_weights / sgm_cnn_adam)
 *   x0      bfloat16 NHWC [n][H][W][16] network input
 *   acts    bfloat16 [3][n][H][W][16] hidden activations (forward output,
 *           backward input)
 *   out     float32 NHWC [n][H][W][2] network output: the two channels
 *           used (centre offset, confidence logit) of the last layer's 16
 *   dy      bfloat16 NHWC [n][H][W][16] loss gradient w.r.t. the last
 *           layer's 16 outputs (zero beyond the first two)
 * Activations and dy must be 16-byte aligned.  Weight gradients are reduced
 * in a fixed order, so training is bitwise reproducible.
 */
int32_t sgm_cnn_num_params(void);
size_t sgm_cnn_scratch_bytes(int32_t width, int32_t height, int32_t nimg);
sgm_status sgm_cnn_pack_weights(const float *params, uint16_t *wf, uint16_t *wb, void *stream);
sgm_status sgm_cnn_prepare_input(const float *coarse_disp, const uint8_t *coarse_left, int32_t width,
                                 int32_t height, int32_t nimg, uint16_t *x0, void *stream);
sgm_status sgm_cnn_forward(const uint16_t *wf, const float *params, const uint16_t *x0, int32_t width,
                           int32_t height, int32_t nimg, uint16_t *acts, float *out, void *stream);
/* Inference form of sgm_cnn_forward: the same out, bit for bit, from one
 * launch that keeps the hidden activations on chip (no acts buffer; x0
 * and wf 8-byte aligned; at most 65535 images). */
sgm_status sgm_cnn_infer(const uint16_t *wf, const float *params, const uint16_t *x0, int32_t width,
                         int32_t height, int32_t nimg, float *out, void *stream);
/* Loss = mean over pixels of Huber(offset - (label - coarse)) + logistic
 * loss of the logit against [|offset - (label - coarse)| < 1]; writes dy
 * and adds the two loss terms to loss_sum[0..1] (may be NULL). */
sgm_status sgm_cnn_loss(const float *out, const float *coarse_disp, const float *label, int32_t width,
                        int32_t height, int32_t nimg, uint16_t *dy, float *loss_sum, void *stream);
/* Parameter gradient (float32 [num_params]) of the loss given dy. */
sgm_status sgm_cnn_backward(const uint16_t *wb, const uint16_t *x0, const uint16_t *acts,
                            const uint16_t *dy, int32_t width, int32_t height, int32_t nimg,
                            float *grad, void *scratch, size_t scratch_bytes, void *stream);
/* One bias-corrected Adam step (step >= 1) on params with moments m, v;
 * refreshes wf and wb. */
sgm_status sgm_cnn_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr,
                        float beta1, float beta2, float eps, uint16_t *wf, uint16_t *wb, void *stream);
/* Per-pixel window starts lo (int32 [H][W]) of width w for a full-range
 * search of ndisp disparities: lo = clamp(floor(centre + 1/2) - w/2, 0,
 * ndisp - w), full pixel (x, y) reading coarse pixel (min(x/4, Wc-1),
 * min(y/4, Hc-1)).  A pixel is confident when logit > log(tau / (1 - tau))
 * (tau <= 0: every pixel, tau >= 1: none).  A pixel that is not confident
 * falls back to the full range when its coarse match lies inside the right
 * image, x - 4 coarse >= fallback_margin (float32; INT32_MIN: always);
 * further left it sees a point outside the right camera's view, which no
 * disparity range can match, and it keeps its window.  Optional outputs (NULL to
 * skip): fallback_mask uint8 [H][W] (1 = falls back); row_stats int32
 * [3][H]: per row the number of fallback pixels, the leftmost and the
 * rightmost fallback column (W and -1 for a row without any); nfallback
 * uint32, the total.  The statistics are cleared by this call.
 * coarse_disp and cnn_out are [Hc][Wc] and [Hc][Wc][2] float32. */
sgm_status sgm_window_map(const float *coarse_disp, const float *cnn_out, int32_t coarse_width,
                          int32_t coarse_height, int32_t width, int32_t height, int32_t ndisp,
                          int32_t w, float conf_threshold, int32_t fallback_margin, int32_t *lo,
                          uint8_t *fallback_mask, int32_t *row_stats, uint32_t *nfallback, void *stream);
/* The same for nimg images at once: every buffer holds the images packed
 * one after another (coarse_disp [nimg][Hc][Wc], cnn_out [nimg][Hc][Wc][2],
 * lo and fallback_mask [nimg][H][W], row_stats [nimg][3][H], nfallback
 * [nimg]). */
sgm_status sgm_window_map_batch(const float *coarse_disp, const float *cnn_out,
                                int32_t coarse_width, int32_t coarse_height, int32_t width,
                                int32_t height, int32_t ndisp, int32_t w, float conf_threshold,
                                int32_t fallback_margin, int32_t nimg, int32_t *lo,
                                uint8_t *fallback_mask, int32_t *row_stats, uint32_t *nfallback,
                                void *stream);
/* The full-range fallback: the full-range SGM result of the rectangle rows
 * y0 .. y0+rows-1, columns x0 .. x0+cols-1 (band_int int16 / band_sub
 * float32, [rows][cols], band_sub may be NULL) replaces the windowed result
 * in disp_int / disp_sub ([height][width]) on the pixels of the rectangle
 * that fallback_mask marks.  Other pixels are left as they are. */
sgm_status sgm_fallback_merge(const uint8_t *fallback_mask, const int16_t *band_int,
                              const float *band_sub, int32_t width, int32_t height, int32_t y0,
                              int32_t rows, int32_t x0, int32_t cols, int16_t *disp_int,
                              float *disp_sub, void *stream);
/* The same for every rectangle of a batch of nframes frames in one launch.
 * rects: device int32 [nrects][6] = (frame, y0, rows, x0, cols, offset of
 * the rectangle's first element in band_int / band_sub), each band
 * [rows][cols] row-major; max_rows / max_cols bound every rectangle's rows
 * and columns (the launch covers them; larger ones are clipped to them).
 * fallback_mask, disp_int, disp_sub: [nframes][height][width]; band_len:
 * elements of the band arrays.  Rectangles of one frame must not overlap
 * (on shared pixels either result may land).  Entries outside the frames
 * or the band arrays are skipped. */
sgm_status sgm_fallback_merge_rects(const uint8_t *fallback_mask, const int32_t *rects, int32_t nrects,
                                    int32_t max_rows, int32_t max_cols, int32_t width, int32_t height,
                                    int32_t nframes, const int16_t *band_int, const float *band_sub,
                                    int64_t band_len, int16_t *disp_int, float *disp_sub, void *stream);
/* Training target at the coarse level: mean of each 4 x 4 block of a full-
 * resolution disparity map, divided by 4 (coarse pixels). */
sgm_status sgm_label_downsample4(const float *label, int32_t width, int32_t height, float *coarse,
                                 void *stream);

/* ------------------------------------------------------------------------
 * Batches: many pairs, of several sizes, matched together.
 *
 * A batch fixes the pairs (sizes and device buffers) at plan time.  A run
 * enqueues five launches for the whole batch: a queue reset, census and
 * cost of every pair, ONE persistent aggregation launch in which waves pull
 * scanline groups of every pair and direction from a shared queue (in the
 * order the tuning selects), and the selection of every pair.  Results are
 * identical to sgm_match on each pair.  Scratch (census codes, cost
 * volumes, per-direction volumes, descriptor tables, the queue counter)
 * lives in the caller's workspace.  One run at a time per workspace.
 */
typedef struct {
    int32_t width, height; /* W, H of this pair                               */
    int32_t ndisp;         /* window width w; must be a multiple of the lane
                              width (2, 4, 8, 12, 16 values for w up to 32,
                              64, 128, 192, 256); W * H * ndisp < 2^31, and
                              < 2^30 when Cmax + P2 > 255                  */
    int32_t pitch;         /* bytes between image rows, >= width             */
    const uint8_t *left, *right; /* device images [H][pitch]                 */
    const int32_t *d_lo;   /* device [H] window starts, or NULL for all 0    */
    uint16_t *disp_int;    /* device [H][W] output                           */
    float *disp_sub;       /* device [H][W] output, or NULL                  */
} sgm_pair;

typedef struct {
    int32_t census, npaths, p1, p2; /* shared by every pair, as in sgm_params */
    uint32_t flags;                 /* reserved, must be 0                    */
} sgm_batch_params;

typedef struct sgm_batch_s *sgm_batch_t;

/* Validate and lay out a batch (host; allocates pinned host memory for the
 * descriptor tables).  The pairs' buffers must stay valid while the batch
 * is used.  Every run and graph replay uploads the tables from that pinned
 * memory; sgm_batch_set_tuning (and the autotuner), sgm_batch_capture and
 * sgm_batch_free rewrite or release it, and the graph, only after the
 * device has finished every run and replay already enqueued (the host
 * blocks on the batch's last enqueued work). */
sgm_status sgm_batch_plan(const sgm_batch_params *params, const sgm_pair *pairs,
                          int32_t npairs, sgm_batch_t *out);
void sgm_batch_free(sgm_batch_t batch);
sgm_status sgm_batch_workspace_size(sgm_batch_t batch, size_t *bytes);
sgm_status sgm_batch_set_tuning(sgm_batch_t batch, const sgm_tuning *tuning);
sgm_status sgm_batch_get_tuning(sgm_batch_t batch, sgm_tuning *tuning);

/* Enqueue one run of the whole batch on `stream`. */
sgm_status sgm_batch_run(sgm_batch_t batch, void *workspace, size_t workspace_bytes,
                         void *stream);

/* One run like sgm_batch_run that also times its stages with HIP events
 * on `stream` and waits for them (host blocks): ms[0..3] receive the census,
 * cost, aggregation and selection times in milliseconds.  For measurement;
 * results are those of sgm_batch_run. */
sgm_status sgm_batch_run_timed(sgm_batch_t batch, void *workspace, size_t workspace_bytes,
                               void *stream, float *ms);

/* Record one run into a HIP graph owned by the batch (stream capture on
 * `stream`, which must not be the null stream), and replay it.  Changing
 * the tuning drops the graph. */
sgm_status sgm_batch_capture(sgm_batch_t batch, void *workspace, size_t workspace_bytes,
                             void *stream);
sgm_status sgm_batch_launch(sgm_batch_t batch, void *stream);

/* Pick the tuning: reuse the entry for this batch shape from the text file
 * `cache_path` (may be NULL) if it holds one, else time every candidate on
 * the device (synchronising `stream`), keep the fastest and append it to
 * the file.  A missing or unreadable cache falls back to timing; if timing
 * fails the default tuning stays.  *chosen (may be NULL) receives the
 * result. */
sgm_status sgm_batch_autotune(sgm_batch_t batch, void *workspace, size_t workspace_bytes,
                              void *stream, const char *cache_path, sgm_tuning *chosen);

/* ------------------------------------------------------------------------
 * Road model and disparity transformation (Sec. II-A, Sec. II-C).
 *
 * On the road the disparity of pixel (u, v) follows eq. (3),
 *   f(u, v) = a0 + a1 (cos(phi) (v - cy) - sin(phi) (u - cx)),
 * with the roll rotation about the image centre (cx, cy) = ((W-1)/2,
 * (H-1)/2).  sgm_road_fit_batch fits (a0, a1, phi) to disparity maps as
 * Sec. II-C does: for a fixed phi, eq. (11) gives the least-squares a and
 * eq. (12) the residual E0min(phi); phi minimises E0min.  E0min is a ratio
 * of two quadratic forms in (cos(phi), sin(phi)), so its minimum has a
 * closed form: the least-squares plane d ~ c + g_u u + g_v v through the
 * same pixels, read back as g_v = a1 cos(phi), g_u = -a1 sin(phi), with
 * phi in (-pi/2, pi/2] (E0min has period pi).
 *
 * Buffers: disparity maps float32 [nimg][H][W] (dense), masks uint8
 * [nimg][H][W] (dense), window starts int32 [nimg][H], fits
 * sgm_road_fit [nimg]; all device, caller-owned.
 */
typedef struct {
    double a0, a1, phi;  /* eq. (3); phi in radians, (-pi/2, pi/2] */
    double g_u, g_v;     /* the same plane's slopes: -a1 sin(phi), a1 cos(phi) */
    double e0min;        /* residual sum of squares at phi (eq. (12)) */
    double count;        /* pixels that entered the fit */
    int32_t status;      /* 0 fitted; 1 fewer than 3 pixels; 2 the pixels lie on
                            one image line (det of the (u, v) covariance
                            <= 1e-9 var(u) var(v)).  a0, a1, phi, g_u, g_v and
                            e0min are NaN unless 0 */
    int32_t reserved;
} sgm_road_fit;

/* Device scratch bytes of sgm_road_fit_batch for nimg maps of W x H. */
sgm_status sgm_road_workspace_size(int32_t width, int32_t height, int32_t nimg, size_t *bytes);
/* Fit of Sec. II-C to each of nimg disparity maps.  Pixel (u, v) (integer
 * column and row) enters its map's fit when its mask entry is non-zero
 * (mask NULL: every pixel), its disparity d is finite, d >= min_disp and
 * u - d >= margin, i.e. its match lies inside the right image with that
 * much room (compared in float64; pass -INFINITY for no bound; NaN is
 * invalid), and, when `prior` is given (fits of the same maps, e.g. from a
 * first call), |d - f_prior(u, v)| <= tol: the refit over the pixels that
 * lie on the first fit's road, which drops the background and other
 * outliers that bias a plain least-squares fit (tol >= 0, +INFINITY
 * allowed; no pixel of a map whose prior failed is selected; prior may be
 * the same array as fit).  Moments are accumulated in float64 in a fixed order, so the
 * result is deterministic.  workspace: device, 256-byte aligned, at least
 * sgm_road_workspace_size bytes.  The maps are read once (5 bytes per
 * pixel with a mask, 4 without). */
sgm_status sgm_road_fit_batch(const float *disp, const uint8_t *mask, int32_t width, int32_t height,
                              int32_t nimg, float min_disp, double margin, const sgm_road_fit *prior,
                              double tol, sgm_road_fit *fit, void *workspace, size_t workspace_bytes,
                              void *stream);
/* The curve E0min(phi) of eq. (12) (Fig. 3) over the pixels that
 * sgm_road_fit_batch would select with the same arguments: for each map and
 * each roll angle phi[j] (radians), the residual sum of squares of the
 * least-squares fit d ~ a0 + a1 y, y = cos(phi) v - sin(phi) u, computed
 * from the same float64 moments as S_dd - S_yd^2 / S_yy (centred sums).
 * NaN for a map with fewer than 2 selected pixels or where y is constant
 * over them (S_yy <= 1e-12 (S_uu + S_vv)).  phi: float64 [nphi], energy:
 * float64 [nimg][nphi], both device; 1 <= nphi <= 65536; workspace as for
 * sgm_road_fit_batch.  The minimum over phi is the fit's e0min at its phi. */
sgm_status sgm_road_energy_batch(const float *disp, const uint8_t *mask, int32_t width, int32_t height,
                                 int32_t nimg, float min_disp, double margin, const sgm_road_fit *prior,
                                 double tol, const double *phi, int32_t nphi, double *energy, void *workspace,
                                 size_t workspace_bytes, void *stream);
/* Per-row window starts for W x H frames from device-resident fits (the
 * device form of sgm_window_from_road below, with the plane's slopes in
 * place of a1 cos(phi) and -a1 sin(phi)).  With scale s the fits are of
 * maps at 1/s resolution (e.g. s = 4 for the 4x4 reduction): disparities
 * and centred coordinates both scale by s, so f(u, v) = s a0 + g_u (u - cx)
 * + g_v (v - cy) at full resolution; s = 1 for fits of W x H maps.
 *   mode 0: d_lo = max(0, floor(f(cx, v) + 1/2) - floor(w/2));
 *   mode 1: eq. (6), d_lo = max(0, floor(min over x = 0..W-1 of f(x, v) - delta)).
 * Values are clamped to [0, 32767]; rows of a map whose fit failed get 0. */
sgm_status sgm_road_window_batch(const sgm_road_fit *fit, int32_t width, int32_t height, int32_t nimg,
                                 int32_t w, int32_t mode, double delta, double scale, int32_t *d_lo,
                                 void *stream);
/* Per-pixel windows centred on the fitted road plane, for the windowed
 * calls (sgm_match_win_batch): lo(u, v) = max(0, floor(f(u, v) + 1/2) -
 * floor(w/2)) with f = scale a0 + g_u (u - cx) + g_v (v - cy) on W x H
 * frames (scale as in sgm_road_window_batch).  The plane carries the roll
 * of eq. (3), so a window follows the road across a row as well as down
 * the image; clamped to 32767; 0 on maps whose fit failed.  lo: int32
 * [nimg][H][W], device. */
sgm_status sgm_road_window_map_batch(const sgm_road_fit *fit, int32_t width, int32_t height, int32_t nimg,
                                     int32_t w, double scale, int32_t *lo, void *stream);
/* Disparity transformation of eq. (13): out = disp - f(u, v) + delta_dt per
 * pixel, in float64 rounded once to float32; NaN on maps whose fit failed.
 * out may equal disp (in place).  8 bytes of traffic per pixel. */
sgm_status sgm_disparity_transform_batch(const float *disp, const sgm_road_fit *fit, int32_t width,
                                         int32_t height, int32_t nimg, double delta_dt, float *out,
                                         void *stream);
/* Road region for maps without a hand-selected one (the paper selects its
 * road regions by hand): mask = 1 where the fitted road disparity
 * f(u, v) >= f_min (below the horizon line of the fit), u - f >= margin
 * (the road's match lies inside the right image: left of that band no
 * disparity can be measured) and the disparity is finite; 0 elsewhere and
 * on maps whose fit failed.  float64, f from the fit's slopes.  mask:
 * uint8 [nimg][H][W], device. */
sgm_status sgm_road_mask_batch(const float *disp, const sgm_road_fit *fit, int32_t width, int32_t height,
                               int32_t nimg, double f_min, double margin, uint8_t *mask, void *stream);

/* ------------------------------------------------------------------------
 * Pothole threshold and labelling (Sec. II-E, eq. (14), (15)) on
 * transformed disparity maps D2 (eq. (13)), pixel by pixel (the paper's
 * superpixel step is not part of the library).
 *
 * Each pixel p whose 3x3 neighbourhood lies inside the image, with p and
 * its 8 neighbours selected (mask entry non-zero, or mask NULL) and finite,
 * gives a vector g = [D2(p), sum of D2 over the 8 neighbours] (the sum in
 * float64, neighbours in row-major order).  Candidate thresholds are
 * t_r = lo + k b, b = (hi - lo) / nbins, k = 1 .. nbins - 1.  With the bin
 * indices i = clamp(floor((g0 - lo) / b), 0, nbins - 1) and
 * j = clamp(floor((g1 - 8 lo) / (8 b)), 0, nbins - 1) (float64), g is in
 * region 1 (foreground) for k when max(i, j) < k and in region 2
 * (background) when min(i, j) >= k: the split along the histogram's
 * diagonal, with the two mixed regions left out.  E2(k) of eq. (15) is
 * minimised over the k whose two regions are both non-empty (the smallest
 * k on a tie), and t_s = t_r - delta_PD (eq. (14)).
 *
 * Buffers: maps float32 [nimg][H][W], masks uint8 [nimg][H][W], labels
 * int32 [nimg][H][W], results sgm_pothole_threshold [nimg], E2 curves
 * float64 [nimg][nbins + 1] (entries 0 and nbins NaN); all device.
 */
typedef struct {
    double t_r, t_s;  /* eq. (14) */
    double e2;        /* E2 at t_r (eq. (15)) */
    double n1, n2;    /* vectors in regions 1 and 2 at t_r */
    int32_t k;        /* t_r = lo + k b; 0 when status != 0 */
    int32_t status;   /* 0 found; 1 no candidate has two non-empty regions
                         (t_r, t_s, e2 NaN) */
} sgm_pothole_threshold;

/* Device scratch bytes of sgm_pothole_threshold_batch. */
sgm_status sgm_pothole_workspace_size(int32_t nbins, int32_t nimg, size_t *bytes);
/* Threshold search per map.  2 <= nbins <= 512; lo < hi, finite;
 * delta_pd finite; e2_curve may be NULL.  workspace: device, 256-byte
 * aligned, at least sgm_pothole_workspace_size bytes; it is cleared by the
 * call itself.  E2 sums are float64 atomics, so their last bits may vary
 * from run to run; counts are exact. */
sgm_status sgm_pothole_threshold_batch(const float *d2, const uint8_t *mask, int32_t width, int32_t height,
                                       int32_t nimg, double lo, double hi, int32_t nbins, double delta_pd,
                                       sgm_pothole_threshold *result, double *e2_curve, void *workspace,
                                       size_t workspace_bytes, void *stream);
/* Pothole labels: pixels that are selected, finite and below t_s form
 * 8-connected components; each is labelled 1 + the smallest row-major
 * index (within its map) among its pixels, every other pixel 0.  Maps
 * whose threshold has status != 0 get no pothole pixels. */
sgm_status sgm_pothole_label_batch(const float *d2, const uint8_t *mask, int32_t width, int32_t height,
                                   int32_t nimg, const sgm_pothole_threshold *result, int32_t *labels,
                                   void *stream);
/* Removes the potholes that lie in a single superpixel, which Sec. III-B
 * counts as false detections: every component of `labels` (as written by
 * sgm_pothole_label_batch: 1 + root index, 0 elsewhere) whose pixels all
 * have the same entry in `superpixels` (int32 [nimg][H][W], e.g. the SLIC
 * labels of sgm_slic_batch) is set to 0, in place; the other components
 * keep their labels.  Both arrays device, dense. */
sgm_status sgm_pothole_prune_batch(const int32_t *superpixels, int32_t width, int32_t height, int32_t nimg,
                                   int32_t *labels, void *stream);

/* ------------------------------------------------------------------------
 * Superpixels on D2 (SLIC, Sec. II-D) and the superpixel-mean map D3
 * (Sec. II-E).
 *
 * Grid step S: K = ceil(W/S) * ceil(H/S) centres; centre k = j * ceil(W/S)
 * + i starts at (min(i S + S/2, W-1), min(j S + S/2, H-1)) (S/2 rounded
 * down) and moves to the first position of its 3x3 neighbourhood
 * (row-major) whose gradient G = (v(x+1,y) - v(x-1,y))^2 +
 * (v(x,y+1) - v(x,y-1))^2 (float64, coordinates clamped; +inf unless the
 * four pixels are used) is strictly below G at the start.  A pixel is used
 * when its mask entry is non-zero (mask NULL: all), its value is finite
 * and |v| < 2048; unused pixels get label -1 and D3 NaN.  Each of up to
 * `iters` rounds assigns every used pixel of grid cell (i, j) to the nearest of
 * the centres of cells (i+di, j+dj), |di|, |dj| <= 1, in index order, by
 * d = (v - v_c)^2 + ((x - x_c)^2 + (y - y_c)^2) w, w = (m / S)^2, float64
 * without fused multiply-add, first smallest wins; then every centre with
 * pixels moves to their mean position and mean value, the value mean taken
 * over v rounded to multiples of 2^-20 and summed exactly.  The rounds stop
 * when the residual between the previous and the updated centres has
 * converged (Sec. II-D): the residual of a round is the largest change
 * dv^2 + (dx^2 + dy^2) w of a centre with pixels (float64, no fused
 * multiply-add), and a map's rounds stop after the first whose residual is
 * <= tol^2.  tol = 0 stops only once no centre moves, which leaves every
 * result as if all `iters` rounds had run.  Labels are the last
 * assignment's centre indices; D3(p) = value of p's centre after the last
 * update (float32).  The result does not depend on the order of any sum,
 * so it is the same on every run.
 *
 * Buffers: maps float32 [nimg][H][W], mask uint8 [nimg][H][W] or NULL,
 * labels int32 [nimg][H][W], d3 float32 [nimg][H][W], centres float64
 * [nimg][K][3] (x, y, v after the last update), rounds int32 [nimg] (the
 * rounds each map ran) or NULL; all device.
 */
sgm_status sgm_slic_workspace_size(int32_t width, int32_t height, int32_t S, int32_t nimg, size_t *bytes);
/* 2 <= S <= 256, ceil(H/S) <= 65535, m finite and >= 0, 1 <= iters <= 100,
 * tol finite and >= 0.  workspace: device, 256-byte aligned, at least
 * sgm_slic_workspace_size bytes.  Every round's kernels are enqueued; those
 * of a map whose rounds have stopped return at once. */
sgm_status sgm_slic_batch(const float *d2, const uint8_t *mask, int32_t width, int32_t height, int32_t nimg,
                          int32_t S, double m, int32_t iters, double tol, int32_t *rounds, int32_t *labels,
                          float *d3, double *centres, void *workspace, size_t workspace_bytes, void *stream);

/* Per-row window starts from the road model of eq. (3),
 *   f(u,v) = a0 + a1 (cos(phi) (v - cy) - sin(phi) (u - cx)),
 * with (cx, cy) = ((W-1)/2, (H-1)/2) the centre of the roll rotation.
 * Host only; d_lo_host is a host int32 [H] array.
 *   mode 0: window of width w centred on the road disparity at the row
 *           centre: d_lo = max(0, floor(f(cx, v) + 1/2) - floor(w/2)).
 *   mode 1: the shift of eq. (6): d_lo = max(0, floor(min over
 *           x = 0..W-1 of f(x, v) - delta)). */
sgm_status sgm_window_from_road(double a0, double a1, double phi, int32_t width,
                                int32_t height, int32_t w, int32_t mode,
                                double delta, int32_t *d_lo_host);

/* Failure-handling tests: arm a one-shot injected failure.  kind 1: the
 * next call that would launch work returns SGM_ERR_HIP and enqueues
 * nothing; kind 2: the next batch plan fails its pinned-memory allocation
 * with SGM_ERR_HIP; 0 disarms.  The environment variable
 * SGM_FAULT_INJECT=launch|alloc arms the same at the library's first call. */
sgm_status sgm_debug_inject_fault(int32_t kind);

const char *sgm_status_str(sgm_status status);
const char *sgm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SGM_H */
