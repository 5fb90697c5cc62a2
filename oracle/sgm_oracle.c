/*
 * Plain CPU oracle for the SGM hot path of the road-disparity pipeline
 * (Fan et al., "Rethinking Road Surface 3D Reconstruction and Pothole
 * Detection", Sec. II-A and II-B).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU baseline of
 * the benchmark do.  It shares no code, header, table or helper with the
 * HIP library.
 *
 * It is written to be read against the paper, not to be fast: every stage
 * is a direct loop over pixels and disparities, in the order the method
 * states it, with int32/int64 arithmetic and one IEEE fp32 division for the
 * sub-pixel step.  The only concession to speed is an OpenMP loop over the
 * independent path directions.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *  - matching cost c(p,d) (Sec. II-B, eq. (7)) is not specified: n x n
 *    census with Hamming distance is used;
 *  - census bit is set iff the neighbour is strictly darker than the
 *    centre; window coordinates are clamped at the image border; offsets
 *    are enumerated row by row (dy outer, dx inner), centre skipped;
 *  - a right-image column left of the image costs the maximum n*n-1;
 *  - the aggregation of eq. (8) additionally subtracts min_k L_r(p-r,k)
 *    (this shifts each L_r(p,.) by a constant, so the selected disparity
 *    and the sub-pixel offset are unchanged);
 *  - a path starts at the first pixel whose predecessor is outside the
 *    image, with L_r = C there; neighbour terms d+-1 outside the window
 *    are dropped;
 *  - "all directions" = 4 (+-x, +-y) or 8 (plus the four diagonals);
 *  - eq. (9) is read as an argmin, ties to the smallest disparity;
 *  - sub-pixel: parabola through S(k*-1), S(k*), S(k*+1), only for
 *    0 < k* < w-1;
 *  - perspective transformation (eq. (6), eq. (10)): the search window of
 *    row v starts at an integer d_lo(v) >= 0, the cost at window index k
 *    compares left column u with right column u - d_lo(v) - k, and the
 *    output disparity is d_lo(v) + k (+ sub-pixel offset).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

static int popcount64(uint64_t x)
{
    int c = 0;
    while (x) { c += (int)(x & 1u); x >>= 1; }
    return c;
}

/* ------------------------------------------------------------------ */
/* matching cost: census transform (reading of c(p,d), Sec. II-B)       */

/* code[v*W+u] = census bits of pixel (u,v) over an n x n window. */
int oracle_census(const uint8_t *img, int W, int H, int pitch, int n,
                  uint64_t *code)
{
    if (!img || !code || W < 1 || H < 1 || pitch < W || n < 3 || n > 7 || !(n & 1))
        return -1;
    int r = n / 2;
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            int centre = img[(size_t)v * pitch + u];
            uint64_t bits = 0;
            int b = 0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    int q = img[(size_t)clampi(v + dy, 0, H - 1) * pitch +
                                clampi(u + dx, 0, W - 1)];
                    if (q < centre) bits |= (uint64_t)1 << b;
                    ++b;
                }
            code[(size_t)v * W + u] = bits;
        }
    return 0;
}

/* cost[(v*W+u)*w+k] = Hamming distance between the left code at (u,v) and
 * the right code at (u - d_lo[v] - k, v); n*n-1 when that column is < 0.
 * d_lo == NULL means a zero window start on every row (plain SGM). */
int oracle_cost(const uint64_t *cl, const uint64_t *cr, int W, int H, int n,
                int w, const int32_t *d_lo, uint8_t *cost)
{
    if (!cl || !cr || !cost || W < 1 || H < 1 || w < 1 || w > 256) return -1;
    int cmax = n * n - 1;
    for (int v = 0; v < H; ++v) {
        int lo = d_lo ? d_lo[v] : 0;
        if (lo < 0) return -1;
        for (int u = 0; u < W; ++u)
            for (int k = 0; k < w; ++k) {
                int ur = u - lo - k;
                int c = ur >= 0 ? popcount64(cl[(size_t)v * W + u] ^ cr[(size_t)v * W + ur])
                                : cmax;
                cost[((size_t)v * W + u) * w + k] = (uint8_t)c;
            }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* path aggregation, eq. (8)                                            */

/* The R path directions r = (du, dv); the predecessor of p is p - r. */
static const int PATH_DU[8] = {+1, -1, 0, 0, +1, -1, +1, -1};
static const int PATH_DV[8] = {0, 0, +1, -1, +1, +1, -1, -1};

int oracle_path_dir(int path, int *du, int *dv)
{
    if (path < 0 || path > 7) return -1;
    *du = PATH_DU[path];
    *dv = PATH_DV[path];
    return 0;
}

/* Aggregated cost along direction (du,dv), normalised form:
 *   L(p,k) = C(p,k) + min(L(q,k), L(q,k-1)+P1, L(q,k+1)+P1, m_q+P2) - m_q,
 *   q = p - r,  m_q = min_i L(q,i).
 * Pixels are visited so that q is always finished before p: rows in the
 * direction of dv, columns in the direction of du. */
int oracle_path(const uint8_t *cost, int W, int H, int w, int du, int dv,
                int p1, int p2, uint16_t *L)
{
    if (!cost || !L || W < 1 || H < 1 || w < 1 || p1 < 0 || p2 < p1) return -1;
    if (du < -1 || du > 1 || dv < -1 || dv > 1 || (du == 0 && dv == 0)) return -1;
    for (int i = 0; i < H; ++i) {
        int v = dv >= 0 ? i : H - 1 - i;
        for (int j = 0; j < W; ++j) {
            int u = du >= 0 ? j : W - 1 - j;
            const uint8_t *c = cost + ((size_t)v * W + u) * w;
            uint16_t *out = L + ((size_t)v * W + u) * w;
            int qu = u - du, qv = v - dv;
            if (qu < 0 || qu >= W || qv < 0 || qv >= H) {
                for (int k = 0; k < w; ++k) out[k] = c[k];
                continue;
            }
            const uint16_t *prev = L + ((size_t)qv * W + qu) * w;
            int m = prev[0];
            for (int k = 1; k < w; ++k) if (prev[k] < m) m = prev[k];
            for (int k = 0; k < w; ++k) {
                int best = prev[k];
                if (k > 0 && prev[k - 1] + p1 < best) best = prev[k - 1] + p1;
                if (k + 1 < w && prev[k + 1] + p1 < best) best = prev[k + 1] + p1;
                if (m + p2 < best) best = m + p2;
                out[k] = (uint16_t)(c[k] + best - m);
            }
        }
    }
    return 0;
}

/* The literal recursion of eq. (8), without the -m_q term, in int64. */
int oracle_path_raw(const uint8_t *cost, int W, int H, int w, int du, int dv,
                    int p1, int p2, int64_t *U)
{
    if (!cost || !U || W < 1 || H < 1 || w < 1 || p1 < 0 || p2 < p1) return -1;
    if (du < -1 || du > 1 || dv < -1 || dv > 1 || (du == 0 && dv == 0)) return -1;
    for (int i = 0; i < H; ++i) {
        int v = dv >= 0 ? i : H - 1 - i;
        for (int j = 0; j < W; ++j) {
            int u = du >= 0 ? j : W - 1 - j;
            const uint8_t *c = cost + ((size_t)v * W + u) * w;
            int64_t *out = U + ((size_t)v * W + u) * w;
            int qu = u - du, qv = v - dv;
            if (qu < 0 || qu >= W || qv < 0 || qv >= H) {
                for (int k = 0; k < w; ++k) out[k] = c[k];
                continue;
            }
            const int64_t *prev = U + ((size_t)qv * W + qu) * w;
            int64_t m = prev[0];
            for (int k = 1; k < w; ++k) if (prev[k] < m) m = prev[k];
            for (int k = 0; k < w; ++k) {
                int64_t best = prev[k];
                if (k > 0 && prev[k - 1] + p1 < best) best = prev[k - 1] + p1;
                if (k + 1 < w && prev[k + 1] + p1 < best) best = prev[k + 1] + p1;
                if (m + p2 < best) best = m + p2;
                out[k] = c[k] + best;
            }
        }
    }
    return 0;
}

/* S(p,k) = sum over the first npaths directions of L_r(p,k)  (eq. (9)). */
int oracle_sum(const uint8_t *cost, int W, int H, int w, int npaths, int p1,
               int p2, uint32_t *S)
{
    if (!cost || !S || (npaths != 4 && npaths != 8)) return -1;
    size_t n = (size_t)W * H * w;
    uint16_t *Lr = (uint16_t *)malloc(n * sizeof(uint16_t) * (size_t)npaths);
    if (!Lr) return -2;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int r = 0; r < npaths; ++r)
        err |= oracle_path(cost, W, H, w, PATH_DU[r], PATH_DV[r], p1, p2, Lr + n * r) ? 1 : 0;
    if (!err) {
        memset(S, 0, n * sizeof(uint32_t));
        for (int r = 0; r < npaths; ++r)
            for (size_t i = 0; i < n; ++i) S[i] += Lr[n * r + i];
    }
    free(Lr);
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* disparity selection, sub-pixel step and eq. (10)                     */

int oracle_wta(const uint32_t *S, int W, int H, int w, const int32_t *d_lo,
               uint16_t *dint, float *dsub)
{
    if (!S || !dint || W < 1 || H < 1 || w < 1) return -1;
    for (int v = 0; v < H; ++v) {
        int lo = d_lo ? d_lo[v] : 0;
        for (int u = 0; u < W; ++u) {
            const uint32_t *s = S + ((size_t)v * W + u) * w;
            int best = 0;
            for (int k = 1; k < w; ++k) if (s[k] < s[best]) best = k;
            dint[(size_t)v * W + u] = (uint16_t)(lo + best);
            if (dsub) {
                float delta = 0.0f;
                if (best > 0 && best < w - 1) {
                    int sm = (int)s[best - 1], s0 = (int)s[best], sp = (int)s[best + 1];
                    int num = sm - sp;
                    int den = 2 * (sm - 2 * s0 + sp);
                    delta = (float)num / (float)den;
                }
                dsub[(size_t)v * W + u] = (float)(lo + best) + delta;
            }
        }
    }
    return 0;
}

/* Full path: census of both images, cost, aggregation, selection. */
int oracle_sgm(const uint8_t *left, const uint8_t *right, int W, int H, int pitch,
               int n, int w, int npaths, int p1, int p2, const int32_t *d_lo,
               uint16_t *dint, float *dsub)
{
    size_t np = (size_t)W * H, nv = np * (size_t)w;
    uint64_t *cl = (uint64_t *)malloc(np * sizeof(uint64_t));
    uint64_t *cr = (uint64_t *)malloc(np * sizeof(uint64_t));
    uint8_t *c = (uint8_t *)malloc(nv);
    uint32_t *S = (uint32_t *)malloc(nv * sizeof(uint32_t));
    int rc = -2;
    if (cl && cr && c && S) {
        rc = oracle_census(left, W, H, pitch, n, cl);
        if (!rc) rc = oracle_census(right, W, H, pitch, n, cr);
        if (!rc) rc = oracle_cost(cl, cr, W, H, n, w, d_lo, c);
        if (!rc) rc = oracle_sum(c, W, H, w, npaths, p1, p2, S);
        if (!rc) rc = oracle_wta(S, W, H, w, d_lo, dint, dsub);
    }
    free(cl); free(cr); free(c); free(S);
    return rc;
}

/* ------------------------------------------------------------------ */
/* per-row search window from the road model (eq. (3), eq. (6))        */

/* Road disparity of eq. (3) at pixel (u, v), with the roll rotation taken
 * about the image centre. */
static double road_disp(double a0, double a1, double phi, double u, double v,
                        int W, int H)
{
    double cx = (W - 1) / 2.0, cy = (H - 1) / 2.0;
    return a0 + a1 * (cos(phi) * (v - cy) - sin(phi) * (u - cx));
}

/* mode 0 (centred): window of width w centred on the road disparity at the
 *   row centre, d_lo = max(0, floor(f + 1/2) - floor(w/2)).
 * mode 1 (eq. (6)): d_lo = max(0, floor(min over x = 0..W-1 of f(x, v) - delta)). */
int oracle_window_from_road(double a0, double a1, double phi, int W, int H,
                            int w, int mode, double delta, int32_t *d_lo)
{
    if (!d_lo || W < 1 || H < 1 || w < 1 || (mode != 0 && mode != 1)) return -1;
    double cx = (W - 1) / 2.0;
    for (int v = 0; v < H; ++v) {
        double lo;
        if (mode == 0) {
            lo = floor(road_disp(a0, a1, phi, cx, v, W, H) + 0.5) - (double)(w / 2);
        } else {
            double k = road_disp(a0, a1, phi, 0, v, W, H) - delta;
            for (int x = 1; x < W; ++x) {
                double t = road_disp(a0, a1, phi, x, v, W, H) - delta;
                if (t < k) k = t;
            }
            lo = floor(k);
        }
        d_lo[v] = lo > 0.0 ? (int32_t)lo : 0;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* per-pixel windows in absolute disparity (learned-window form)        */
/*
 * Every pixel p has its own window of w disparities [lo(p), lo(p) + w).
 * The cost is taken over that window; the aggregation of eq. (8) is
 * written in absolute disparity, a predecessor's values outside its own
 * window counting as infinite (so those neighbour terms drop out and the
 * m_q + P2 term keeps the result finite).  L is stored by window index
 * j = d - lo(p).  lo is int32 [H][W], every entry >= 0.
 */

#define ORACLE_INF ((int64_t)1 << 40)

int oracle_cost_win(const uint64_t *cl, const uint64_t *cr, int W, int H, int n, int w,
                    const int32_t *lo, uint8_t *cost)
{
    if (!cl || !cr || !lo || !cost || W < 1 || H < 1 || w < 1 || w > 256) return -1;
    int cmax = n * n - 1;
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            int l = lo[(size_t)v * W + u];
            if (l < 0) return -1;
            for (int j = 0; j < w; ++j) {
                int ur = u - l - j;
                cost[((size_t)v * W + u) * w + j] =
                    (uint8_t)(ur >= 0 ? popcount64(cl[(size_t)v * W + u] ^ cr[(size_t)v * W + ur]) : cmax);
            }
        }
    return 0;
}

int oracle_path_win(const uint8_t *cost, const int32_t *lo, int W, int H, int w, int du, int dv,
                    int p1, int p2, uint16_t *L)
{
    if (!cost || !lo || !L || W < 1 || H < 1 || w < 1 || p1 < 0 || p2 < p1) return -1;
    if (du < -1 || du > 1 || dv < -1 || dv > 1 || (du == 0 && dv == 0)) return -1;
    for (int i = 0; i < H; ++i) {
        int v = dv >= 0 ? i : H - 1 - i;
        for (int jx = 0; jx < W; ++jx) {
            int u = du >= 0 ? jx : W - 1 - jx;
            const uint8_t *c = cost + ((size_t)v * W + u) * w;
            uint16_t *out = L + ((size_t)v * W + u) * w;
            int qu = u - du, qv = v - dv;
            if (qu < 0 || qu >= W || qv < 0 || qv >= H) {
                for (int k = 0; k < w; ++k) out[k] = c[k];
                continue;
            }
            const uint16_t *prev = L + ((size_t)qv * W + qu) * w;
            int lp = lo[(size_t)v * W + u], lq = lo[(size_t)qv * W + qu];
            int64_t m = prev[0];
            for (int k = 1; k < w; ++k) if (prev[k] < m) m = prev[k];
            for (int k = 0; k < w; ++k) {
                int d = lp + k;  /* absolute disparity */
                int64_t at[3];   /* L(q, d - 1), L(q, d), L(q, d + 1) */
                for (int e = -1; e <= 1; ++e) {
                    int jq = d + e - lq;
                    at[e + 1] = (jq >= 0 && jq < w) ? (int64_t)prev[jq] : ORACLE_INF;
                }
                int64_t best = at[1];
                if (at[0] + p1 < best) best = at[0] + p1;
                if (at[2] + p1 < best) best = at[2] + p1;
                if (m + p2 < best) best = m + p2;
                out[k] = (uint16_t)(c[k] + best - m);
            }
        }
    }
    return 0;
}

int oracle_sgm_win(const uint8_t *left, const uint8_t *right, int W, int H, int pitch, int n, int w,
                   int npaths, int p1, int p2, const int32_t *lo, uint16_t *dint, float *dsub)
{
    if (!lo || (npaths != 4 && npaths != 8)) return -1;
    size_t np = (size_t)W * H, nv = np * (size_t)w;
    uint64_t *cl = (uint64_t *)malloc(np * sizeof(uint64_t));
    uint64_t *cr = (uint64_t *)malloc(np * sizeof(uint64_t));
    uint8_t *c = (uint8_t *)malloc(nv);
    uint32_t *S = (uint32_t *)calloc(nv, sizeof(uint32_t));
    uint16_t *Lr = (uint16_t *)malloc(nv * sizeof(uint16_t) * (size_t)npaths);
    int rc = -2;
    if (cl && cr && c && S && Lr) {
        rc = oracle_census(left, W, H, pitch, n, cl);
        if (!rc) rc = oracle_census(right, W, H, pitch, n, cr);
        if (!rc) rc = oracle_cost_win(cl, cr, W, H, n, w, lo, c);
        if (!rc) {
            int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
            for (int r = 0; r < npaths; ++r)
                err |= oracle_path_win(c, lo, W, H, w, PATH_DU[r], PATH_DV[r], p1, p2, Lr + nv * r) ? 1 : 0;
            rc = err ? -1 : 0;
        }
        if (!rc) {
            for (int r = 0; r < npaths; ++r)
                for (size_t i = 0; i < nv; ++i) S[i] += Lr[nv * r + i];
            /* selection on window indices, output lo(p) + k (+ parabola) */
            for (size_t pix = 0; pix < np; ++pix) {
                const uint32_t *s = S + pix * w;
                int best = 0;
                for (int k = 1; k < w; ++k) if (s[k] < s[best]) best = k;
                int l = lo[pix];
                dint[pix] = (uint16_t)(l + best);
                if (dsub) {
                    float delta = 0.0f;
                    if (best > 0 && best < w - 1) {
                        int sm = (int)s[best - 1], s0 = (int)s[best], sp = (int)s[best + 1];
                        delta = (float)(sm - sp) / (float)(2 * (sm - 2 * s0 + sp));
                    }
                    dsub[pix] = (float)(l + best) + delta;
                }
            }
        }
    }
    free(cl); free(cr); free(c); free(S); free(Lr);
    return rc;
}

/* 4 x 4 box reduction of an 8-bit image: each output pixel is the rounded
 * mean (sum + 8) / 16 of its block; blocks past the border are dropped
 * (output size floor(W/4) x floor(H/4)). */
int oracle_downsample4(const uint8_t *img, int W, int H, int pitch, uint8_t *out)
{
    if (!img || !out || W < 4 || H < 4 || pitch < W) return -1;
    int Wc = W / 4, Hc = H / 4;
    for (int y = 0; y < Hc; ++y)
        for (int x = 0; x < Wc; ++x) {
            int sum = 0;
            for (int dy = 0; dy < 4; ++dy)
                for (int dx = 0; dx < 4; ++dx) sum += img[(size_t)(4 * y + dy) * pitch + 4 * x + dx];
            out[(size_t)y * Wc + x] = (uint8_t)((sum + 8) / 16);
        }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the direction loop in oracle_sum (timing only; results do not
 * depend on it). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
