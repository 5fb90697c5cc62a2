// Pothole threshold and labelling on the transformed disparity map D2
// (Sec. II-E, eq. (14), (15)): the threshold from D2's vectors, the
// labelling of any map below it (D2 pixel by pixel, or the superpixel
// means D3).
//
// Vectors g = [D2(p), sum of D2 over the 8-neighbourhood] of pixels whose
// 3x3 neighbourhood is inside the image, selected and finite.  For a
// threshold index k (t_r = lo + k b) a vector with bin indices (i, j) is in
// region 1 when max(i, j) < k and in region 2 when min(i, j) >= k, so two
// 1-D histograms of per-bin sums (count, g0, g1, |g|^2), one over max(i, j)
// and one over min(i, j), give E2 of eq. (15) for every k by a prefix and a
// suffix sum.
//
// Kernels:
//   k_pd_clear    zero the histograms (a kernel, so a captured graph can
//                 replay it);
//   k_pd_hist     one thread per column of a strip of rows, a sliding 3x3
//                 window (three loads per pixel, the next row in flight),
//                 bins in float64, sums of a run of equal bins kept in
//                 registers, float64 LDS atomics into several copies of the
//                 histograms (road pixels crowd into few bins), one global
//                 atomic per bin and workgroup;
//   k_pd_select   one workgroup per map: prefix / suffix sums, E2 per k,
//                 the smallest k with minimal E2 among those with both
//                 regions non-empty, t_s = t_r - delta_PD;
//   k_pd_label_*  8-connected components of D2 < t_s by union-find with
//                 atomicMin on parent links (parents always point to a
//                 smaller index, so every find ends and the root of a
//                 component is its smallest index):
//                   local    per 32 x 32 tile, union-find in LDS over the
//                            edges inside the tile; every pixel points at
//                            its tile component's smallest pixel;
//                   union    the edges between tiles (only tile-border
//                            pixels have any), on the global forest;
//                   flatten  every pixel to its root;
//                   name     root + 1.
//                 Row-major order inside a tile agrees with the image's,
//                 so a tile component's root is its smallest image index
//                 and the global roots come out as in a pixel-level pass;
//   k_pd_prune_*  components lying in a single superpixel removed (Sec.
//                 III-B counts them as false detections): mark the roots of
//                 components with a pixel in another superpixel than the
//                 root's (sign bit of the root's label), drop the unmarked,
//                 clear the marks.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/sgm.h"
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr int kPdThreads = 256;
constexpr int kPdRows = 32;  // rows per histogram workgroup
constexpr int kPdSums = 4;   // count, g0, g1, |g|^2
constexpr int kPdCopies = 4;              // most LDS histogram copies per workgroup
constexpr size_t kPdLds = 65536;          // LDS bytes a workgroup may take

__device__ inline bool finite_f(float d) { return fabsf(d) <= 3.402823466e38f; }

// floor(x / d) clamped to [0, top], with x / d the correctly rounded float64
// quotient: the product with 1/d is within a few ulps of it, so its floor
// is taken unless the product lies that close to an integer, where the
// division itself decides.
__device__ inline int bin_index(double x, double d, double inv_d, double top)
{
    const double q = x * inv_d;
    const double f = floor(q);
    const double e = 8.0 * 2.220446049250313e-16 * fmax(fabs(q), 1.0);
    const double qq = (q - f < e || f + 1.0 - q < e) ? x / d : q;
    return (int)fmin(fmax(floor(qq), 0.0), top);
}

// One pending (key, sums) entry per histogram and thread: consecutive
// pixels of a column often share a bin, so their sums are added in
// registers and reach LDS only when the key changes.
struct BinCache {
    int key = -1;
    double c = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    __device__ void add(double *hist, int k, double g0, double g1, double sq)
    {
        if (k != key) {
            flush(hist);
            key = k;
        }
        if (k >= 0) {
            c += 1.0;
            s0 += g0;
            s1 += g1;
            s2 += sq;
        }
    }
    __device__ void flush(double *hist)
    {
        if (key >= 0) {
            atomicAdd(&hist[key * kPdSums + 0], c);
            atomicAdd(&hist[key * kPdSums + 1], s0);
            atomicAdd(&hist[key * kPdSums + 2], s1);
            atomicAdd(&hist[key * kPdSums + 3], s2);
        }
        key = -1;
        c = s0 = s1 = s2 = 0.0;
    }
};

__global__ void k_pd_clear(double *__restrict__ p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// Workgroup (bx, by, img): interior columns 1 + 256 bx + t, interior rows
// [1 + kPdRows by, ...).  hist: [nimg][2][nbins][4] (max-index histogram,
// then min-index histogram).  The workgroup keeps `copies` LDS copies of
// both histograms, lane l adding to copy l % copies: road pixels crowd into
// few bins, and the copies cut the lanes that collide on one LDS address.
__global__ __launch_bounds__(kPdThreads) void k_pd_hist(const float *__restrict__ d2,
                                                        const uint8_t *__restrict__ mask, int W, int H,
                                                        double lo, double b, int nbins, int copies,
                                                        double *__restrict__ hist)
{
    extern __shared__ double sh[];  // [copies][2][nbins][4]
    const int img = blockIdx.z, t = threadIdx.x;
    const int per = 2 * nbins * kPdSums;
    for (int i = t; i < copies * per; i += kPdThreads) sh[i] = 0.0;
    __syncthreads();
    double *mine = sh + (size_t)((t & 63) % copies) * per;

    const size_t base = (size_t)img * W * H;
    const int x = 1 + blockIdx.x * kPdThreads + t;
    const bool col = x <= W - 2;
    const int xc = col ? x : 1;  // loads of idle lanes stay in bounds (W, H >= 3 here)
    const int v0 = 1 + blockIdx.y * kPdRows, v1 = min(H - 1, v0 + kPdRows);
    float a[4][3];
    uint8_t m[4][3];  // mask bytes (1 without a mask); used only once the row is binned
    auto load_row = [&](int r, int v) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t at = base + (size_t)v * W + (xc - 1 + c);
            a[r][c] = d2[at];
            m[r][c] = mask ? mask[at] : (uint8_t)1;
        }
    };
    // rows v - 1, v, v + 1 in a[0..2]; row v + 2 is loaded into a[3] while
    // row v is binned
    load_row(0, v0 - 1);
    load_row(1, v0);
    load_row(2, v0 + 1);
    const double b8 = 8.0 * b, lo8 = 8.0 * lo, top = (double)(nbins - 1);
    const double inv_b = 1.0 / b, inv_b8 = 1.0 / b8;
    BinCache cmax, cmin;
    for (int v = v0; v < v1; ++v) {
        load_row(3, min(v + 2, H - 1));
        bool ok = col;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) ok = ok & (m[r][c] != 0) & finite_f(a[r][c]);
        int kmax = -1, kmin = -1;
        double g0 = 0.0, g1 = 0.0, sq = 0.0;
        if (ok) {
            // neighbours in row-major order, summed left to right in float64
            g1 = (double)a[0][0];
            g1 += (double)a[0][1];
            g1 += (double)a[0][2];
            g1 += (double)a[1][0];
            g1 += (double)a[1][2];
            g1 += (double)a[2][0];
            g1 += (double)a[2][1];
            g1 += (double)a[2][2];
            g0 = (double)a[1][1];
            sq = g0 * g0 + g1 * g1;
            const int i = bin_index(g0 - lo, b, inv_b, top);
            const int j = bin_index(g1 - lo8, b8, inv_b8, top);
            kmax = max(i, j);
            kmin = nbins + min(i, j);
        }
        cmax.add(mine, kmax, g0, g1, sq);
        cmin.add(mine, kmin, g0, g1, sq);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a[0][c] = a[1][c];
            m[0][c] = m[1][c];
            a[1][c] = a[2][c];
            m[1][c] = m[2][c];
            a[2][c] = a[3][c];
            m[2][c] = m[3][c];
        }
    }
    cmax.flush(mine);
    cmin.flush(mine);
    __syncthreads();
    double *gh = hist + (size_t)img * per;
    for (int i = t; i < 2 * nbins; i += kPdThreads) {
        double tot[kPdSums] = {0.0, 0.0, 0.0, 0.0};
        for (int c = 0; c < copies; ++c)
            for (int q = 0; q < kPdSums; ++q) tot[q] += sh[(size_t)c * per + i * kPdSums + q];
        if (tot[0] != 0.0)
            for (int q = 0; q < kPdSums; ++q) atomicAdd(&gh[i * kPdSums + q], tot[q]);
    }
}

__device__ inline double region_e2(const double *r)
{
    return r[0] > 0.0 ? r[3] - (r[1] * r[1] + r[2] * r[2]) / r[0] : 0.0;
}

// One workgroup per map: the 64 threads copy both histograms to LDS, then
// thread 0 scans (nbins <= 512).  LDS: h1 [nbins][4], suffix sums of h2
// [nbins + 1][4].
__global__ __launch_bounds__(64) void k_pd_select(const double *__restrict__ hist, int nbins, double lo, double b,
                                                  double delta_pd, sgm_pothole_threshold *__restrict__ out,
                                                  double *__restrict__ curve)
{
    extern __shared__ double lds[];
    const int img = blockIdx.x;
    const int per = nbins * kPdSums;
    double *h1 = lds, *suf = lds + per;
    const double *g = hist + (size_t)img * 2 * per;
    for (int i = threadIdx.x; i < 2 * per; i += 64) lds[i] = g[i];  // h1, then h2 where suf starts
    __syncthreads();
    if (threadIdx.x != 0) return;
    // suffix sums in place over h2: suf[k] = sum of h2[k .. nbins - 1], suf[nbins] = 0
    double run[kPdSums] = {0.0, 0.0, 0.0, 0.0};
    for (int k = nbins - 1; k >= 0; --k)
        for (int q = 0; q < kPdSums; ++q) {
            run[q] += suf[k * kPdSums + q];
            suf[k * kPdSums + q] = run[q];
        }
    for (int q = 0; q < kPdSums; ++q) suf[per + q] = 0.0;
    const double nan = __builtin_nan("");
    double pre[kPdSums] = {0.0, 0.0, 0.0, 0.0};
    int best = 0;
    double best_e = 0.0, bn1 = 0.0, bn2 = 0.0;
    double *cv = curve ? curve + (size_t)img * (nbins + 1) : nullptr;
    if (cv) cv[0] = cv[nbins] = nan;
    for (int k = 1; k < nbins; ++k) {
        for (int q = 0; q < kPdSums; ++q) pre[q] += h1[(k - 1) * kPdSums + q];
        const double *r2 = suf + k * kPdSums;
        const double e = region_e2(pre) + region_e2(r2);
        if (cv) cv[k] = e;
        if (pre[0] > 0.0 && r2[0] > 0.0 && (best == 0 || e < best_e)) {
            best = k;
            best_e = e;
            bn1 = pre[0];
            bn2 = r2[0];
        }
    }
    sgm_pothole_threshold r;
    r.k = best;
    r.status = best ? 0 : 1;
    r.t_r = best ? lo + best * b : nan;
    r.t_s = best ? r.t_r - delta_pd : nan;
    r.e2 = best ? best_e : nan;
    r.n1 = bn1;
    r.n2 = bn2;
    out[img] = r;
}

template <typename T>
__device__ inline int pd_find(const T *lab, int x)
{
    int p = lab[x];
    while (p != x) {
        x = p;
        p = lab[x];
    }
    return x;
}

// link the roots of a and c, the larger under the smaller; a failed link
// (the root gained a parent meanwhile) retries from the new, smaller value
template <typename T>
__device__ inline void pd_link(T *lab, int a, int c)
{
    a = pd_find(lab, a);
    c = pd_find(lab, c);
    while (a != c) {
        if (a < c) {
            const int old = atomicMin(&lab[c], a);
            if (old == c) break;
            c = pd_find(lab, old);
        } else {
            const int old = atomicMin(&lab[a], c);
            if (old == a) break;
            a = pd_find(lab, old);
        }
    }
}

constexpr int kLabTile = 32;                                        // tile side, a power of two
constexpr int kLabThreads = 256;
constexpr int kLabRowsPerPass = kLabThreads / kLabTile;             // 8
constexpr int kLabPasses = kLabTile * kLabTile / kLabThreads;       // 4

// Edges linked: a pixel's left and upper neighbours always, its upper-left
// one only when neither the upper nor the left neighbour is foreground, its
// upper-right one only when the upper one is not: a skipped diagonal joins
// pixels already joined through the upper (or left) neighbour, whose own
// left (or upper) edge is always linked, so the components are those of
// all 8-neighbour edges.
//
// One 32 x 32 tile per workgroup (tiles in row-major order along x, maps
// along y): foreground test, union-find in LDS over the tile's own edges,
// then every pixel's entry = the image index of its tile component's root
// (-1 off the foreground).
__global__ __launch_bounds__(kLabThreads) void k_pd_label_local(const float *__restrict__ d2,
                                                                const uint8_t *__restrict__ mask, int W, int H,
                                                                const sgm_pothole_threshold *__restrict__ thr,
                                                                int32_t *__restrict__ lab)
{
    __shared__ int t[kLabTile * kLabTile];
    const int img = blockIdx.y;
    const int ntx = (W + kLabTile - 1) / kLabTile;
    const int x0 = (int)(blockIdx.x % ntx) * kLabTile, y0 = (int)(blockIdx.x / ntx) * kLabTile;
    const size_t base = (size_t)img * W * H;
    const sgm_pothole_threshold r = thr[img];
    const int lx = threadIdx.x % kLabTile, ly0 = threadIdx.x / kLabTile;
#pragma unroll
    for (int k = 0; k < kLabPasses; ++k) {
        const int ly = ly0 + kLabRowsPerPass * k, l = ly * kLabTile + lx;
        const int x = x0 + lx, y = y0 + ly;
        bool fg = false;
        if (x < W && y < H) {
            const size_t at = base + (size_t)y * W + x;
            const float d = d2[at];
            fg = r.status == 0 && (!mask || mask[at] != 0) && finite_f(d) && (double)d < r.t_s;
        }
        t[l] = fg ? l : -1;
    }
    __syncthreads();
    // an entry's sign never changes after the barrier (links only lower
    // non-negative entries), so the foreground tests below are stable
#pragma unroll
    for (int k = 0; k < kLabPasses; ++k) {
        const int ly = ly0 + kLabRowsPerPass * k, l = ly * kLabTile + lx;
        if (t[l] < 0) continue;
        const bool left = lx > 0 && t[l - 1] >= 0;
        const bool up = ly > 0 && t[l - kLabTile] >= 0;
        if (left) pd_link(t, l, l - 1);
        if (up) {
            pd_link(t, l, l - kLabTile);
        } else if (ly > 0) {  // the diagonals matter only when the pixel above is background
            if (!left && lx > 0 && t[l - kLabTile - 1] >= 0) pd_link(t, l, l - kLabTile - 1);
            if (lx + 1 < kLabTile && t[l - kLabTile + 1] >= 0) pd_link(t, l, l - kLabTile + 1);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kLabPasses; ++k) {
        const int ly = ly0 + kLabRowsPerPass * k, l = ly * kLabTile + lx;
        const int x = x0 + lx, y = y0 + ly;
        if (x >= W || y >= H) continue;
        int v = -1;
        if (t[l] >= 0) {
            const int root = pd_find(t, l);
            v = (y0 + root / kLabTile) * W + x0 + root % kLabTile;
        }
        lab[base + (size_t)y * W + x] = v;
    }
}

constexpr int kLabBorder = 3 * kLabTile - 2;  // a tile's top row, left and right columns

// The edges between tiles, the same subset as inside them.  Only the pixels
// of a tile's top row and left and right columns have a preceding neighbour
// in another tile: one workgroup per tile, one thread per such pixel.
__global__ __launch_bounds__(128) void k_pd_label_union(int W, int H, int32_t *__restrict__ lab_all)
{
    const int i = threadIdx.x;
    if (i >= kLabBorder) return;
    const int img = blockIdx.y;
    const int ntx = (W + kLabTile - 1) / kLabTile;
    const int tx = i < kLabTile ? i : (i < 2 * kLabTile - 1 ? 0 : kLabTile - 1);
    const int ty = i < kLabTile ? 0 : (i < 2 * kLabTile - 1 ? i - (kLabTile - 1) : i - (2 * kLabTile - 2));
    const int x = (int)(blockIdx.x % ntx) * kLabTile + tx, y = (int)(blockIdx.x / ntx) * kLabTile + ty;
    if (x >= W || y >= H) return;
    int32_t *lab = lab_all + (size_t)img * W * H;
    const int p = y * W + x;
    if (lab[p] < 0) return;
    const bool left = x > 0 && lab[p - 1] >= 0;
    const bool up = y > 0 && lab[p - W] >= 0;
    if (left && tx == 0) pd_link(lab, p, p - 1);
    if (up) {
        if (ty == 0) pd_link(lab, p, p - W);
    } else if (y > 0) {
        if (!left && x > 0 && (tx == 0 || ty == 0) && lab[p - W - 1] >= 0) pd_link(lab, p, p - W - 1);
        if (x + 1 < W && (tx == kLabTile - 1 || ty == 0) && lab[p - W + 1] >= 0) pd_link(lab, p, p - W + 1);
    }
}

// Points every foreground pixel at its root.  Entries only ever move to
// another ancestor of the same root, so concurrent finds stay on the chain.
__global__ void k_pd_label_flatten(int W, int H, int32_t *__restrict__ lab_all)
{
    const int img = blockIdx.y;
    const int n = W * H;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t *lab = lab_all + (size_t)img * n;
    if (lab[p] >= 0) lab[p] = pd_find(lab, p);
}

// Final names: root + 1 on the foreground, 0 (from -1) elsewhere.  A kernel
// of its own: no find may run while the names change.
__global__ void k_pd_label_name(size_t n, int32_t *__restrict__ lab)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        lab[i] += 1;
}

// root label mark (the sign bit; labels are >= 0): the component spans
// several superpixels
constexpr int32_t kMulti = (int32_t)0x80000000u;
constexpr int32_t kName = 0x7FFFFFFF;

__global__ void k_pd_prune_mark(const int32_t *__restrict__ sp, size_t n, int npix, int32_t *__restrict__ lab)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int32_t l = lab[i] & kName;
        if (l == 0) continue;
        const size_t root = i - i % npix + (size_t)(l - 1);
        if (sp[i] != sp[root] && !(lab[root] & kMulti)) atomicOr(&lab[root], kMulti);
    }
}

// A root without the mark is dropped by its own thread; the others read its
// label before or after that, and see no mark either way.
__global__ void k_pd_prune_drop(size_t n, int npix, int32_t *__restrict__ lab)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int32_t l = lab[i] & kName;
        if (l == 0) continue;
        const size_t root = i - i % npix + (size_t)(l - 1);
        if (!(lab[root] & kMulti)) lab[i] = 0;
    }
}

__global__ void k_pd_prune_clear(size_t n, int32_t *__restrict__ lab)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        lab[i] &= kName;
}

}  // namespace

hipError_t launch_pothole_prune(const int32_t *superpixels, int W, int H, int nimg, int32_t *labels, hipStream_t s)
{
    const int npix = W * H;
    const size_t total = (size_t)npix * nimg;
    const unsigned blocks = (unsigned)((total + 255) / 256 < 8192 ? (total + 255) / 256 : 8192);
    k_pd_prune_mark<<<blocks, 256, 0, s>>>(superpixels, total, npix, labels);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_pd_prune_drop<<<blocks, 256, 0, s>>>(total, npix, labels);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_pd_prune_clear<<<blocks, 256, 0, s>>>(total, labels);
    return hipGetLastError();
}

size_t pothole_workspace_bytes(int nbins, int nimg)
{
    return (size_t)nimg * 2 * nbins * kPdSums * sizeof(double);
}

hipError_t launch_pothole_threshold(const float *d2, const uint8_t *mask, int W, int H, int nimg, double lo,
                                    double b, int nbins, double delta_pd, sgm_pothole_threshold *out,
                                    double *curve, void *ws, hipStream_t s)
{
    double *hist = static_cast<double *>(ws);
    const size_t n = (size_t)nimg * 2 * nbins * kPdSums;
    k_pd_clear<<<(unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), 256, 0, s>>>(hist, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (W >= 3 && H >= 3) {
        const dim3 grid((W - 2 + kPdThreads - 1) / kPdThreads, (H - 2 + kPdRows - 1) / kPdRows, nimg);
        const size_t one = 2 * (size_t)nbins * kPdSums * sizeof(double);
        int copies = 1;
        while (copies < kPdCopies && 2 * copies * one <= kPdLds) copies *= 2;
        k_pd_hist<<<grid, kPdThreads, copies * one, s>>>(d2, mask, W, H, lo, b, nbins, copies, hist);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_pd_select<<<nimg, 64, (2 * nbins + 1) * kPdSums * sizeof(double), s>>>(hist, nbins, lo, b, delta_pd, out,
                                                                              curve);
    return hipGetLastError();
}

hipError_t launch_pothole_label(const float *d2, const uint8_t *mask, int W, int H, int nimg,
                                const sgm_pothole_threshold *thr, int32_t *labels, hipStream_t s)
{
    const int n = W * H;
    const dim3 grid((n + 255) / 256, nimg);
    const dim3 tiles((unsigned)(((W + kLabTile - 1) / kLabTile) * ((H + kLabTile - 1) / kLabTile)), nimg);
    k_pd_label_local<<<tiles, kLabThreads, 0, s>>>(d2, mask, W, H, thr, labels);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_pd_label_union<<<tiles, 128, 0, s>>>(W, H, labels);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_pd_label_flatten<<<grid, 256, 0, s>>>(W, H, labels);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t total = (size_t)n * nimg;
    k_pd_label_name<<<(unsigned)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096), 256, 0, s>>>(total, labels);
    return hipGetLastError();
}

}  // namespace sgm
