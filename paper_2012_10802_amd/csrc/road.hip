// Road model fit (Sec. II-A eq. (3), Sec. II-C eq. (11), (12)), per-row
// windows from it (eq. (6)) and the disparity transformation (eq. (13)).
//
// The fit needs ten sums over the selected pixels: n, sum u, sum v,
// sum u^2, sum u v, sum v^2, sum d, sum u d, sum v d, sum d^2 (raw integer
// pixel coordinates).  From them the centred second moments give the
// least-squares plane d ~ c + g_u u + g_v v, which is the minimum of
// E0min(phi) over phi: with y = cos(phi) v - sin(phi) u, eq. (12) equals
// var(d) - cov(y, d)^2 / var(y) (sums over the pixels), and that ratio of
// quadratic forms in (-sin(phi), cos(phi)) peaks in the direction of
// C^-1 b, C the (u, v) covariance and b = cov((u, v), d).  So one HBM pass
// and a closed form replace the 1-D search.
//
// Kernels:
//   k_road_moments   one pass over the maps: per-block partial sums (float64,
//                    fixed order), 4-5 bytes read per pixel, HBM-bound
//                    (k_road_moments_vec: float4 loads, two rows in flight);
//   k_road_solve     one wave per map: ordered reduction of the partials and
//                    the closed form;
//   k_road_energy    one wave per map: the same reduction, then eq. (12) at
//                    each of a list of roll angles (the curve of Fig. 3);
//   k_road_window    one thread per row: window starts from the fit;
//   k_disp_transform eq. (13), float4 in and out, HBM-bound.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/sgm.h"
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr int kMoments = 10;  // n, su, sv, suu, suv, svv, sd, sud, svd, sdd
constexpr int kRoadThreads = 256;
constexpr int kTargetBlocks = 4096;  // workgroups per launch (rows per workgroup follow)

__device__ inline double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Selection of pixel (u, d): d finite, d >= min_disp and u - d >= margin,
// in float64 (exact: u and d convert exactly, and so does their
// difference); `lim` = u - margin.  NaN fails every comparison.
__device__ inline bool selected(double d, double min_disp, double lim)
{
    return (d >= min_disp) & (d <= lim) & (fabs(d) <= 3.4028234663852886e38);
}

// Optional prior fit of the same map: only pixels within `tol` of its road
// line, |d - f(u, v)| <= tol, are selected (none if the prior failed).
struct Prior {
    bool use, none;
    double gu, gv, base, tol, cy;
    __device__ Prior(const sgm_road_fit *p, int img, int W, int H, double t)
        : use(p != nullptr), none(false), gu(0.0), gv(0.0), base(0.0), tol(t), cy(0.5 * (H - 1))
    {
        if (use) {
            const sgm_road_fit f = p[img];
            none = f.status != 0;
            gu = f.g_u;
            gv = f.g_v;
            base = f.a0 - f.g_u * 0.5 * (W - 1);  // f(u, v) = base + g_v (v - cy) + g_u u
        }
    }
    __device__ double row(int v) const { return base + gv * ((double)v - cy); }
    __device__ bool near(double d, double frow, int u) const
    {
        return !use || (!none && fabs(d - (frow + gu * (double)u)) <= tol);
    }
};

// Block-wide sum of the ten moments (fixed order), written as this
// workgroup's partial.
__device__ inline void store_partial(const double (&acc)[kMoments], double *__restrict__ part)
{
    __shared__ double red[kRoadThreads / 64][kMoments];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int i = 0; i < kMoments; ++i) {
        const double s = wave_sum(acc[i]);
        if (lane == 0) red[wave][i] = s;
    }
    __syncthreads();
    if (t < kMoments) {
        double s = 0.0;
        for (int w = 0; w < kRoadThreads / 64; ++w) s += red[w][t];
        part[t] = s;
    }
}

// Folds one row's per-thread sums (u and d only) into the totals with the
// row's v.
__device__ inline void fold_row(double (&acc)[kMoments], double v, double rn, double ru, double ruu, double rd,
                                double rud, double rdd)
{
    acc[0] += rn;
    acc[1] += ru;
    acc[2] += v * rn;
    acc[3] += ruu;
    acc[4] += v * ru;
    acc[5] += v * v * rn;
    acc[6] += rd;
    acc[7] += rud;
    acc[8] += v * rd;
    acc[9] += rdd;
}

// Rows [v0, v0 + rows) of one map per workgroup, W % 4 == 0 and
// W <= 1024 K: thread t owns the float4 groups t + 256 k (k < K) of every
// row.  Two rows' loads (2 K float4 + 2 K mask words) are issued before any
// is used, at clamped in-bounds addresses, and pixels outside the rows or
// the row are dropped by the selection, so the body is straight-line code.
// Per-row sums of the selected pixels' count, u and u^2 are exact int32
// (at most 4 K pixels of u < 4096 per thread and row).
template <int K>
__global__ __launch_bounds__(kRoadThreads) void k_road_moments_vec(const float *__restrict__ disp,
                                                                     const uint8_t *__restrict__ mask, int W,
                                                                     int H, int rows, int nblk, double min_disp,
                                                                     double margin,
                                                                     const sgm_road_fit *__restrict__ prior,
                                                                     double tol, double *__restrict__ part)
{
    const int img = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
    const size_t base = (size_t)img * W * H;
    const int v0 = b * rows, v1 = min(H, v0 + rows);
    const Prior pr(prior, img, W, H, tol);
    double acc[kMoments];
#pragma unroll
    for (int i = 0; i < kMoments; ++i) acc[i] = 0.0;

    for (int v = v0; v < v1; v += 2) {
        float4 d4[2][K];
        uint32_t m4[2][K];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int vr = min(v + r, v1 - 1);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int x = min(4 * (t + kRoadThreads * k), W - 4);
                d4[r][k] = *reinterpret_cast<const float4 *>(disp + base + (size_t)vr * W + x);
                m4[r][k] = mask ? *reinterpret_cast<const uint32_t *>(mask + base + (size_t)vr * W + x)
                                : 0xFFFFFFFFu;
            }
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            if (v + r >= v1) break;
            int rn = 0, ru = 0, ruu = 0;
            double rd = 0.0, rud = 0.0, rdd = 0.0;
            const double frow = pr.row(v + r);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int x = 4 * (t + kRoadThreads * k);
                const bool in = x < W;
                const float dv[4] = {d4[r][k].x, d4[r][k].y, d4[r][k].z, d4[r][k].w};
                const double lim0 = (double)x - margin;
                double se = 0.0, we = 0.0;  // sum d and sum e d over the four pixels x + e
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double de = (double)dv[e];
                    const bool sel = in & (((m4[r][k] >> (8 * e)) & 0xFFu) != 0) &
                                     selected(de, min_disp, lim0 + (double)e) & pr.near(de, frow, x + e);
                    const double d = sel ? de : 0.0;
                    const int u = x + e;
                    rn += sel ? 1 : 0;
                    ru += sel ? u : 0;
                    ruu += sel ? u * u : 0;
                    se += d;
                    if (e) we += (double)e * d;
                    rdd += d * d;
                }
                rd += se;
                rud += (double)x * se + we;
            }
            fold_row(acc, (double)(v + r), (double)rn, (double)ru, (double)ruu, rd, rud, rdd);
        }
    }
    store_partial(acc, part + ((size_t)img * nblk + b) * kMoments);
}

// Any width, one pixel per load.
__global__ __launch_bounds__(kRoadThreads) void k_road_moments(const float *__restrict__ disp,
                                                               const uint8_t *__restrict__ mask, int W, int H,
                                                               int rows, int nblk, double min_disp, double margin,
                                                               const sgm_road_fit *__restrict__ prior, double tol,
                                                               double *__restrict__ part)
{
    const int img = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
    const size_t base = (size_t)img * W * H;
    const int v0 = b * rows, v1 = min(H, v0 + rows);
    const Prior pr(prior, img, W, H, tol);
    double acc[kMoments];
#pragma unroll
    for (int i = 0; i < kMoments; ++i) acc[i] = 0.0;

    for (int v = v0; v < v1; ++v) {
        const float *drow = disp + base + (size_t)v * W;
        const uint8_t *mrow = mask ? mask + base + (size_t)v * W : nullptr;
        double rn = 0.0, ru = 0.0, ruu = 0.0, rd = 0.0, rud = 0.0, rdd = 0.0;
        const double frow = pr.row(v);
        for (int x = t; x < W; x += kRoadThreads) {
            const double d = (double)drow[x], u = (double)x;
            if ((!mrow || mrow[x] != 0) && selected(d, min_disp, u - margin) && pr.near(d, frow, x)) {
                rn += 1.0;
                ru += u;
                ruu += u * u;
                rd += d;
                rud += u * d;
                rdd += d * d;
            }
        }
        fold_row(acc, (double)v, rn, ru, ruu, rd, rud, rdd);
    }
    store_partial(acc, part + ((size_t)img * nblk + b) * kMoments);
}

// The ten sums of map img: lane l adds partials l, l + 64, ... in order,
// then a fixed butterfly leaves the totals in every lane.
__device__ inline void reduce_moments(const double *__restrict__ part, int nblk, int img, int lane,
                                      double (&m)[kMoments])
{
#pragma unroll
    for (int i = 0; i < kMoments; ++i) m[i] = 0.0;
    for (int j = lane; j < nblk; j += 64) {
        const double *p = part + ((size_t)img * nblk + j) * kMoments;
#pragma unroll
        for (int i = 0; i < kMoments; ++i) m[i] += p[i];
    }
#pragma unroll
    for (int i = 0; i < kMoments; ++i) m[i] = wave_sum(m[i]);
}

// One wave per map: the sums, then lane 0 solves.
__global__ __launch_bounds__(64) void k_road_solve(const double *__restrict__ part, int nblk, int W, int H,
                                                   sgm_road_fit *__restrict__ fit)
{
    const int img = blockIdx.x, lane = threadIdx.x;
    double m[kMoments];
    reduce_moments(part, nblk, img, lane, m);
    if (lane != 0) return;

    sgm_road_fit f;
    const double nan = __builtin_nan("");
    f.a0 = f.a1 = f.phi = f.g_u = f.g_v = f.e0min = nan;
    f.count = m[0];
    f.status = 0;
    f.reserved = 0;
    const double n = m[0];
    if (n < 3.0) {
        f.status = 1;
    } else {
        const double mu = m[1] / n, mv = m[2] / n, md = m[6] / n;
        const double cuu = m[3] - m[1] * mu, cuv = m[4] - m[1] * mv, cvv = m[5] - m[2] * mv;
        const double cud = m[7] - m[1] * md, cvd = m[8] - m[2] * md, cdd = m[9] - m[6] * md;
        const double det = cuu * cvv - cuv * cuv;
        if (!(det > 1e-9 * cuu * cvv)) {
            f.status = 2;
        } else {
            const double gu = (cvv * cud - cuv * cvd) / det;
            const double gv = (cuu * cvd - cuv * cud) / det;
            double phi, a1;
            if (gv != 0.0) {
                phi = atan(-gu / gv);
                a1 = gv > 0.0 ? hypot(gu, gv) : -hypot(gu, gv);
            } else if (gu != 0.0) {
                phi = 1.5707963267948966;  // pi / 2
                a1 = -gu;
            } else {
                phi = 0.0;
                a1 = 0.0;
            }
            const double cx = 0.5 * (W - 1), cy = 0.5 * (H - 1);
            f.a0 = md + gu * (cx - mu) + gv * (cy - mv);
            f.a1 = a1;
            f.phi = phi;
            f.g_u = gu;
            f.g_v = gv;
            f.e0min = cdd - (gu * cud + gv * cvd);
        }
    }
    fit[img] = f;
}

// eq. (12) at roll angle phi[j] for every j: with y = cos(phi) v -
// sin(phi) u, E0min = S_dd - S_yd^2 / S_yy, where S are sums of centred
// products over the selected pixels (T = [1, y] projects d onto the
// constant and y).  NaN with fewer than 2 pixels or when y takes a single
// value over them (S_yy <= 1e-12 (S_uu + S_vv): T has rank 1).
__global__ __launch_bounds__(64) void k_road_energy(const double *__restrict__ part, int nblk,
                                                    const double *__restrict__ phi, int nphi,
                                                    double *__restrict__ energy)
{
    const int img = blockIdx.x, lane = threadIdx.x;
    double m[kMoments];
    reduce_moments(part, nblk, img, lane, m);
    const double n = m[0];
    const double nan = __builtin_nan("");
    double cuu = 0.0, cuv = 0.0, cvv = 0.0, cud = 0.0, cvd = 0.0, cdd = 0.0;
    if (n >= 2.0) {
        const double mu = m[1] / n, mv = m[2] / n, md = m[6] / n;
        cuu = m[3] - m[1] * mu;
        cuv = m[4] - m[1] * mv;
        cvv = m[5] - m[2] * mv;
        cud = m[7] - m[1] * md;
        cvd = m[8] - m[2] * md;
        cdd = m[9] - m[6] * md;
    }
    for (int j = lane; j < nphi; j += 64) {
        double e = nan;
        if (n >= 2.0) {
            double s, c;
            sincos(phi[j], &s, &c);
            const double syy = c * c * cvv - 2.0 * s * c * cuv + s * s * cuu;
            const double syd = c * cvd - s * cud;
            if (syy > 1e-12 * (cuu + cvv)) e = cdd - syd * syd / syy;
        }
        energy[(size_t)img * nphi + j] = e;
    }
}

__global__ __launch_bounds__(256) void k_road_window(const sgm_road_fit *__restrict__ fit, int W, int H, int w,
                                                     int mode, double delta, double scale,
                                                     int32_t *__restrict__ d_lo)
{
    const int img = blockIdx.y, v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= H) return;
    const sgm_road_fit f = fit[img];
    int32_t out = 0;
    if (f.status == 0) {
        const double cx = 0.5 * (W - 1), cy = 0.5 * (H - 1);
        // a fit of a map at 1/scale resolution: disparities and centred
        // coordinates both scale, so a0 scales and the slopes stay
        const double row = scale * f.a0 + f.g_v * ((double)v - cy);
        double lo;
        if (mode == 0) {
            lo = floor(row + 0.5) - (double)(w / 2);
        } else {
            // linear along the row: the minimum over x = 0..W-1 is at an end
            const double x = f.g_u < 0.0 ? (double)(W - 1) : 0.0;
            lo = floor(row + f.g_u * (x - cx) - delta);
        }
        if (lo > 0.0) out = lo < 32767.0 ? (int32_t)lo : 32767;  // NaN stays 0
    }
    d_lo[(size_t)img * H + v] = out;
}

// eq. (13) over rows [v0, v0 + rows) of one map per workgroup:
// D2 = D1 - (a0 + g_v (v - cy) + g_u (u - cx)) + delta = D1 + (c(v) - g_u u).
__device__ inline float transform_px(float d, double c, double gu, int u, bool ok)
{
    return ok ? (float)((double)d + (c - gu * (double)u)) : __builtin_nanf("");
}

// W % 4 == 0, W <= 1024 K: thread t owns float4 groups t + 256 k of every
// row; two rows' loads are issued before the first store.
template <int K>
__global__ __launch_bounds__(kRoadThreads) void k_disp_transform_vec(const float *__restrict__ disp,
                                                                       const sgm_road_fit *__restrict__ fit,
                                                                       int W, int H, int rows, double delta,
                                                                       float *__restrict__ out)
{
    const int img = blockIdx.y, t = threadIdx.x;
    const int v0 = blockIdx.x * rows, v1 = min(H, v0 + rows);
    const size_t base = (size_t)img * W * H;
    const sgm_road_fit f = fit[img];
    const bool ok = f.status == 0;
    const double cx = 0.5 * (W - 1), cy = 0.5 * (H - 1);
    for (int v = v0; v < v1; v += 2) {
        float4 d4[2][K];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int vr = min(v + r, v1 - 1);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int x = min(4 * (t + kRoadThreads * k), W - 4);
                d4[r][k] = *reinterpret_cast<const float4 *>(disp + base + (size_t)vr * W + x);
            }
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            if (v + r >= v1) break;
            const double c = delta - f.a0 - f.g_v * ((double)(v + r) - cy) + f.g_u * cx;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int x = 4 * (t + kRoadThreads * k);
                if (x < W) {
                    float4 o;
                    o.x = transform_px(d4[r][k].x, c, f.g_u, x + 0, ok);
                    o.y = transform_px(d4[r][k].y, c, f.g_u, x + 1, ok);
                    o.z = transform_px(d4[r][k].z, c, f.g_u, x + 2, ok);
                    o.w = transform_px(d4[r][k].w, c, f.g_u, x + 3, ok);
                    *reinterpret_cast<float4 *>(out + base + (size_t)(v + r) * W + x) = o;
                }
            }
        }
    }
}

// Any width, one pixel per access.
__global__ __launch_bounds__(kRoadThreads) void k_disp_transform(const float *__restrict__ disp,
                                                                 const sgm_road_fit *__restrict__ fit, int W,
                                                                 int H, int rows, double delta,
                                                                 float *__restrict__ out)
{
    const int img = blockIdx.y, t = threadIdx.x;
    const int v0 = blockIdx.x * rows, v1 = min(H, v0 + rows);
    const size_t base = (size_t)img * W * H;
    const sgm_road_fit f = fit[img];
    const bool ok = f.status == 0;
    const double cx = 0.5 * (W - 1), cy = 0.5 * (H - 1);
    for (int v = v0; v < v1; ++v) {
        const double c = delta - f.a0 - f.g_v * ((double)v - cy) + f.g_u * cx;
        for (int x = t; x < W; x += kRoadThreads)
            out[base + (size_t)v * W + x] = transform_px(disp[base + (size_t)v * W + x], c, f.g_u, x, ok);
    }
}

// Per-pixel windows centred on the road line: lo(u, v) = max(0,
// floor(f(u, v) + 1/2) - floor(w/2)), f of a fit at 1/scale resolution
// (a0 scaled), clamped to 32767; 0 for a failed fit.
__global__ __launch_bounds__(256) void k_road_window_map(const sgm_road_fit *__restrict__ fit, int W, int H, int w,
                                                         double scale, int32_t *__restrict__ lo)
{
    const int img = blockIdx.y;
    const int n = W * H;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const sgm_road_fit f = fit[img];
    const int v = p / W, u = p - v * W;
    int32_t out = 0;
    if (f.status == 0) {
        const double road = scale * f.a0 + f.g_v * ((double)v - 0.5 * (H - 1)) + f.g_u * ((double)u - 0.5 * (W - 1));
        const double l = floor(road + 0.5) - (double)(w / 2);
        if (l > 0.0) out = l < 32767.0 ? (int32_t)l : 32767;  // NaN stays 0
    }
    lo[(size_t)img * n + p] = out;
}

// Road region: f(u, v) >= f_min (below the horizon line of the fit),
// u - f >= margin (the road's match inside the right image) and the
// disparity finite (float64); 0 for a failed fit.
__global__ __launch_bounds__(256) void k_road_mask(const float *__restrict__ disp,
                                                   const sgm_road_fit *__restrict__ fit, int W, int H,
                                                   double f_min, double margin, uint8_t *__restrict__ mask)
{
    const int img = blockIdx.y;
    const int n = W * H;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const size_t at = (size_t)img * n + p;
    const sgm_road_fit f = fit[img];
    const int v = p / W, u = p - v * W;
    const double d = (double)disp[at];
    const double road = f.a0 + f.g_v * ((double)v - 0.5 * (H - 1)) + f.g_u * ((double)u - 0.5 * (W - 1));
    const bool in = f.status == 0 && road >= f_min && (double)u - road >= margin && fabs(d) <= 3.4028234663852886e38;
    mask[at] = in ? 1 : 0;
}

// Rows per workgroup so that a launch has about `target` workgroups.
int road_rows(int H, int nimg, int target)
{
    const long long want = (target + nimg - 1) / nimg;
    const long long rows = (H + want - 1) / want;
    return (int)(rows < 1 ? 1 : rows);
}

bool vec_ok(const void *a, const void *b, const void *c, int W)
{
    auto al = [](const void *p) { return p == nullptr || ((uintptr_t)p & 15) == 0; };
    return W % 4 == 0 && al(a) && al(b) && al(c);
}

}  // namespace

hipError_t launch_road_window_map(const sgm_road_fit *fit, int W, int H, int nimg, int w, double scale, int32_t *lo,
                                  hipStream_t s)
{
    const int n = W * H;
    k_road_window_map<<<dim3((n + 255) / 256, nimg), 256, 0, s>>>(fit, W, H, w, scale, lo);
    return hipGetLastError();
}

hipError_t launch_road_mask(const float *disp, const sgm_road_fit *fit, int W, int H, int nimg, double f_min,
                            double margin, uint8_t *mask, hipStream_t s)
{
    const int n = W * H;
    k_road_mask<<<dim3((n + 255) / 256, nimg), 256, 0, s>>>(disp, fit, W, H, f_min, margin, mask);
    return hipGetLastError();
}

size_t road_workspace_bytes(int W, int H, int nimg)
{
    (void)W;
    const int rows = road_rows(H, nimg, kTargetBlocks);
    const size_t nblk = (size_t)((H + rows - 1) / rows);
    return nblk * (size_t)nimg * kMoments * sizeof(double);
}

// The moments pass of the fit: per-block partial sums into ws; returns the
// number of blocks per map through nblk_out.
static hipError_t launch_moments(const float *disp, const uint8_t *mask, int W, int H, int nimg, float min_disp,
                                 double margin, const sgm_road_fit *prior, double tol, void *ws, hipStream_t s,
                                 int *nblk_out)
{
    const int rows = road_rows(H, nimg, kTargetBlocks);
    const int nblk = (H + rows - 1) / rows;
    *nblk_out = nblk;
    double *part = static_cast<double *>(ws);
    const dim3 grid(nblk, nimg);
    const bool vec = vec_ok(disp, mask, nullptr, W);
    if (vec && W <= 1024)
        k_road_moments_vec<1><<<grid, kRoadThreads, 0, s>>>(disp, mask, W, H, rows, nblk, min_disp, margin, prior, tol, part);
    else if (vec && W <= 2048)
        k_road_moments_vec<2><<<grid, kRoadThreads, 0, s>>>(disp, mask, W, H, rows, nblk, min_disp, margin, prior, tol, part);
    else if (vec && W <= 4096)
        k_road_moments_vec<4><<<grid, kRoadThreads, 0, s>>>(disp, mask, W, H, rows, nblk, min_disp, margin, prior, tol, part);
    else
        k_road_moments<<<grid, kRoadThreads, 0, s>>>(disp, mask, W, H, rows, nblk, min_disp, margin, prior, tol, part);
    return hipGetLastError();
}

hipError_t launch_road_fit(const float *disp, const uint8_t *mask, int W, int H, int nimg, float min_disp,
                           double margin, const sgm_road_fit *prior, double tol, sgm_road_fit *fit, void *ws,
                           hipStream_t s)
{
    int nblk = 0;
    hipError_t e = launch_moments(disp, mask, W, H, nimg, min_disp, margin, prior, tol, ws, s, &nblk);
    if (e != hipSuccess) return e;
    k_road_solve<<<nimg, 64, 0, s>>>(static_cast<const double *>(ws), nblk, W, H, fit);
    return hipGetLastError();
}

hipError_t launch_road_energy(const float *disp, const uint8_t *mask, int W, int H, int nimg, float min_disp,
                              double margin, const sgm_road_fit *prior, double tol, const double *phi, int nphi,
                              double *energy, void *ws, hipStream_t s)
{
    int nblk = 0;
    hipError_t e = launch_moments(disp, mask, W, H, nimg, min_disp, margin, prior, tol, ws, s, &nblk);
    if (e != hipSuccess) return e;
    k_road_energy<<<nimg, 64, 0, s>>>(static_cast<const double *>(ws), nblk, phi, nphi, energy);
    return hipGetLastError();
}

hipError_t launch_road_window(const sgm_road_fit *fit, int W, int H, int nimg, int w, int mode, double delta,
                              double scale, int32_t *d_lo, hipStream_t s)
{
    const dim3 grid((H + 255) / 256, nimg);
    k_road_window<<<grid, 256, 0, s>>>(fit, W, H, w, mode, delta, scale, d_lo);
    return hipGetLastError();
}

hipError_t launch_disp_transform(const float *disp, const sgm_road_fit *fit, int W, int H, int nimg,
                                 double delta, float *out, hipStream_t s)
{
    const int rows = road_rows(H, nimg, kTargetBlocks);
    const dim3 grid((H + rows - 1) / rows, nimg);
    const bool vec = vec_ok(disp, out, nullptr, W);
    if (vec && W <= 1024)
        k_disp_transform_vec<1><<<grid, kRoadThreads, 0, s>>>(disp, fit, W, H, rows, delta, out);
    else if (vec && W <= 2048)
        k_disp_transform_vec<2><<<grid, kRoadThreads, 0, s>>>(disp, fit, W, H, rows, delta, out);
    else if (vec && W <= 4096)
        k_disp_transform_vec<4><<<grid, kRoadThreads, 0, s>>>(disp, fit, W, H, rows, delta, out);
    else
        k_disp_transform<<<grid, kRoadThreads, 0, s>>>(disp, fit, W, H, rows, delta, out);
    return hipGetLastError();
}

}  // namespace sgm
