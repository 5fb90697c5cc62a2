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
//                    fixed order), 4-5 bytes read per pixel, HBM-bound;
//   k_road_solve     one wave per map: ordered reduction of the partials and
//                    the closed form;
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
constexpr int kTargetBlocks = 4096;

__device__ inline double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ inline bool selected(float d, float min_disp)
{
    return d >= min_disp && fabsf(d) <= 3.402823466e38f;  // finite and above the bound (NaN fails)
}

// Rows [v0, v0 + rows) of one map per workgroup.  Each thread keeps the
// sums that depend on u and d for the current row and folds them into its
// totals with that row's v.  VEC: four consecutive pixels per load (W % 4 == 0
// and 16-byte aligned maps).
template <bool VEC>
__global__ __launch_bounds__(kRoadThreads) void k_road_moments(const float *__restrict__ disp,
                                                                 const uint8_t *__restrict__ mask, int W,
                                                                 int H, int rows, int nblk, float min_disp,
                                                                 double *__restrict__ part)
{
    const int img = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
    const size_t base = (size_t)img * W * H;
    const int v0 = b * rows, v1 = min(H, v0 + rows);
    double acc[kMoments];
#pragma unroll
    for (int i = 0; i < kMoments; ++i) acc[i] = 0.0;

    for (int v = v0; v < v1; ++v) {
        const float *drow = disp + base + (size_t)v * W;
        const uint8_t *mrow = mask ? mask + base + (size_t)v * W : nullptr;
        double rn = 0.0, ru = 0.0, ruu = 0.0, rd = 0.0, rud = 0.0, rdd = 0.0;
        auto take = [&](int u, float df, bool m) {
            if (m && selected(df, min_disp)) {
                const double d = (double)df, uu = (double)u;
                rn += 1.0;
                ru += uu;
                ruu += uu * uu;
                rd += d;
                rud += uu * d;
                rdd += d * d;
            }
        };
        if (VEC) {
            for (int x = 4 * t; x < W; x += 4 * kRoadThreads) {
                const float4 d4 = *reinterpret_cast<const float4 *>(drow + x);
                uint32_t m4 = 0xFFFFFFFFu;
                if (mrow) m4 = *reinterpret_cast<const uint32_t *>(mrow + x);
                take(x + 0, d4.x, (m4 & 0xFFu) != 0);
                take(x + 1, d4.y, (m4 & 0xFF00u) != 0);
                take(x + 2, d4.z, (m4 & 0xFF0000u) != 0);
                take(x + 3, d4.w, (m4 & 0xFF000000u) != 0);
            }
        } else {
            for (int x = t; x < W; x += kRoadThreads) take(x, drow[x], !mrow || mrow[x] != 0);
        }
        const double vv = (double)v;
        acc[0] += rn;
        acc[1] += ru;
        acc[2] += vv * rn;
        acc[3] += ruu;
        acc[4] += vv * ru;
        acc[5] += vv * vv * rn;
        acc[6] += rd;
        acc[7] += rud;
        acc[8] += vv * rd;
        acc[9] += rdd;
    }

    __shared__ double red[kRoadThreads / 64][kMoments];
    const int lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int i = 0; i < kMoments; ++i) {
        const double s = wave_sum(acc[i]);
        if (lane == 0) red[wave][i] = s;
    }
    __syncthreads();
    if (t < kMoments) {
        double s = 0.0;
        for (int w = 0; w < kRoadThreads / 64; ++w) s += red[w][t];
        part[((size_t)img * nblk + b) * kMoments + t] = s;
    }
}

// One wave per map: lane l sums partials l, l + 64, ... in order, then a
// fixed butterfly; lane 0 solves.
__global__ __launch_bounds__(64) void k_road_solve(const double *__restrict__ part, int nblk, int W, int H,
                                                   sgm_road_fit *__restrict__ fit)
{
    const int img = blockIdx.x, lane = threadIdx.x;
    double m[kMoments];
#pragma unroll
    for (int i = 0; i < kMoments; ++i) m[i] = 0.0;
    for (int j = lane; j < nblk; j += 64) {
        const double *p = part + ((size_t)img * nblk + j) * kMoments;
#pragma unroll
        for (int i = 0; i < kMoments; ++i) m[i] += p[i];
    }
#pragma unroll
    for (int i = 0; i < kMoments; ++i) m[i] = wave_sum(m[i]);
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

__global__ __launch_bounds__(256) void k_road_window(const sgm_road_fit *__restrict__ fit, int W, int H, int w,
                                                     int mode, double delta, int32_t *__restrict__ d_lo)
{
    const int img = blockIdx.y, v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= H) return;
    const sgm_road_fit f = fit[img];
    int32_t out = 0;
    if (f.status == 0) {
        const double cx = 0.5 * (W - 1), cy = 0.5 * (H - 1);
        const double row = f.a0 + f.g_v * ((double)v - cy);
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

// eq. (13) over rows [v0, v0 + rows) of one map per workgroup.
template <bool VEC>
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
        // D2 = D1 - (a0 + g_v (v - cy) + g_u (u - cx)) + delta = D1 + (c0 - g_u u)
        const double c0 = delta - f.a0 - f.g_v * ((double)v - cy) + f.g_u * cx;
        const float *src = disp + base + (size_t)v * W;
        float *dst = out + base + (size_t)v * W;
        if (VEC) {
            for (int x = 4 * t; x < W; x += 4 * kRoadThreads) {
                const float4 d = *reinterpret_cast<const float4 *>(src + x);
                float4 r;
                r.x = ok ? (float)((double)d.x + (c0 - f.g_u * (double)(x + 0))) : __builtin_nanf("");
                r.y = ok ? (float)((double)d.y + (c0 - f.g_u * (double)(x + 1))) : __builtin_nanf("");
                r.z = ok ? (float)((double)d.z + (c0 - f.g_u * (double)(x + 2))) : __builtin_nanf("");
                r.w = ok ? (float)((double)d.w + (c0 - f.g_u * (double)(x + 3))) : __builtin_nanf("");
                *reinterpret_cast<float4 *>(dst + x) = r;
            }
        } else {
            for (int x = t; x < W; x += kRoadThreads)
                dst[x] = ok ? (float)((double)src[x] + (c0 - f.g_u * (double)x)) : __builtin_nanf("");
        }
    }
}

// Rows per workgroup so that a launch has about kTargetBlocks workgroups.
int road_rows(int H, int nimg)
{
    const long long want = (kTargetBlocks + nimg - 1) / nimg;
    const long long rows = (H + want - 1) / want;
    return (int)(rows < 1 ? 1 : rows);
}

bool vec_ok(const void *a, const void *b, const void *c, int W)
{
    auto al = [](const void *p) { return p == nullptr || ((uintptr_t)p & 15) == 0; };
    return W % 4 == 0 && al(a) && al(b) && al(c);
}

}  // namespace

size_t road_workspace_bytes(int W, int H, int nimg)
{
    (void)W;
    const int rows = road_rows(H, nimg);
    const size_t nblk = (size_t)((H + rows - 1) / rows);
    return nblk * (size_t)nimg * kMoments * sizeof(double);
}

hipError_t launch_road_fit(const float *disp, const uint8_t *mask, int W, int H, int nimg, float min_disp,
                           sgm_road_fit *fit, void *ws, hipStream_t s)
{
    const int rows = road_rows(H, nimg);
    const int nblk = (H + rows - 1) / rows;
    double *part = static_cast<double *>(ws);
    const dim3 grid(nblk, nimg);
    if (vec_ok(disp, mask, nullptr, W))
        k_road_moments<true><<<grid, kRoadThreads, 0, s>>>(disp, mask, W, H, rows, nblk, min_disp, part);
    else
        k_road_moments<false><<<grid, kRoadThreads, 0, s>>>(disp, mask, W, H, rows, nblk, min_disp, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_road_solve<<<nimg, 64, 0, s>>>(part, nblk, W, H, fit);
    return hipGetLastError();
}

hipError_t launch_road_window(const sgm_road_fit *fit, int W, int H, int nimg, int w, int mode, double delta,
                              int32_t *d_lo, hipStream_t s)
{
    const dim3 grid((H + 255) / 256, nimg);
    k_road_window<<<grid, 256, 0, s>>>(fit, W, H, w, mode, delta, d_lo);
    return hipGetLastError();
}

hipError_t launch_disp_transform(const float *disp, const sgm_road_fit *fit, int W, int H, int nimg,
                                 double delta, float *out, hipStream_t s)
{
    const int rows = road_rows(H, nimg);
    const dim3 grid((H + rows - 1) / rows, nimg);
    if (vec_ok(disp, out, nullptr, W))
        k_disp_transform<true><<<grid, kRoadThreads, 0, s>>>(disp, fit, W, H, rows, delta, out);
    else
        k_disp_transform<false><<<grid, kRoadThreads, 0, s>>>(disp, fit, W, H, rows, delta, out);
    return hipGetLastError();
}

}  // namespace sgm
