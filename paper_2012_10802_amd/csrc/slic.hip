// Superpixels on the transformed disparity map (SLIC, Sec. II-D) and the
// superpixel-mean map D3 (Sec. II-E).
//
// Grid step S, centres (i, j) on a ceil(W/S) x ceil(H/S) grid, each moved
// to the lowest-gradient position of its 3x3 neighbourhood; then up to
// `iters` rounds of
//   assignment: a pixel of grid cell (i, j) joins the nearest of the
//               centres of cells (i + di, j + dj), |di|, |dj| <= 1, by
//               d = (v - v_c)^2 + ((x - x_c)^2 + (y - y_c)^2) (m / S)^2;
//   update:     each centre moves to the mean position and value of its
//               pixels (values summed as integers in units of 2^-20, so the
//               mean does not depend on the order of the sums);
// the rounds stop once the residual between the previous and the updated
// centres has converged: after the first round whose largest centre change
// dv^2 + (dx^2 + dy^2) (m / S)^2 is <= tol^2 (per map; the later rounds'
// kernels find that round's residual and return at once).
// D3(p) is the value of p's centre after the last update.
//
// Kernels:
//   k_slic_init   one thread per centre: start position, gradient move,
//                 value; clears the centre's accumulators and the
//                 residuals of every round;
//   k_slic_cell   one wave per grid cell, four adjacent cells per
//                 workgroup: the nine candidate centres in LDS, each pixel of the cell assigned (float64, no fused
//                 multiply-add, first smallest in index order), its label
//                 written; sums for the cell's own centre in registers (most
//                 pixels), for the other eight in LDS, then int64 global
//                 atomics (exact, any order);
//   k_slic_update one thread per centre: means, accumulators cleared, the
//                 round's residual by a wave maximum and one atomic max
//                 per wave (non-negative float64 values order like their
//                 bit patterns);
//   k_slic_d3     one thread per pixel; the rounds run per map.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/sgm.h"
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr double kQScale = 1048576.0;  // 2^20
constexpr float kVMax = 2048.0f;

__device__ inline bool px_used(const float *d, const uint8_t *mask, size_t at)
{
    const float v = d[at];
    return (!mask || mask[at] != 0) & (fabsf(v) < kVMax);  // NaN fails the comparison
}

// G(x, y) of the centre move, +inf unless the four pixels are used.
__device__ inline double slic_gradient(const float *d, const uint8_t *mask, int W, int H, int x, int y)
{
#pragma clang fp contract(off)
    const int xp = min(x + 1, W - 1), xm = max(x - 1, 0), yp = min(y + 1, H - 1), ym = max(y - 1, 0);
    const size_t a = (size_t)y * W + xp, b = (size_t)y * W + xm, c = (size_t)yp * W + x, e = (size_t)ym * W + x;
    if (!(px_used(d, mask, a) & px_used(d, mask, b) & px_used(d, mask, c) & px_used(d, mask, e)))
        return __builtin_inf();
    const double gx = (double)d[a] - (double)d[b];
    const double gy = (double)d[c] - (double)d[e];
    return gx * gx + gy * gy;
}

// centres: [nimg][K][3] (x, y, v); acc: [nimg][K][4] int64 (count, sum x,
// sum y, sum of v in units of 2^-20); resid: [nimg][kSlicMaxRounds] float64
// bit patterns, the residual of each round.
__global__ void k_slic_init(const float *__restrict__ d2, const uint8_t *__restrict__ mask, int W, int H, int S,
                            int nx, int K, double *__restrict__ centres, long long *__restrict__ acc,
                            unsigned long long *__restrict__ resid)
{
    const int img = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t < kSlicMaxRounds; t += blockDim.x) resid[(size_t)img * kSlicMaxRounds + t] = 0ull;
    if (k >= K) return;
    const size_t off = (size_t)img * W * H;
    const float *d = d2 + off;
    const uint8_t *m = mask ? mask + off : nullptr;
    const int i = k % nx, j = k / nx;
    const int x0 = min(i * S + S / 2, W - 1), y0 = min(j * S + S / 2, H - 1);
    int bx = x0, by = y0;
    double best = slic_gradient(d, m, W, H, x0, y0);
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int x = x0 + dx, y = y0 + dy;
            if (x < 0 || x >= W || y < 0 || y >= H) continue;
            const double g = slic_gradient(d, m, W, H, x, y);
            if (g < best) {
                best = g;
                bx = x;
                by = y;
            }
        }
    const size_t at = (size_t)by * W + bx;
    double *c = centres + ((size_t)img * K + k) * 3;
    c[0] = (double)bx;
    c[1] = (double)by;
    c[2] = px_used(d, m, at) ? (double)d[at] : __builtin_nan("");
    long long *a = acc + ((size_t)img * K + k) * 4;
    a[0] = a[1] = a[2] = a[3] = 0;
}

__device__ inline long long wave_sum_ll(long long x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// true when the rounds of map `img` stopped before round t
__device__ inline bool slic_stopped(const unsigned long long *resid, int img, int t, double tol2)
{
    return t > 0 && __longlong_as_double((long long)resid[(size_t)img * kSlicMaxRounds + t - 1]) <= tol2;
}

// Four adjacent grid cells (4 blockIdx.x + wave, blockIdx.y) of map
// blockIdx.z per workgroup, one wave each: a row of the four cells is
// contiguous in memory, so the workgroup's loads fill whole cache lines on
// one CU.
constexpr int kSlicCellsPerGroup = 4;

__global__ __launch_bounds__(64 * kSlicCellsPerGroup) void k_slic_cell(
    const float *__restrict__ d2, const uint8_t *__restrict__ mask, int W, int H, int S, int nx, int ny, double w,
    const double *__restrict__ centres, unsigned long long *__restrict__ acc, int32_t *__restrict__ labels,
    const unsigned long long *__restrict__ resid, int t, double tol2)
{
#pragma clang fp contract(off)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ci = blockIdx.x * kSlicCellsPerGroup + wave, cj = blockIdx.y, img = blockIdx.z;
    if (slic_stopped(resid, img, t, tol2)) return;  // uniform over the workgroup
    const int K = nx * ny;
    // per wave: the nine candidate centres (LDS broadcast reads) and the
    // sums for the eight neighbouring ones
    __shared__ double cand[kSlicCellsPerGroup][9][3];
    __shared__ int cidx[kSlicCellsPerGroup][9];
    __shared__ unsigned long long lacc[kSlicCellsPerGroup][9][4];
    if (lane < 9) {
        const int i = ci + lane % 3 - 1, j = cj + lane / 3 - 1;
        const bool in = ci < nx && i >= 0 && i < nx && j >= 0 && j < ny;
        const int k = in ? j * nx + i : -1;
        cidx[wave][lane] = k;
        for (int q = 0; q < 3; ++q) cand[wave][lane][q] = 0.0;
        if (in)
            for (int q = 0; q < 3; ++q) cand[wave][lane][q] = centres[((size_t)img * K + k) * 3 + q];
    }
    if (lane < 36) lacc[wave][lane / 4][lane % 4] = 0ull;
    __syncthreads();
    if (ci < nx) {  // a wave past the last column of cells has nothing to do
        const size_t off = (size_t)img * W * H;
        const float *d = d2 + off;
        const uint8_t *m = mask ? mask + off : nullptr;
        int32_t *lab = labels + off;
        long long own_n = 0, own_x = 0, own_y = 0, own_q = 0;
        // pixel p = lane + 64 t of the cell at (column c, row r), stepped
        // without a division per pixel
        int c = lane % S, r = lane / S;
        const int dc_step = 64 % S, dr_step = 64 / S;
        for (int p = lane; p < S * S; p += 64) {
            const int x = ci * S + c, y = cj * S + r;
            c += dc_step;
            r += dr_step;
            if (c >= S) {
                c -= S;
                r += 1;
            }
            if (x >= W || y >= H) continue;
            const size_t at = (size_t)y * W + x;
            int best_s = -1;
            if (px_used(d, m, at)) {
                const double v = (double)d[at], xf = (double)x, yf = (double)y;
                double best = __builtin_inf();
                for (int s = 0; s < 9; ++s) {
                    if (cidx[wave][s] < 0) continue;
                    const double dv = v - cand[wave][s][2];
                    const double dx = xf - cand[wave][s][0], dy = yf - cand[wave][s][1];
                    const double ds2 = dx * dx + dy * dy;
                    const double dist = dv * dv + ds2 * w;
                    if (dist < best) {  // NaN (a centre without a value) never wins
                        best = dist;
                        best_s = s;
                    }
                }
            }
            lab[at] = best_s < 0 ? -1 : cidx[wave][best_s];
            if (best_s < 0) continue;
            const long long q = llrint((double)d[at] * kQScale);
            if (best_s == 4) {
                own_n += 1;
                own_x += x;
                own_y += y;
                own_q += q;
            } else {
                atomicAdd(&lacc[wave][best_s][0], 1ull);
                atomicAdd(&lacc[wave][best_s][1], (unsigned long long)x);
                atomicAdd(&lacc[wave][best_s][2], (unsigned long long)y);
                atomicAdd(&lacc[wave][best_s][3], (unsigned long long)q);
            }
        }
        own_n = wave_sum_ll(own_n);
        own_x = wave_sum_ll(own_x);
        own_y = wave_sum_ll(own_y);
        own_q = wave_sum_ll(own_q);
        if (lane == 0 && own_n > 0) {
            unsigned long long *a = acc + ((size_t)img * K + cidx[wave][4]) * 4;
            atomicAdd(&a[0], (unsigned long long)own_n);
            atomicAdd(&a[1], (unsigned long long)own_x);
            atomicAdd(&a[2], (unsigned long long)own_y);
            atomicAdd(&a[3], (unsigned long long)own_q);
        }
    }
    __syncthreads();  // the LDS sums of every wave are complete
    if (ci < nx && lane < 36) {
        const int sl = lane / 4, qq = lane % 4;
        if (sl != 4 && lacc[wave][sl][0] != 0ull)  // only in-grid candidates ever win
            atomicAdd(&acc[((size_t)img * K + cidx[wave][sl]) * 4 + qq], lacc[wave][sl][qq]);
    }
}

__global__ __launch_bounds__(64) void k_slic_update(int K, double w, double *__restrict__ centres,
                                                    long long *__restrict__ acc, unsigned long long *__restrict__ resid,
                                                    int t, double tol2)
{
#pragma clang fp contract(off)
    const int img = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (slic_stopped(resid, img, t, tol2)) return;  // nothing accumulated, nothing moves
    unsigned long long e = 0ull;  // this centre's change (+0.0 without pixels)
    if (k < K) {
        long long *a = acc + ((size_t)img * K + k) * 4;
        double *c = centres + ((size_t)img * K + k) * 3;
        if (a[0] > 0) {
            const double n = (double)a[0];
            const double x = (double)a[1] / n, y = (double)a[2] / n, v = ((double)a[3] / n) * (1.0 / kQScale);
            const double dx = x - c[0], dy = y - c[1], dv = v - c[2];
            e = (unsigned long long)__double_as_longlong(dv * dv + (dx * dx + dy * dy) * w);
            c[0] = x;
            c[1] = y;
            c[2] = v;
        }
        a[0] = a[1] = a[2] = a[3] = 0;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(e, off);
        e = o > e ? o : e;
    }
    if ((threadIdx.x & 63) == 0 && e != 0ull) atomicMax(&resid[(size_t)img * kSlicMaxRounds + t], e);
}

__global__ void k_slic_d3(int W, int H, int K, const double *__restrict__ centres,
                          const int32_t *__restrict__ labels, float *__restrict__ d3,
                          const unsigned long long *__restrict__ resid, int iters, double tol2,
                          int32_t *__restrict__ rounds)
{
    const int img = blockIdx.y;
    const int n = W * H;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (rounds && p == 0) {
        int r = iters;
        for (int t = 1; t < iters; ++t)
            if (slic_stopped(resid, img, t, tol2)) {
                r = t;
                break;
            }
        rounds[img] = r;
    }
    if (p >= n) return;
    const size_t at = (size_t)img * n + p;
    const int l = labels[at];
    d3[at] = l < 0 ? __builtin_nanf("") : (float)centres[((size_t)img * K + l) * 3 + 2];
}

}  // namespace

// [nimg][K][4] int64 accumulators, then [nimg][kSlicMaxRounds] residuals
size_t slic_workspace_bytes(int W, int H, int S, int nimg)
{
    const size_t K = (size_t)((W + S - 1) / S) * ((H + S - 1) / S);
    return K * nimg * 4 * sizeof(long long) + (size_t)nimg * kSlicMaxRounds * sizeof(unsigned long long);
}

hipError_t launch_slic(const float *d2, const uint8_t *mask, int W, int H, int nimg, int S, double m, int iters,
                       double tol, int32_t *rounds, int32_t *labels, float *d3, double *centres, void *ws,
                       hipStream_t s)
{
    const int nx = (W + S - 1) / S, ny = (H + S - 1) / S, K = nx * ny;
    long long *acc = static_cast<long long *>(ws);
    unsigned long long *resid = reinterpret_cast<unsigned long long *>(acc + (size_t)K * nimg * 4);
    const double t = m / S, w = t * t;
    const double tol2 = tol * tol;
    const dim3 cgrid((K + 63) / 64, nimg);
    k_slic_init<<<cgrid, 64, 0, s>>>(d2, mask, W, H, S, nx, K, centres, acc, resid);
    hipError_t e = hipGetLastError();
    for (int it = 0; it < iters && e == hipSuccess; ++it) {
        k_slic_cell<<<dim3((nx + kSlicCellsPerGroup - 1) / kSlicCellsPerGroup, ny, nimg), 64 * kSlicCellsPerGroup, 0,
                      s>>>(d2, mask, W, H, S, nx, ny, w, centres, reinterpret_cast<unsigned long long *>(acc), labels,
                           resid, it, tol2);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        k_slic_update<<<cgrid, 64, 0, s>>>(K, w, centres, acc, resid, it, tol2);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    const int n = W * H;
    k_slic_d3<<<dim3((n + 255) / 256, nimg), 256, 0, s>>>(W, H, K, centres, labels, d3, resid, iters, tol2, rounds);
    return hipGetLastError();
}

}  // namespace sgm
