// Per-pixel search windows in absolute disparity (the learned-window form).
//
// Pixel p searches the w <= 16 disparities [lo(p), lo(p) + w).  The cost is
// the census Hamming distance over that window; the path aggregation of
// eq. (8) runs in absolute disparity: stepping from q to p, the
// predecessor's window is re-indexed by s = lo(p) - lo(q), and values
// outside q's window count as the sentinel 0x3FFF, which never wins
// because m_q + P2 <= Cmax + 2 P2 < 0x3FFF.  Volumes are [H][W][w] by
// window index, as for the plain path.
//
// Lane mapping of the aggregation: one scanline per 16-lane DPP row, lane j
// holds window index j (one value per lane); the re-indexing is one
// ds_bpermute per neighbour offset (-1, 0, +1), which also covers the
// window edges.

#include "sgm_device.h"
#include "sgm_internal.h"

namespace sgm {
namespace {

using namespace dev;

// ---------------------------------------------------------------------------
// 4 x 4 box reduction: out = (sum of the block + 8) / 16

__global__ __launch_bounds__(256) void k_downsample4(const uint8_t *__restrict__ img, int W, int H, int pitch,
                                                     uint8_t *__restrict__ out)
{
    const int Wc = W / 4, Hc = H / 4;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= Wc || y >= Hc) return;
    uint32_t sum = 0;
#pragma unroll
    for (int dy = 0; dy < 4; ++dy) {
        const uint8_t *row = img + (size_t)(4 * y + dy) * pitch + 4 * x;
#pragma unroll
        for (int dx = 0; dx < 4; ++dx) sum += row[dx];
    }
    out[(size_t)y * Wc + x] = (uint8_t)((sum + 8) >> 4);
}

// ---------------------------------------------------------------------------
// windowed cost: C(u,v,j) = popcount(cL(u,v) ^ cR(u - lo(u,v) - j, v))

constexpr int kWinTile = 64;    // pixels of one row per workgroup
constexpr int kWinReach = 256;  // right columns reachable left of the tile

__global__ __launch_bounds__(64) void k_cost_win(const uint64_t *__restrict__ cl, const uint64_t *__restrict__ cr,
                                                 const int32_t *__restrict__ lo, int W, int H, int w, int cmax,
                                                 uint8_t *__restrict__ cost)
{
    __shared__ uint64_t s_cr[kWinTile + kWinReach];
    const int v = blockIdx.y, u0 = blockIdx.x * kWinTile;
    const int first = u0 - kWinReach;  // right column held in s_cr[0]
    for (int t = threadIdx.x; t < kWinTile + kWinReach; t += blockDim.x) {
        const int col = first + t;
        s_cr[t] = (col >= 0 && col < W) ? cr[(size_t)v * W + col] : 0ull;
    }
    __syncthreads();
    const int u = u0 + threadIdx.x;
    if (u >= W) return;
    const size_t pix = (size_t)v * W + u;
    const uint64_t a = cl[pix];
    const int l = lo[pix];
    uint32_t word[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int col = u - l - j;
        const int idx = col - first;
        uint32_t c = (uint32_t)cmax;
        if (j < w && col >= 0 && idx >= 0 && idx < kWinTile + kWinReach) c = (uint32_t)__popcll(a ^ s_cr[idx]);
        word[j / 4] |= c << (8 * (j % 4));
    }
    uint8_t *dst = cost + pix * w;
    if (w == 16) {
        *reinterpret_cast<uint4 *>(dst) = make_uint4(word[0], word[1], word[2], word[3]);
    } else {
        for (int j = 0; j < w; ++j) dst[j] = (uint8_t)(word[j / 4] >> (8 * (j % 4)));
    }
}

// ---------------------------------------------------------------------------
// windowed aggregation

struct WinParams {
    const uint8_t *cost;
    const int32_t *lo;
    void *out;
    long long vstride;
    int W, H, w;
    uint32_t p1, p2;
    int np;
    int paths[8];   // per dispatch slot: direction | output volume << 8
    int gstart[9];  // first workgroup of each slot
};

constexpr int kNoLo = -0x40000000;  // "no predecessor window yet"
constexpr uint32_t kInf1 = 0x3FFFu;

__device__ __forceinline__ uint32_t lane_pick(uint32_t v, int src_lane)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)v);
}

template <bool L8, int PF, int KIND>
__device__ __forceinline__ void agg_scan_win(const WinParams &a, __amdgpu_buffer_rsrc_t rc, __amdgpu_buffer_rsrc_t rl,
                                             __amdgpu_buffer_rsrc_t ro, int du, int dv, int g)
{
    const int lane = threadIdx.x & 15;
    const int lw = threadIdx.x >> 4;
    const int row_base = threadIdx.x & 0x30;  // first lane of this scanline in the wave
    const int W = a.W, H = a.H, w = a.w;
    const int lpw = blockDim.x >> 4;

    int I0 = 0, I1;
    int idx = g * lpw + lw;
    if constexpr (KIND == kHorizontal) {
        idx = min(idx, H - 1);
        I1 = W;
    } else if constexpr (KIND == kVertical) {
        idx = min(idx, W - 1);
        I1 = H;
    } else {
        I0 = 1 << 30;
        I1 = 0;
        for (int l = 0; l < lpw; ++l) {
            const Line t = line_geom(g * lpw + l, du, dv, W, H);
            if (t.i1 > t.i0) {
                I0 = min(I0, t.i0);
                I1 = max(I1, t.i1);
            }
        }
        if (I1 <= I0) return;
    }
    const Line ln = line_geom(idx, du, dv, W, H);
    const bool has = lane < w;
    // element offsets at step i: pixel = pix0 + i * pstep (lo map), value = pixel * w + lane
    const uint32_t pstep = (uint32_t)(ln.sv * W + ln.su);
    const uint32_t pix0 = (uint32_t)(ln.vb * W + ln.ub);
    const uint32_t li0 = (uint32_t)ln.i0, llen = (uint32_t)(ln.i1 - ln.i0);
    auto inside = [&](int i) -> bool {
        if constexpr (KIND == kDiagonal)
            return i < I1 && ((uint32_t)i - li0 < llen);
        else
            return i < I1;
    };

    uint32_t ring_c[PF], ring_l[PF];
#pragma unroll
    for (int s = 0; s < PF; ++s) {
        const int i = I0 + s;
        const uint32_t px = pix0 + (uint32_t)i * pstep;
        const bool in = inside(i);
        ring_c[s] = __builtin_amdgcn_raw_buffer_load_b8(rc, (in && has) ? px * (uint32_t)w + lane : kOff, 0, 0);
        ring_l[s] = __builtin_amdgcn_raw_buffer_load_b32(rl, in ? px * 4u : kOff, 0, 0);
    }
    uint32_t Lq = 0;
    int loq = kNoLo;
    const int nblk = (I1 - I0 + PF - 1) / PF;
    for (int blk = 0; blk < nblk; ++blk) {
#pragma unroll
        for (int s = 0; s < PF; ++s) {
            const int i = I0 + blk * PF + s;
            const bool act = inside(i);
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(1 + (PF - 1) * 3));
            const uint32_t c = ring_c[s];
            const int lop = (int)ring_l[s];
            {
                const int ip = i + PF;
                const uint32_t px = pix0 + (uint32_t)ip * pstep;
                const bool in = inside(ip);
                ring_c[s] =
                    __builtin_amdgcn_raw_buffer_load_b8(rc, (in && has) ? px * (uint32_t)w + lane : kOff, 0, 0);
                ring_l[s] = __builtin_amdgcn_raw_buffer_load_b32(rl, in ? px * 4u : kOff, 0, 0);
            }
            // m_q over the predecessor's window
            const uint32_t m = row_min16(has ? Lq : 0xFFFFu);
            // predecessor's values at absolute disparities lo(p) + lane + {-1, 0, +1}
            const int sh = (loq == kNoLo) ? 0 : lop - loq;
            const int src = lane + sh;
            uint32_t P0 = lane_pick(Lq, row_base + src);
            uint32_t Pm = lane_pick(Lq, row_base + src - 1);
            uint32_t Pp = lane_pick(Lq, row_base + src + 1);
            P0 = ((uint32_t)src < (uint32_t)w) ? P0 : kInf1;
            Pm = ((uint32_t)(src - 1) < (uint32_t)w) ? Pm : kInf1;
            Pp = ((uint32_t)(src + 1) < (uint32_t)w) ? Pp : kInf1;
            uint32_t t = min(Pm, Pp) + a.p1;
            t = min(min(t, P0), m + a.p2);
            const uint32_t Ln = (c + t - m) & 0xFFFFu;
            const uint32_t o = (act && has) ? (pix0 + (uint32_t)i * pstep) * (uint32_t)w + lane : kOff;
            if (L8)
                __builtin_amdgcn_raw_buffer_store_b8((unsigned char)Ln, ro, o, 0, kStreamPolicy);
            else
                __builtin_amdgcn_raw_buffer_store_b16((unsigned short)Ln, ro, o == kOff ? kOff : 2 * o, 0,
                                                      kStreamPolicy);
            Lq = Ln;
            loq = act ? lop : kNoLo;
        }
    }
}

template <bool L8, int PF>
__global__ __launch_bounds__(256) void k_aggregate_win(WinParams a)
{
    int slot = 0;
    while (slot + 1 < a.np && (int)blockIdx.x >= a.gstart[slot + 1]) ++slot;
    slot = __builtin_amdgcn_readfirstlane(slot);
    const int r = __builtin_amdgcn_readfirstlane(a.paths[slot] & 0xFF);
    const int vol = __builtin_amdgcn_readfirstlane(a.paths[slot] >> 8);
    const int g = __builtin_amdgcn_readfirstlane((int)blockIdx.x - a.gstart[slot]);
    const int du = __builtin_amdgcn_readfirstlane(dir_du(r)), dv = __builtin_amdgcn_readfirstlane(dir_dv(r));
    const uint32_t npix = (uint32_t)a.W * (uint32_t)a.H;
    const uint32_t nbytes = npix * (uint32_t)a.w;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cost, nbytes);
    const __amdgpu_buffer_rsrc_t rl = make_rsrc(a.lo, npix * 4u);
    const __amdgpu_buffer_rsrc_t ro =
        L8 ? make_rsrc(static_cast<const uint8_t *>(a.out) + (size_t)vol * a.vstride, nbytes)
           : make_rsrc(static_cast<const uint16_t *>(a.out) + (size_t)vol * a.vstride, nbytes * 2u);
    if (dv == 0) {
        __builtin_amdgcn_s_setprio(2);
        agg_scan_win<L8, PF, kHorizontal>(a, rc, rl, ro, du, dv, g);
    } else if (du == 0) {
        agg_scan_win<L8, PF, kVertical>(a, rc, rl, ro, du, dv, g);
    } else {
        agg_scan_win<L8, PF, kDiagonal>(a, rc, rl, ro, du, dv, g);
    }
}

// ---------------------------------------------------------------------------
// windowed selection: one thread per pixel, S summed SWAR style

template <bool L8>
__global__ __launch_bounds__(256) void k_wta_win(const void *__restrict__ vols, long long vstride, int np,
                                                 const int32_t *__restrict__ lo, int W, int H, int w,
                                                 uint16_t *__restrict__ dint, float *__restrict__ dsub)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= (long long)W * H) return;
    uint32_t S[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) S[j] = 0;
    if (L8 && w == 16) {
        uint32_t ev[4] = {0, 0, 0, 0}, od[4] = {0, 0, 0, 0};
        for (int r = 0; r < np; ++r) {
            const v4u x = __builtin_nontemporal_load(
                reinterpret_cast<const v4u *>(static_cast<const uint8_t *>(vols) + r * vstride + pix * 16));
            const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ev[q] += xs[q] & 0x00FF00FFu;
                od[q] += (xs[q] >> 8) & 0x00FF00FFu;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            S[4 * q] = ev[q] & 0xFFFFu;
            S[4 * q + 1] = od[q] & 0xFFFFu;
            S[4 * q + 2] = ev[q] >> 16;
            S[4 * q + 3] = od[q] >> 16;
        }
    } else {
        for (int r = 0; r < np; ++r)
            for (int j = 0; j < w; ++j)
                S[j] += L8 ? static_cast<const uint8_t *>(vols)[r * vstride + pix * w + j]
                           : static_cast<const uint16_t *>(vols)[r * vstride + pix * w + j];
    }
    int ks = 0;
    uint32_t s0 = S[0];
#pragma unroll
    for (int j = 1; j < 16; ++j)
        if (j < w && S[j] < s0) {
            s0 = S[j];
            ks = j;
        }
    uint32_t sm = 0, sp = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j == ks - 1) sm = S[j];
        if (j == ks + 1) sp = S[j];
    }
    const int l = lo[pix];
    dint[pix] = (uint16_t)(l + ks);
    if (dsub) {
        float delta = 0.0f;
        if (ks > 0 && ks < w - 1) {
            const int num = (int)sm - (int)sp;
            const int den = 2 * ((int)sm - 2 * (int)s0 + (int)sp);
            delta = __fdiv_rn((float)num, (float)den);
        }
        dsub[pix] = __fadd_rn((float)(l + ks), delta);
    }
}

constexpr int kWinPrefetch = 8;

}  // namespace

hipError_t launch_downsample4(const uint8_t *img, int W, int H, int pitch, uint8_t *out, hipStream_t s)
{
    dim3 grid((W / 4 + 63) / 64, (H / 4 + 3) / 4), block(256);
    hipLaunchKernelGGL(k_downsample4, grid, block, 0, s, img, W, H, pitch, out);
    return hipGetLastError();
}

hipError_t launch_cost_win(const Problem &pb, const uint64_t *cl, const uint64_t *cr, const int32_t *lo,
                           uint8_t *cost, hipStream_t s)
{
    dim3 grid((pb.W + kWinTile - 1) / kWinTile, pb.H), block(kWinTile);
    hipLaunchKernelGGL(k_cost_win, grid, block, 0, s, cl, cr, lo, pb.W, pb.H, pb.w, pb.cmax, cost);
    return hipGetLastError();
}

hipError_t launch_aggregate_win(const Problem &pb, const uint8_t *cost, const int32_t *lo, const int *paths, int np,
                                bool l8, void *out, long long vstride, hipStream_t s)
{
    WinParams p{};
    p.cost = cost;
    p.lo = lo;
    p.out = out;
    p.vstride = vstride;
    p.W = pb.W;
    p.H = pb.H;
    p.w = pb.w;
    p.p1 = (uint32_t)pb.p1;
    p.p2 = (uint32_t)pb.p2;
    p.np = np;
    const int lpw = 16;  // scanlines per 256-thread workgroup
    int no = 0, acc = 0;
    for (int kind = 0; kind < 3; ++kind)
        for (int i = 0; i < np; ++i) {
            const int r = paths[i];
            const int k = (r <= 1) ? 0 : (r >= 4 ? 1 : 2);
            if (k != kind) continue;
            const int nl = (r <= 1) ? pb.H : (r <= 3 ? pb.W : pb.W + pb.H - 1);
            p.paths[no] = r | (i << 8);
            p.gstart[no] = acc;
            acc += (nl + lpw - 1) / lpw;
            ++no;
        }
    p.gstart[np] = acc;
    if (l8) hipLaunchKernelGGL((k_aggregate_win<true, kWinPrefetch>), dim3(acc), dim3(256), 0, s, p);
    else hipLaunchKernelGGL((k_aggregate_win<false, kWinPrefetch>), dim3(acc), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_wta_win(const Problem &pb, const void *vols, long long vstride, int np, bool l8, const int32_t *lo,
                          uint16_t *dint, float *dsub, hipStream_t s)
{
    const long long npix = (long long)pb.W * pb.H;
    dim3 grid((unsigned)((npix + 255) / 256)), block(256);
    if (l8) hipLaunchKernelGGL(k_wta_win<true>, grid, block, 0, s, vols, vstride, np, lo, pb.W, pb.H, pb.w, dint, dsub);
    else hipLaunchKernelGGL(k_wta_win<false>, grid, block, 0, s, vols, vstride, np, lo, pb.W, pb.H, pb.w, dint, dsub);
    return hipGetLastError();
}

}  // namespace sgm
