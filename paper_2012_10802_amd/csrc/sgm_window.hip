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

#include <mutex>

#include "sgm_device.h"
#include "sgm_internal.h"

namespace sgm {
namespace {

using namespace dev;

// ---------------------------------------------------------------------------
// 4 x 4 box reduction: out = (sum of the block + 8) / 16

__global__ __launch_bounds__(256) void k_downsample4(const uint8_t *__restrict__ img, int W, int H, int pitch,
                                                     uint8_t *__restrict__ out, long long img_stride)
{
    const int Wc = W / 4, Hc = H / 4;
    // image blockIdx.z of a stack (img_stride bytes apart; outputs packed)
    img += blockIdx.z * img_stride;
    out += (size_t)blockIdx.z * Wc * Hc;
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

// minimum / maximum over the 64 lanes of a wave (every lane active): the
// DPP reduction of each 16-lane row, then the four rows' results as scalars
__device__ __forceinline__ int wave_min(int x)
{
    const int u = (int)group_min<16>((uint32_t)x ^ 0x80000000u);  // signed order as unsigned
    const uint32_t m = min(min((uint32_t)__builtin_amdgcn_readlane(u, 0), (uint32_t)__builtin_amdgcn_readlane(u, 16)),
                           min((uint32_t)__builtin_amdgcn_readlane(u, 32), (uint32_t)__builtin_amdgcn_readlane(u, 48)));
    return (int)(m ^ 0x80000000u);
}
__device__ __forceinline__ int wave_max(int x)
{
    const int u = (int)group_max<16>((uint32_t)x ^ 0x80000000u);
    const uint32_t m = max(max((uint32_t)__builtin_amdgcn_readlane(u, 0), (uint32_t)__builtin_amdgcn_readlane(u, 16)),
                           max((uint32_t)__builtin_amdgcn_readlane(u, 32), (uint32_t)__builtin_amdgcn_readlane(u, 48)));
    return (int)(m ^ 0x80000000u);
}

// One row tile of 64 pixels per workgroup (one wave).  Only the right
// columns that the tile's windows reach are staged: [u0 - max lo - 15,
// u0 + 63 - min lo], clipped to the image and to the staging array.
__global__ __launch_bounds__(64) void k_cost_win(const uint64_t *__restrict__ cl, const uint64_t *__restrict__ cr,
                                                 const int32_t *__restrict__ lo, int W, int H, int w, int cmax,
                                                 uint8_t *__restrict__ cost, long long codes_pair,
                                                 long long pix_pair, long long cost_pair,
                                                 uint8_t *__restrict__ lo8)
{
    __shared__ uint64_t s_cr[kWinTile + kWinReach];
    // pair blockIdx.z of a batch (strides 0 for one pair)
    cl += blockIdx.z * codes_pair;
    cr += blockIdx.z * codes_pair;
    lo += blockIdx.z * pix_pair;
    cost += blockIdx.z * cost_pair;
    if (lo8) lo8 += blockIdx.z * cost_pair;  // (in the pair's workspace slice)
    const int v = blockIdx.y, u0 = blockIdx.x * kWinTile;
    const int first = u0 - kWinReach;  // right column held in s_cr[0]
    const int u = u0 + threadIdx.x;
    const bool act = u < W;
    const size_t pix = (size_t)v * W + u;
    const int l = act ? lo[pix] : 0;
    const int lmax = __builtin_amdgcn_readfirstlane(wave_max(act ? l : -0x7FFFFFFF - 1));
    const int lmin = __builtin_amdgcn_readfirstlane(wave_min(act ? l : 0x7FFFFFFF));
    // columns read below: u - l - j, j in [0, 16), of the active lanes, and
    // only those >= 0 inside the staging array (the rest cost cmax); columns
    // past the right edge hold 0
    const long long c0 = max(max((long long)u0 - lmax - 15, (long long)first), 0ll);
    const long long c1 = min((long long)u0 + kWinTile - 1 - lmin, (long long)u0 + kWinTile - 1);
    for (long long col = c0 + threadIdx.x; col <= c1; col += blockDim.x)
        s_cr[col - first] = col < W ? cr[(size_t)v * W + col] : 0ull;
    __syncthreads();
    if (!act) return;
    // byte copy of the window start for the batched aggregation (window
    // starts are at most 256 - w)
    if (lo8) lo8[pix] = (uint8_t)l;
    const uint64_t a = cl[pix];
    uint32_t word[4] = {0, 0, 0, 0};
    if (w == 16 && lmin >= 0 && lmax <= kWinReach - 16 && u0 - lmax - 15 >= 0) {
        // (uniform) every window value of the tile reads a staged column
        // inside the image: no checks
        const uint64_t *src = s_cr + (u - l - first);
#pragma unroll
        for (int j = 0; j < 16; ++j) word[j / 4] |= (uint32_t)__popcll(a ^ src[-j]) << (8 * (j % 4));
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int col = u - l - j;
            const int idx = col - first;
            uint32_t c = (uint32_t)cmax;
            if (j < w && col >= 0 && idx >= 0 && idx < kWinTile + kWinReach) c = (uint32_t)__popcll(a ^ s_cr[idx]);
            word[j / 4] |= c << (8 * (j % 4));
        }
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
constexpr int kWinPrefetch = 8;     // steps of cost prefetched by agg_scan_win
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
                                                 uint16_t *__restrict__ dint, float *__restrict__ dsub,
                                                 long long vol_pair, long long pix_pair)
{
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= (long long)W * H) return;
    // pair blockIdx.y of a batch (strides 0 for one pair); vol_pair in elements
    vols = static_cast<const uint8_t *>(vols) + blockIdx.y * vol_pair * (L8 ? 1 : 2);
    lo += blockIdx.y * pix_pair;
    dint += blockIdx.y * pix_pair;
    if (dsub) dsub += blockIdx.y * pix_pair;
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

// ---------------------------------------------------------------------------
// census of every image of a batch: grid z = image (left images, then right)

template <int N>
__global__ __launch_bounds__(256) void k_census_pairs(const uint8_t *__restrict__ left, const uint8_t *__restrict__ right,
                                                      int pitch, long long img_pair, int W, int H, int npairs,
                                                      uint64_t *__restrict__ codes_l, uint64_t *__restrict__ codes_r,
                                                      long long ws_pair_words)
{
    const int z = blockIdx.z;
    const int pr = z < npairs ? z : z - npairs;
    const uint8_t *img = (z < npairs ? left : right) + pr * img_pair;
    uint64_t *out = (z < npairs ? codes_l : codes_r) + pr * ws_pair_words;
    census_tile<N>(img, pitch, W, H, out, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// windowed aggregation for w = 16, one scanline per lane
//
// Each lane carries the 16 values of its scanline as 8 packed u16 pairs, so
// a step needs no cross-lane traffic: k +- 1 neighbours are funnel shifts
// of adjacent registers.  When lo(p) = lo(q) on every lane of the wave (the
// common case: windows are constant over 4 x 4 blocks) the predecessor is
// used as it is; otherwise each lane re-indexes its own values through a
// private LDS row padded with the sentinel.  Waves of a batch's pairs share
// one launch (grid y = pair), which is what keeps the chip busy: one
// 1920x1080 pair has only 18 000 scanlines.

constexpr int kW16Lines = 256;       // scanlines (lanes) per workgroup
constexpr int kW16Row = 27;          // dwords of LDS per lane: 18 + 16 + 20 u16
constexpr int kW16Pad = 18;          // u16 index of value 0 in the lane's row

struct Win16Params {
    const uint8_t *cost;
    const uint8_t *lo;  // window starts, one byte per pixel
    uint8_t *out;
    long long cost_pair, lo_pair, out_pair, vstride;  // bytes
    int W, H;
    uint32_t p1, p2;
    int np;
    int paths[8];   // per slot: direction | output volume << 8
    int gstart[9];  // first workgroup (grid x) of each slot
};

__device__ __forceinline__ uint32_t bytes_lo(uint32_t c) { return __builtin_amdgcn_perm(0u, c, 0x0C010C00u); }
__device__ __forceinline__ uint32_t bytes_hi(uint32_t c) { return __builtin_amdgcn_perm(0u, c, 0x0C030C02u); }
// low bytes of two u16 pairs (values <= 255) -> 4 bytes
__device__ __forceinline__ uint32_t pack4(uint32_t a, uint32_t b) { return __builtin_amdgcn_perm(b, a, 0x06040200u); }
__device__ __forceinline__ uint32_t funnel16(uint32_t hi, uint32_t lo) { return __builtin_amdgcn_alignbit(hi, lo, 16); }


// One step of eq. (8) on per-pixel windows for one lane (one scanline):
// L, m hold the predecessor's 16 values (packed u16 pairs) and their
// minimum (in both u16 halves) and are replaced by the new ones; c4 holds
// the 16 cost bytes; sh = lo(p) - lo(q) (0 where q has no window).  Returns
// the new values as bytes.  Every lane of the wave must call it
// (wave-uniform branches).
__device__ __forceinline__ v4u win16_update(uint32_t (&L)[8], uint32_t &m, const v4u c4, const int sh,
                                            const uint32_t P1, const uint32_t P2, uint32_t *row)
{
    // predecessor values at window indices j - 1, j, j + 1 of p's window,
    // V(j) = Lq(j + sh) (sentinel outside q's window), as packed pairs:
    // Pm[k] = (V(2k-1), V(2k)), P0[k] = (V(2k), V(2k+1)), Pp[k] = (V(2k+1), V(2k+2))
    auto Ld = [&](int q) -> uint32_t { return (q >= 0 && q < 8) ? L[q] : kInf2; };
    uint32_t Pm[8], P0[8], Pp[8];
    {
        // sh = 0: P0 is L itself, Pm and Pp are L moved by half a pair
        uint32_t F[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) F[q] = funnel16(Ld(q), Ld(q - 1));
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            Pm[k] = F[k];
            P0[k] = L[k];
            Pp[k] = F[k + 1];
        }
    }
    if (__ballot(sh != 0) != 0) {
        // any lane re-indexes: every lane goes through its LDS row, where
        // q's 16 values sit between sentinels (lanes with sh = 0 read them
        // back unmoved).  Value V(j - 1) = Lq(j + e), e = sh - 1, starts
        // at u16 index kW16Pad + e of the row: dword `base`, half e & 1,
        // taken with a per-lane funnel shift of 0 or 16 bits.
#pragma unroll
        for (int k = 0; k < 8; ++k) row[kW16Pad / 2 + k] = L[k];
        const int e = min(max(sh - 1, -kW16Pad), 16);
        const int base = (kW16Pad + e) >> 1;
        const uint32_t half = (uint32_t)(e & 1) << 4;
        uint32_t D[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) D[q] = row[base + q];
        uint32_t V[9];  // V[q] = (V(2q-1), V(2q))
#pragma unroll
        for (int q = 0; q < 9; ++q) V[q] = __builtin_amdgcn_alignbit(D[q + 1], D[q], half);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            Pm[k] = V[k];
            P0[k] = funnel16(V[k + 1], V[k]);
            Pp[k] = V[k + 1];
        }
    }
    // C + min(V(j), V(j+-1) + P1, m_q + P2) - m_q = C + min(t - m_q, P2) with
    // t = min(V(j), V(j+-1) + P1) >= m_q (sentinels included), so m_q enters
    // last and the step's dependency chain stays short
    const uint32_t cw[4] = {c4.x, c4.y, c4.z, c4.w};
    uint32_t Ln[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t t = pk_min(P0[k], pk_add(pk_min(Pm[k], Pp[k]), P1));
        const uint32_t c = (k & 1) ? bytes_hi(cw[k >> 1]) : bytes_lo(cw[k >> 1]);
        Ln[k] = pk_add(pk_min(pk_sub(t, m), P2), c);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) L[k] = Ln[k];
    m = pk_min_halves(pk_min_tree<8>(Ln));
    return (v4u){pack4(Ln[0], Ln[1]), pack4(Ln[2], Ln[3]), pack4(Ln[4], Ln[5]), pack4(Ln[6], Ln[7])};
}

template <int PF, int KIND>
__device__ __forceinline__ void win16_scan(const Win16Params &a, __amdgpu_buffer_rsrc_t rc,
                                           __amdgpu_buffer_rsrc_t rl, __amdgpu_buffer_rsrc_t ro, int du, int dv,
                                           int g, uint32_t *row)
{
    const int W = a.W, H = a.H;
    const int idx = g * kW16Lines + (int)threadIdx.x;
    const Line ln = line_geom(KIND == kHorizontal ? (idx < H ? idx : H) : idx, du, dv, W, H);
    // wave-uniform step range
    int I0, I1;
    if constexpr (KIND == kDiagonal) {
        const bool any = ln.i1 > ln.i0;
        I0 = __builtin_amdgcn_readfirstlane(wave_min(any ? ln.i0 : 1 << 30));
        I1 = __builtin_amdgcn_readfirstlane(wave_max(any ? ln.i1 : 0));
        if (I1 <= I0) return;
    } else {
        I0 = 0;
        I1 = KIND == kHorizontal ? W : H;
    }
    const uint32_t pstep = (uint32_t)(ln.sv * W + ln.su);
    const uint32_t pix0 = (uint32_t)(ln.vb * W + ln.ub);
    const uint32_t li0 = (uint32_t)ln.i0, llen = (uint32_t)(ln.i1 - ln.i0);
    auto inside = [&](int i) -> bool { return (uint32_t)i - li0 < llen; };

    v4u ring_c[PF];
    uint32_t ring_l[PF];
#pragma unroll
    for (int s = 0; s < PF; ++s) {
        const int i = I0 + s;
        const uint32_t px = pix0 + (uint32_t)i * pstep;
        const bool in = inside(i);
        ring_c[s] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rc, in ? px * 16u : kOff, 0, 0));
        ring_l[s] = __builtin_amdgcn_raw_buffer_load_b8(rl, in ? px : kOff, 0, 0);
    }
    const uint32_t P1 = a.p1 | (a.p1 << 16), P2 = a.p2 | (a.p2 << 16);
    uint32_t L[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) L[k] = 0u;
    uint32_t m = 0u;  // min of L (in both halves)
    int loq = kNoLo;

    // one step: consume ring slot S (loaded PF steps ago), refill it for
    // step i + PF, aggregate, store
    auto step = [&](const int i, const int S) __attribute__((always_inline)) {
        const bool act = inside(i);
        // later loads and the stores since may stay in flight (2 loads + 1
        // store per step)
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(1 + (PF - 1) * 3));
        const v4u c4 = ring_c[S];
        const int lop = (int)ring_l[S];
        {
            const int ip = i + PF;
            const uint32_t px = pix0 + (uint32_t)ip * pstep;
            const bool in = inside(ip);
            ring_c[S] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rc, in ? px * 16u : kOff, 0, 0));
            ring_l[S] = __builtin_amdgcn_raw_buffer_load_b8(rl, in ? px : kOff, 0, 0);
        }
        const int sh = (act && loq != kNoLo) ? lop - loq : 0;
        const v4u o4 = win16_update(L, m, c4, sh, P1, P2, row);
        const uint32_t o = act ? (pix0 + (uint32_t)i * pstep) * 16u : kOff;
        __builtin_amdgcn_raw_buffer_store_b128(o4, ro, o, 0, kStreamPolicy);
        loq = act ? lop : kNoLo;
    };

    // The first turn of the ring runs outside the loop: at the loop head
    // every slot was then refilled by a step, exactly as on the back edge,
    // so the loads in flight there need no deeper wait than inside the loop.
#pragma unroll
    for (int S = 0; S < PF; ++S) step(I0 + S, S);
    // two turns of the ring per iteration keep each slot in its registers
    constexpr int UNROLL = 2 * PF;
    const int nblk = (I1 - I0 - PF + UNROLL - 1) / UNROLL;
    for (int blk = 0; blk < nblk; ++blk) {
#pragma unroll
        for (int S = 0; S < UNROLL; ++S) step(I0 + PF + blk * UNROLL + S, S % PF);
    }
}

// Horizontal scanlines, one per lane, staged through LDS.  The 64 lanes of
// a wave hold 64 rows, so a direct access per step would touch 64 cache
// lines.  Instead the wave moves tiles of 8 pixels x 64 rows: the cost tile
// (8 KB) and the window starts (2 KB) are fetched with 8 rows x 128 bytes
// per load instruction into a register ring one tile ahead, written to LDS,
// read back one pixel per lane and step, and the results go out the same
// way.  The cost and output tiles are XOR-swizzled (unit (r, p) at
// r * 8 + (p ^ (r & 7))) so that both the row-wise copies and the per-lane
// reads are free of bank conflicts; the window-start tile has rows of 9
// dwords.  One wave per workgroup: LDS is private to the wave and needs no
// barrier.

constexpr int kHT = 8;      // pixels per tile
constexpr int kHRing = 1;   // tiles in flight ahead of the one processed

__global__ __launch_bounds__(64) void k_aggregate_win16_h(Win16Params a)
{
    __shared__ v4u s_c[64 * kHT];
    __shared__ v4u s_o[64 * kHT];
    __shared__ uint32_t s_l[64 * (kHT + 1)];
    __shared__ uint32_t rows[64 * kW16Row];
    // few, long scanlines sharing SIMDs with the vertical and diagonal
    // waves: let them issue first
    __builtin_amdgcn_s_setprio(3);
    const int lane = threadIdx.x;
    uint32_t *row = rows + lane * kW16Row;
#pragma unroll
    for (int q = 0; q < kW16Row; ++q) row[q] = kInf2;
    int slot = 0;
    while (slot + 1 < a.np && (int)blockIdx.x >= a.gstart[slot + 1]) ++slot;
    slot = __builtin_amdgcn_readfirstlane(slot);
    const int r = __builtin_amdgcn_readfirstlane(a.paths[slot] & 0xFF);
    const int vol = __builtin_amdgcn_readfirstlane(a.paths[slot] >> 8);
    const int g = __builtin_amdgcn_readfirstlane((int)blockIdx.x - a.gstart[slot]);
    const int du = __builtin_amdgcn_readfirstlane(dir_du(r));
    const int pr = blockIdx.y;
    const int W = a.W, H = a.H;
    const uint32_t npix = (uint32_t)W * (uint32_t)H;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cost + pr * a.cost_pair, npix * 16u);
    const __amdgpu_buffer_rsrc_t rl = make_rsrc(a.lo + pr * a.lo_pair, npix);
    const __amdgpu_buffer_rsrc_t ro = make_rsrc(a.out + pr * a.out_pair + (size_t)vol * a.vstride, npix * 16u);
    const int R0 = g * 64;            // first row of this wave
    const int K = (W + kHT - 1) / kHT;  // tiles per row
    // row-wise copy mapping: copy q (0..7) moves rows 8q .. 8q+7, lane l at
    // row 8q + l/8, pixel unit (l % 8) ^ (row & 7); its LDS unit is 64q + l
    const int crow = lane >> 3, cu = lane & 7;
    // (unsigned compares and bitwise & keep these branch-free)
    auto cost_off = [&](int k, int q) -> uint32_t {
        const int rr = 8 * q + crow, x = kHT * k + (cu ^ (rr & 7)), y = R0 + rr;
        const bool in = ((uint32_t)y < (uint32_t)H) & ((uint32_t)x < (uint32_t)W);
        return in ? ((uint32_t)y * (uint32_t)W + (uint32_t)x) * 16u : kOff;
    };
    auto lo_off = [&](int k, int q) -> uint32_t {
        const int rr = 8 * q + crow, x = kHT * k + cu, y = R0 + rr;
        const bool in = ((uint32_t)y < (uint32_t)H) & ((uint32_t)x < (uint32_t)W);
        return in ? (uint32_t)y * (uint32_t)W + (uint32_t)x : kOff;
    };
    v4u ring_c[kHRing][8];
    uint32_t ring_l[kHRing][8];
    auto fetch = [&](int t, int slot_) __attribute__((always_inline)) {
        // tile number t of the scan (t >= K loads nothing)
        // (t >= K gives k outside 0..K-1, so every offset is kOff)
        const int k = du > 0 ? t : K - 1 - t;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            ring_c[slot_][q] = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rc, cost_off(k, q), 0, 0));
            ring_l[slot_][q] = __builtin_amdgcn_raw_buffer_load_b8(rl, lo_off(k, q), 0, 0);
        }
    };
#pragma unroll
    for (int t = 0; t < kHRing; ++t) fetch(t, t);

    const uint32_t P1 = a.p1 | (a.p1 << 16), P2 = a.p2 | (a.p2 << 16);
    uint32_t L[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) L[k] = 0u;
    uint32_t m = 0u;
    int loq = kNoLo;
    const int y = R0 + lane;
    // 16 loads and 8 stores per tile; the tile's loads were issued kHRing
    // tiles ago, followed by that tile's stores and, for each tile since,
    // its loads and stores
    constexpr int kAfter = 8 + (kHRing - 1) * (16 + 8);
    auto tile = [&](const int t, const int sl) __attribute__((always_inline)) {
        const int k = du > 0 ? t : K - 1 - t;
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(kAfter));
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            s_c[64 * q + lane] = ring_c[sl][q];
            s_l[(8 * q + crow) * (kHT + 1) + cu] = ring_l[sl][q];
        }
        // this lane's 8 pixels of the tile, read before the dependent chain
        v4u c4s[kHT];
        int lops[kHT];
#pragma unroll
        for (int s = 0; s < kHT; ++s) {
            const int pp = du > 0 ? s : kHT - 1 - s;
            c4s[s] = s_c[lane * 8 + (pp ^ (lane & 7))];
            lops[s] = (int)s_l[lane * (kHT + 1) + pp];
        }
        fetch(t + kHRing, sl);
#pragma unroll
        for (int s = 0; s < kHT; ++s) {
            const int pp = du > 0 ? s : kHT - 1 - s;
            const int x = kHT * k + pp;
            const bool act = t < K && x < W && y < H;
            const v4u c4 = c4s[s];
            const int lop = lops[s];
            const int sh = (act && loq != kNoLo) ? lop - loq : 0;
            const v4u o4 = win16_update(L, m, c4, sh, P1, P2, row);
            s_o[lane * 8 + (pp ^ (lane & 7))] = o4;
            loq = act ? lop : kNoLo;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            __builtin_amdgcn_raw_buffer_store_b128(s_o[64 * q + lane], ro, cost_off(k, q), 0, kStreamPolicy);
    };
    // the first turn of the ring outside the loop, so that the loop head
    // sees the same loads in flight from both sides
#pragma unroll
    for (int sl = 0; sl < kHRing; ++sl) tile(sl, sl);
    for (int tb = kHRing; tb < K; tb += kHRing) {
#pragma unroll
        for (int sl = 0; sl < kHRing; ++sl) tile(tb + sl, sl);
    }
}

// Vertical and diagonal scanlines: neighbouring lanes are neighbouring
// pixels of one row at every step, so one scanline per lane keeps every
// access contiguous.
template <int PF, int MINWG>
__global__ __launch_bounds__(256, MINWG) void k_aggregate_win16(Win16Params a)
{
    __shared__ uint32_t rows[kW16Lines * kW16Row];
    uint32_t *row = rows + threadIdx.x * kW16Row;
    int slot = 0;
    while (slot + 1 < a.np && (int)blockIdx.x >= a.gstart[slot + 1]) ++slot;
    slot = __builtin_amdgcn_readfirstlane(slot);
    const int r = __builtin_amdgcn_readfirstlane(a.paths[slot] & 0xFF);
    const int vol = __builtin_amdgcn_readfirstlane(a.paths[slot] >> 8);
    const int g = __builtin_amdgcn_readfirstlane((int)blockIdx.x - a.gstart[slot]);
    const int du = __builtin_amdgcn_readfirstlane(dir_du(r)), dv = __builtin_amdgcn_readfirstlane(dir_dv(r));
    const int pr = blockIdx.y;
    const uint32_t npix = (uint32_t)a.W * (uint32_t)a.H;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cost + pr * a.cost_pair, npix * 16u);
    const __amdgpu_buffer_rsrc_t rl = make_rsrc(a.lo + pr * a.lo_pair, npix);
    const __amdgpu_buffer_rsrc_t ro = make_rsrc(a.out + pr * a.out_pair + (size_t)vol * a.vstride, npix * 16u);
#pragma unroll
    for (int q = 0; q < kW16Row; ++q) row[q] = kInf2;  // sentinel padding; values are written per use
    if (du == 0)
        win16_scan<PF, kVertical>(a, rc, rl, ro, du, dv, g, row);
    else
        win16_scan<PF, kDiagonal>(a, rc, rl, ro, du, dv, g, row);
}

// Steps of cost prefetched by k_aggregate_win16, by frame size (measured on
// batches of 16 pairs): on 1920x1080, 12 steps (about 200 registers, two
// waves per SIMD) beat 6 (four waves per SIMD) by 6 %; on 1280x720, with
// fewer scanlines to spread, 6 steps beat 12 by 13 %.
constexpr long long kWin16DeepPixels = 1500000;  // pixels per pair from which 12 steps are used

}  // namespace

hipError_t launch_downsample4(const uint8_t *img, int W, int H, int pitch, long long img_stride, int nimg,
                              uint8_t *out, hipStream_t s)
{
    dim3 grid((W / 4 + 63) / 64, (H / 4 + 3) / 4, nimg), block(256);
    hipLaunchKernelGGL(k_downsample4, grid, block, 0, s, img, W, H, pitch, out, img_stride);
    return hipGetLastError();
}

hipError_t launch_cost_win(const Problem &pb, const uint64_t *cl, const uint64_t *cr, const int32_t *lo,
                           uint8_t *cost, hipStream_t s)
{
    dim3 grid((pb.W + kWinTile - 1) / kWinTile, pb.H), block(kWinTile);
    hipLaunchKernelGGL(k_cost_win, grid, block, 0, s, cl, cr, lo, pb.W, pb.H, pb.w, pb.cmax, cost, 0ll, 0ll, 0ll,
                       nullptr);
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
    if (l8)
        hipLaunchKernelGGL(k_wta_win<true>, grid, block, 0, s, vols, vstride, np, lo, pb.W, pb.H, pb.w, dint, dsub, 0ll,
                           0ll);
    else
        hipLaunchKernelGGL(k_wta_win<false>, grid, block, 0, s, vols, vstride, np, lo, pb.W, pb.H, pb.w, dint, dsub,
                           0ll, 0ll);
    return hipGetLastError();
}

// A second stream per device for the horizontal aggregation, which has
// too few scanlines (one wave per 64 rows) to fill the chip on its own and
// runs beside the vertical and diagonal one.  Created on first use; the
// fork / join (event record + stream wait) is serialised across host threads.
struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool ok = false, tried = false;
};
static std::mutex g_side_mutex;
static SideStream g_side[64];

static SideStream *side_stream()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    SideStream &ss = g_side[dev];
    if (!ss.tried) {
        ss.tried = true;
        ss.ok = hipStreamCreateWithFlags(&ss.stream, hipStreamNonBlocking) == hipSuccess &&
                hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) == hipSuccess &&
                hipEventCreateWithFlags(&ss.join, hipEventDisableTiming) == hipSuccess;
    }
    return ss.ok ? &ss : nullptr;
}

hipError_t launch_match_win_pairs(const Problem &pb, const WinPairs &b, hipStream_t s)
{
    const long long npix = (long long)pb.W * pb.H;
    const long long ws_words = (long long)(b.ws_pair / 8);
    // census of every left and right image
    {
        dim3 grid((pb.W + kCensusTW - 1) / kCensusTW, (pb.H + kCensusTH - 1) / kCensusTH, 2 * b.npairs), block(256);
        switch (pb.n) {
        case 3:
            hipLaunchKernelGGL(k_census_pairs<3>, grid, block, 0, s, b.left, b.right, b.pitch, b.img_pair, pb.W, pb.H,
                               b.npairs, b.codes_l, b.codes_r, ws_words);
            break;
        case 5:
            hipLaunchKernelGGL(k_census_pairs<5>, grid, block, 0, s, b.left, b.right, b.pitch, b.img_pair, pb.W, pb.H,
                               b.npairs, b.codes_l, b.codes_r, ws_words);
            break;
        case 7:
            hipLaunchKernelGGL(k_census_pairs<7>, grid, block, 0, s, b.left, b.right, b.pitch, b.img_pair, pb.W, pb.H,
                               b.npairs, b.codes_l, b.codes_r, ws_words);
            break;
        default: return hipErrorInvalidValue;
        }
    }
    // windowed cost of every pair
    {
        dim3 grid((pb.W + kWinTile - 1) / kWinTile, pb.H, b.npairs), block(kWinTile);
        hipLaunchKernelGGL(k_cost_win, grid, block, 0, s, b.codes_l, b.codes_r, b.lo, pb.W, pb.H, pb.w, pb.cmax, b.cost,
                           ws_words, npix, (long long)b.ws_pair, b.lo8);
    }
    // aggregation of every pair and direction in one launch
    {
        Win16Params p{};
        p.cost = b.cost;
        p.lo = b.lo8;
        p.out = b.paths;
        p.cost_pair = (long long)b.ws_pair;
        p.lo_pair = (long long)b.ws_pair;
        p.out_pair = (long long)b.ws_pair;
        p.vstride = b.vstride;
        p.W = pb.W;
        p.H = pb.H;
        p.p1 = (uint32_t)pb.p1;
        p.p2 = (uint32_t)pb.p2;
        p.np = pb.npaths;
        // horizontal directions: one wave (64 rows) per workgroup, LDS-staged
        Win16Params h = p;
        int acc = 0, no = 0;
        for (int r = 0; r < 2 && r < pb.npaths; ++r) {
            h.paths[no] = r | (r << 8);
            h.gstart[no] = acc;
            acc += (pb.H + 63) / 64;
            ++no;
        }
        h.np = no;
        h.gstart[no] = acc;
        std::unique_lock<std::mutex> lock(g_side_mutex);
        SideStream *ss = side_stream();
        hipStream_t hs = s;
        if (ss && hipEventRecord(ss->fork, s) == hipSuccess && hipStreamWaitEvent(ss->stream, ss->fork, 0) == hipSuccess)
            hs = ss->stream;
        if (no > 0) hipLaunchKernelGGL(k_aggregate_win16_h, dim3(acc, b.npairs), dim3(64), 0, hs, h);
        // vertical and diagonal directions: diagonal groups first
        acc = 0;
        no = 0;
        for (const int kind : {2, 1})
            for (int r = 2; r < pb.npaths; ++r) {
                const int k = r >= 4 ? 2 : 1;
                if (k != kind) continue;
                const int nl = r <= 3 ? pb.W : pb.W + pb.H - 1;
                p.paths[no] = r | (r << 8);
                p.gstart[no] = acc;
                acc += (nl + kW16Lines - 1) / kW16Lines;
                ++no;
            }
        p.np = no;
        p.gstart[no] = acc;
        if (no > 0) {
            if ((long long)pb.W * pb.H >= kWin16DeepPixels)
                hipLaunchKernelGGL((k_aggregate_win16<12, 2>), dim3(acc, b.npairs), dim3(kW16Lines), 0, s, p);
            else
                hipLaunchKernelGGL((k_aggregate_win16<6, 4>), dim3(acc, b.npairs), dim3(kW16Lines), 0, s, p);
        }
        if (hs != s) {
            const hipError_t e1 = hipEventRecord(ss->join, hs);
            const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(s, ss->join, 0) : e1;
            if (e2 != hipSuccess) return e2;
        }
    }
    // selection of every pair
    {
        dim3 grid((unsigned)((npix + 255) / 256), b.npairs), block(256);
        hipLaunchKernelGGL(k_wta_win<true>, grid, block, 0, s, b.paths, b.vstride, pb.npaths, b.lo, pb.W, pb.H, pb.w,
                           b.dint, b.dsub, (long long)b.ws_pair, npix);
    }
    return hipGetLastError();
}

}  // namespace sgm
