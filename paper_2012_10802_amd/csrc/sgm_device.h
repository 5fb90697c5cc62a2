// Device code shared by the single-pair kernels (sgm_kernels.hip) and the
// batched kernels (sgm_batch.hip): packed-u16 helpers, DPP reductions, lane
// I/O, the census and cost tiles, the scanline aggregation and the
// selection.  Every function here is inlined into the kernels that use it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sgm_internal.h"

namespace sgm {
namespace dev {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr uint32_t kInf2 = 0x3FFF3FFFu;  // pair of "outside the window" values
constexpr uint32_t kPad = 0x3FFFu;

__device__ __forceinline__ uint32_t pk_min(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) - __builtin_bit_cast(u16x2, b));
}
// the minimum of the two halves, in both halves
__device__ __forceinline__ uint32_t pk_min_halves(uint32_t a)
{
    const u16x2 v = __builtin_bit_cast(u16x2, a);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(v, __builtin_shufflevector(v, v, 1, 0)));
}
// packed minimum of n pairs as a balanced tree (a short dependency chain)
template <int N>
__device__ __forceinline__ uint32_t pk_min_tree(const uint32_t *v)
{
    if constexpr (N == 1) {
        return v[0];
    } else {
        return pk_min(pk_min_tree<N / 2>(v), pk_min_tree<N - N / 2>(v + N / 2));
    }
}

// DPP move with zero fill: lanes whose source lies outside their row read 0
template <int CTRL>
__device__ __forceinline__ uint32_t dpp0(uint32_t src)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)src, CTRL, 0xF, 0xF, true);
}
constexpr int kQuadSwap1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kQuadSwap2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int kRowShl1 = 0x101;   // lane i reads lane i+1
constexpr int kRowShr1 = 0x111;   // lane i reads lane i-1
constexpr int kRowRor4 = 0x124;
constexpr int kRowRor8 = 0x128;

// minimum / maximum over the 16 lanes of a DPP row, broadcast to all of them
// (quad permutations and row rotations never leave the row)
template <int CTRL>
__device__ __forceinline__ uint32_t rot(uint32_t src)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)src, CTRL, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t row_min16(uint32_t x)
{
    x = min(x, rot<kQuadSwap1>(x));
    x = min(x, rot<kQuadSwap2>(x));
    x = min(x, rot<kRowRor4>(x));
    x = min(x, rot<kRowRor8>(x));
    return x;
}
__device__ __forceinline__ uint32_t row_max16(uint32_t x)
{
    x = max(x, rot<kQuadSwap1>(x));
    x = max(x, rot<kQuadSwap2>(x));
    x = max(x, rot<kRowRor4>(x));
    x = max(x, rot<kRowRor8>(x));
    return x;
}

// the same over aligned groups of G = 4, 8 or 16 lanes (a quad, a half row,
// a row): after the two quad swaps every lane holds its quad's extremum, and
// the half-row mirror (lane i reads lane 7 - i of its half row) brings in
// the other quad of the half row
constexpr int kRowHalfMirror = 0x141;
template <int G>
__device__ __forceinline__ uint32_t group_min(uint32_t x)
{
    static_assert(G == 4 || G == 8 || G == 16, "groups of 4, 8 or 16 lanes");
    if constexpr (G == 16) {
        return row_min16(x);
    } else {
        x = min(x, rot<kQuadSwap1>(x));
        x = min(x, rot<kQuadSwap2>(x));
        if constexpr (G == 8) x = min(x, rot<kRowHalfMirror>(x));
        return x;
    }
}
template <int G>
__device__ __forceinline__ uint32_t group_max(uint32_t x)
{
    static_assert(G == 4 || G == 8 || G == 16, "groups of 4, 8 or 16 lanes");
    if constexpr (G == 16) {
        return row_max16(x);
    } else {
        x = max(x, rot<kQuadSwap1>(x));
        x = max(x, rot<kQuadSwap2>(x));
        if constexpr (G == 8) x = max(x, rot<kRowHalfMirror>(x));
        return x;
    }
}

// direction table: path r -> r = (du, dv); predecessor of p is p - r
__device__ __forceinline__ int dir_du(int r)
{
    return (r == 0 || r == 4 || r == 6) ? 1 : ((r == 1 || r == 5 || r == 7) ? -1 : 0);
}
__device__ __forceinline__ int dir_dv(int r)
{
    return (r == 2 || r == 4 || r == 5) ? 1 : ((r == 3 || r == 6 || r == 7) ? -1 : 0);
}

// ---------------------------------------------------------------------------
// lane value I/O: VPL bytes (or u16) per lane

// a lane's VPL cost bytes as loaded, in dwords (the two bytes of a 2-value
// lane zero-extended)
template <int VPL>
struct Raw {
    static constexpr int NW = (VPL + 3) / 4;
    uint32_t d[NW];
};

// (used for the per-direction volumes, which are read once: non-temporal)
template <int VPL, bool ALIGNED>
__device__ __forceinline__ void load_u8(Raw<VPL> &r, const uint8_t *p, int nvalid)
{
    if constexpr (ALIGNED) {
        if constexpr (VPL == 2) {
            r.d[0] = *reinterpret_cast<const uint16_t *>(p);
        } else if constexpr (VPL == 4) {
            r.d[0] = *reinterpret_cast<const uint32_t *>(p);
        } else if constexpr (VPL == 8) {
            const unsigned long long t = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long *>(p));
            r.d[0] = (uint32_t)t;
            r.d[1] = (uint32_t)(t >> 32);
        } else if constexpr (VPL == 12) {
            const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
            r.d[0] = __builtin_nontemporal_load(q);
            r.d[1] = __builtin_nontemporal_load(q + 1);
            r.d[2] = __builtin_nontemporal_load(q + 2);
        } else {
            const unsigned long long *q = reinterpret_cast<const unsigned long long *>(p);
            const unsigned long long t0 = __builtin_nontemporal_load(q), t1 = __builtin_nontemporal_load(q + 1);
            r.d[0] = (uint32_t)t0;
            r.d[1] = (uint32_t)(t0 >> 32);
            r.d[2] = (uint32_t)t1;
            r.d[3] = (uint32_t)(t1 >> 32);
        }
    } else {
#pragma unroll
        for (int i = 0; i < Raw<VPL>::NW; ++i) r.d[i] = 0;
#pragma unroll
        for (int i = 0; i < VPL; ++i)
            if (i < nvalid) r.d[i / 4] |= (uint32_t)p[i] << (8 * (i % 4));
    }
}

template <int VPL>
__device__ __forceinline__ void zero(Raw<VPL> &r)
{
#pragma unroll
    for (int i = 0; i < Raw<VPL>::NW; ++i) r.d[i] = 0;
}

// bytes (2j, 2j+1) of the raw lane values -> packed u16 pair j
template <int VPL>
__device__ __forceinline__ uint32_t unpack_pair(const Raw<VPL> &r, int j)
{
    const uint32_t x = r.d[j / 2];
    return (j & 1) ? __builtin_amdgcn_perm(x, x, 0x0C030C02u) : __builtin_amdgcn_perm(x, x, 0x0C010C00u);
}

// low bytes of packed pairs a (values 0,1) and b (values 2,3) -> one dword
__device__ __forceinline__ uint32_t pack_bytes(uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_perm(b, a, 0x06040200u);
}

template <int VPL, bool ALIGNED>
__device__ __forceinline__ void store_u8_pairs(uint8_t *p, const uint32_t (&v)[VPL / 2], int nvalid)
{
    constexpr int NP = VPL / 2;
    if constexpr (ALIGNED) {
        if constexpr (VPL == 2) {
            *reinterpret_cast<uint16_t *>(p) = (uint16_t)__builtin_amdgcn_perm(v[0], v[0], 0x0C0C0200u);
        } else if constexpr (VPL == 4) {
            *reinterpret_cast<uint32_t *>(p) = pack_bytes(v[0], v[1]);
        } else if constexpr (VPL == 8) {
            *reinterpret_cast<uint2 *>(p) = make_uint2(pack_bytes(v[0], v[1]), pack_bytes(v[2], v[3]));
        } else if constexpr (VPL == 12) {
            uint32_t *q = reinterpret_cast<uint32_t *>(p);
            q[0] = pack_bytes(v[0], v[1]);
            q[1] = pack_bytes(v[2], v[3]);
            q[2] = pack_bytes(v[4], v[5]);
        } else {
            *reinterpret_cast<uint4 *>(p) = make_uint4(pack_bytes(v[0], v[1]), pack_bytes(v[2], v[3]),
                                                       pack_bytes(v[4], v[5]), pack_bytes(v[6], v[7]));
        }
    } else {
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            if (2 * j < nvalid) p[2 * j] = (uint8_t)(v[j] & 0xFF);
            if (2 * j + 1 < nvalid) p[2 * j + 1] = (uint8_t)((v[j] >> 16) & 0xFF);
        }
    }
}

template <int VPL, bool ALIGNED>
__device__ __forceinline__ void store_u16_pairs(uint16_t *p, const uint32_t (&v)[VPL / 2], int nvalid)
{
    constexpr int NP = VPL / 2;
    if constexpr (ALIGNED) {
        uint32_t *q = reinterpret_cast<uint32_t *>(p);
#pragma unroll
        for (int j = 0; j < NP; ++j) q[j] = v[j];
    } else {
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            if (2 * j < nvalid) p[2 * j] = (uint16_t)(v[j] & 0xFFFF);
            if (2 * j + 1 < nvalid) p[2 * j + 1] = (uint16_t)(v[j] >> 16);
        }
    }
}

template <int VPL, bool ALIGNED>
__device__ __forceinline__ void load_u16_pairs(uint32_t (&v)[VPL / 2], const uint16_t *p, int nvalid)
{
    constexpr int NP = VPL / 2;
    if constexpr (ALIGNED) {
        const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
        if constexpr (NP % 4 == 0) {
#pragma unroll
            for (int j = 0; j < NP; j += 4) {
                const uint4 t = reinterpret_cast<const uint4 *>(q)[j / 4];
                v[j] = t.x;
                v[j + 1] = t.y;
                v[j + 2] = t.z;
                v[j + 3] = t.w;
            }
        } else if constexpr (NP % 2 == 0) {
#pragma unroll
            for (int j = 0; j < NP; j += 2) {
                const uint2 t = reinterpret_cast<const uint2 *>(q)[j / 2];
                v[j] = t.x;
                v[j + 1] = t.y;
            }
        } else {
#pragma unroll
            for (int j = 0; j < NP; ++j) v[j] = q[j];
        }
    } else {
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const uint32_t lo = (2 * j < nvalid) ? p[2 * j] : 0u;
            const uint32_t hi = (2 * j + 1 < nvalid) ? p[2 * j + 1] : 0u;
            v[j] = lo | (hi << 16);
        }
    }
}


// ---------------------------------------------------------------------------
// census transform
//
// A workgroup covers a tile of kCensusTW x kCensusTH pixels (256 threads);
// each thread takes four horizontally adjacent pixels of one row and
// compares their neighbours four at a time inside 32-bit words (one byte
// per pixel).  For
// bytes a (neighbour) and c (centre), t = (a | 0x80) - (c & 0x7F) stays
// inside its byte, and its bit 7 says whether the low seven bits of a are
// >= those of c; a >= c is then the majority of (a, not c, t) at bit 7, and
// a < c its complement.  Eight consecutive comparisons are gathered per byte by
// shifting right (the first ends at bit 0), so each 32-bit word holds one
// byte of the code of each of the four pixels; byte permutes then assemble
// the four codes.  Bit b of a code is the b-th comparison in row-major order
// over the window (centre skipped), as the definition orders them.

template <int N>
__device__ __forceinline__ void census_tile(const uint8_t *__restrict__ img, int pitch, int W, int H,
                                            uint64_t *__restrict__ out, int bx, int by)
{
    static_assert(N == 3 || N == 5 || N == 7, "census window 3, 5 or 7");
    constexpr int R = N / 2;
    constexpr int NB = N * N - 1;                  // 8, 24 or 48 bits: whole bytes
    constexpr int NPL = NB / 8;                    // bytes of a code
    constexpr int TW = kCensusTW, TH = kCensusTH;
    constexpr int LW = TW + 8;                     // 4 margin columns on each side (R <= 3)
    constexpr int LH = TH + 2 * R;
    constexpr int QPR = TW / 4;                    // threads (quads) per row
    __shared__ uint32_t tile[LH][LW / 4];
    const int u0 = bx * TW, v0 = by * TH;
    // tile byte (ty, tx) = I(clamp(u0 + tx - 4), clamp(v0 + ty - R)), one
    // dword (four columns) per thread and step
    for (int t = threadIdx.x; t < LH * (LW / 4); t += blockDim.x) {
        const int ty = t / (LW / 4), d = t % (LW / 4);
        const uint8_t *row = img + (size_t)min(max(v0 + ty - R, 0), H - 1) * pitch;
        const int x = u0 - 4 + 4 * d;
        uint32_t wd = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) wd |= (uint32_t)row[min(max(x + e, 0), W - 1)] << (8 * e);
        tile[ty][d] = wd;
    }
    __syncthreads();
    const int q = threadIdx.x % QPR, ty = threadIdx.x / QPR;
    const int v = v0 + ty, ub = u0 + 4 * q;  // the quad's pixels: ub .. ub + 3 of row v
    if (ty >= TH || v >= H || ub >= W) return;
    constexpr uint32_t kTop = 0x80808080u;
    const uint32_t c = tile[ty + R][q + 1];
    const uint32_t c7 = c & ~kTop, nc = ~c;
    uint32_t acc[NPL];
#pragma unroll
    for (int g = 0; g < NPL; ++g) acc[g] = 0u;
    int b = 0;
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
        // tile columns 4q .. 4q + 11 = image columns ub - 4 .. ub + 7
        const uint32_t w0 = tile[ty + R + dy][q], w1 = tile[ty + R + dy][q + 1], w2 = tile[ty + R + dy][q + 2];
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int k = 4 + dx;  // byte offset of the neighbours of the quad in w0 w1 w2
            const uint32_t a = k < 4 ? __builtin_amdgcn_alignbyte(w1, w0, k)
                                     : (k == 4 ? w1 : __builtin_amdgcn_alignbyte(w2, w1, k - 4));
            const uint32_t t = (a | kTop) - c7;
            // a >= c at bit 7: the majority of (a, not c, t); its complement,
            // the borrow out of the byte, is taken once the word is full
            const uint32_t ge = (a & nc) | (a & t) | (nc & t);
            acc[b / 8] = (acc[b / 8] >> 1) | (ge & kTop);
            ++b;
        }
    }
#pragma unroll
    for (int g = 0; g < NPL; ++g) acc[g] = ~acc[g];  // every bit was filled: a >= c becomes a < c
    // pixel i's code: byte g = byte i of acc[g]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (ub + i >= W) break;
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int g = 0; g < NPL; g += 2) {
            const uint32_t s0 = g + 1 < NPL ? acc[g + 1] : 0u;
            // bytes (acc[g].b_i, acc[g+1].b_i) at positions (g % 4, g % 4 + 1)
            const uint32_t sel = (g % 4 == 0) ? ((uint32_t)i | ((uint32_t)(4 + i) << 8) | 0x0C0C0000u)
                                              : (0x00000C0Cu | ((uint32_t)i << 16) | ((uint32_t)(4 + i) << 24));
            const uint32_t pv = __builtin_amdgcn_perm(s0, acc[g], sel);
            if (g < 4)
                lo |= pv;
            else
                hi |= pv;
        }
        out[(size_t)v * W + ub + i] = ((uint64_t)hi << 32) | lo;
    }
}

// ---------------------------------------------------------------------------
// matching cost: C(u,v,k) = popcount(cL(u,v) ^ cR(u - d_lo(v) - k, v))
//
// A workgroup covers kCostTile pixels of one row.  The left codes of the
// tile and the right codes of every column the tile's windows reach are
// staged in LDS.  Each thread then produces CH consecutive window values of
// one pixel per item; neighbouring lanes take neighbouring pixels, so the
// LDS reads of a wave are conflict-free (8-byte stride), and a pixel's
// window is written in CH-byte pieces (through an LDS tile, see CostLds).

constexpr int kCostTile = 64;

// LDS of one cost workgroup: the tile's left codes, the right codes its
// windows reach, and (CH >= 8, w >= 64) the tile's output, whose pixel rows are
// padded to an odd number of CH-byte pieces so that the items' piece stores
// (one pixel per lane) fall on distinct banks; the tile then leaves in
// contiguous CH-byte pieces per lane, whole lines per wave.  Stores of one
// piece per lane at the pixel stride reach only about half the HBM write
// rate of contiguous ones.
struct CostLds {
    uint64_t cl[kCostTile];
    uint64_t cr[kCostTile + 256];
    alignas(16) uint8_t out[kCostTile * (256 + 16)];
};

// the items (pixel, group of CH window values) of one cost tile.  FULL: the
// tile has kCostTile pixels (item -> pixel by shifts).  INIMG (CH >= 8
// only): every right column the tile reads lies inside the image, so no
// value is replaced by Cmax.
template <int CH, bool FULL, bool INIMG>
__device__ __forceinline__ void cost_items(const uint64_t *s_cl, const uint64_t *s_cr, int u0, int lo, int w,
                                           int cmax, int npix, int nch, uint8_t *__restrict__ out, int ostride)
{
    const int np = FULL ? kCostTile : npix;
    for (int it = threadIdx.x; it < np * nch; it += blockDim.x) {
        const int ch = it / np, px = it - ch * np;
        const int k0 = CH * ch;
        const uint64_t a = s_cl[px];
        // right column of window index k: u0 + px - lo - k = first + (px + w - 1 - k)
        const int base = px + w - 1 - k0;
        const int col0 = u0 + px - lo - k0;
        uint32_t word[CH / 4];
#pragma unroll
        for (int q = 0; q < CH / 4; ++q) {
            uint32_t wd = 0;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int kk = 4 * q + h;
                uint32_t c;
                if constexpr (CH >= 8) {
                    // w % CH == 0: every kk is inside the window and base - kk
                    // inside s_cr, so the read is unconditional and only the
                    // off-image columns are replaced (branch-free)
                    const uint32_t pc = (uint32_t)__popcll(a ^ s_cr[base - kk]);
                    c = (INIMG || col0 - kk >= 0) ? pc : (uint32_t)cmax;
                } else {
                    c = (uint32_t)cmax;
                    if (col0 - kk >= 0 && k0 + kk < w) c = (uint32_t)__popcll(a ^ s_cr[base - kk]);
                }
                wd |= c << (8 * h);
            }
            word[q] = wd;
        }
        uint8_t *dst = out + (size_t)px * ostride + k0;
        if constexpr (CH == 16) {
            *reinterpret_cast<uint4 *>(dst) = make_uint4(word[0], word[1], word[2], word[3]);
        } else if constexpr (CH == 8) {
            *reinterpret_cast<uint2 *>(dst) = make_uint2(word[0], word[1]);
        } else {
            for (int h = 0; h < CH && k0 + h < w; ++h) dst[h] = (uint8_t)(word[h / 4] >> (8 * (h % 4)));
        }
    }
}

template <int CH>
__device__ __forceinline__ void cost_tile(const uint64_t *__restrict__ cl, const uint64_t *__restrict__ cr,
                                          const int32_t *__restrict__ d_lo, int W, int H, int w, int cmax,
                                          uint8_t *__restrict__ cost, int bx, int v, CostLds &lds)
{
    uint64_t *s_cl = lds.cl, *s_cr = lds.cr;
    const int u0 = bx * kCostTile;
    const int lo = d_lo ? d_lo[v] : 0;
    const int first = u0 - lo - (w - 1);  // right column held in s_cr[0]
    const uint64_t *crow = cr + (size_t)v * W;
    for (int t = threadIdx.x; t < kCostTile - 1 + w; t += blockDim.x) {
        const int col = first + t;
        s_cr[t] = (col >= 0 && col < W) ? crow[col] : 0ull;
    }
    for (int t = threadIdx.x; t < kCostTile; t += blockDim.x)
        s_cl[t] = (u0 + t < W) ? cl[(size_t)v * W + u0 + t] : 0ull;
    __syncthreads();
    const int npix = min(kCostTile, W - u0);
    const int nch = (w + CH - 1) / CH;
    uint8_t *out = cost + ((size_t)v * W + u0) * w;
    // items into the LDS tile (CH >= 8 and w >= 64: a wave's pieces lie a
    // cache line or more apart) or straight to the volume (narrower windows
    // keep a wave's pieces within a few lines; staging them measured slower)
    const bool staged = CH >= 8 && w >= 64;
    uint8_t *dst = staged ? lds.out : out;
    const int dstride = staged ? (nch | 1) * CH : w;
    // (uniform over the workgroup)
    const bool full = npix == kCostTile, inimg = CH >= 8 && first >= 0;
    if (full && inimg)
        cost_items<CH, true, true>(s_cl, s_cr, u0, lo, w, cmax, npix, nch, dst, dstride);
    else if (full)
        cost_items<CH, true, false>(s_cl, s_cr, u0, lo, w, cmax, npix, nch, dst, dstride);
    else
        cost_items<CH, false, false>(s_cl, s_cr, u0, lo, w, cmax, npix, nch, dst, dstride);
    if (CH >= 8 && staged) {
        // the tile's npix * w bytes are contiguous in the volume: piece t is
        // piece t % nch of pixel t / nch (exact in float: t < 64 * 32)
        __syncthreads();
        const float rn = __fdiv_rn(1.0f, (float)nch);
        for (int t = threadIdx.x; t < npix * nch; t += blockDim.x) {
            const int px = (int)(((float)t + 0.5f) * rn), c = t - px * nch;
            const uint8_t *src = lds.out + px * dstride + c * CH;
            if constexpr (CH == 16)
                *reinterpret_cast<uint4 *>(out + (size_t)t * 16) = *reinterpret_cast<const uint4 *>(src);
            else
                *reinterpret_cast<uint2 *>(out + (size_t)t * 8) = *reinterpret_cast<const uint2 *>(src);
        }
    }
}


// ---------------------------------------------------------------------------
// path aggregation, eq. (8)

struct AggParams {
    const uint8_t *cost;
    void *out;
    long long vstride;  // elements between consecutive output volumes
    int W, H, w;
    uint32_t p1x2, p2x2;  // P1, P2 replicated in both u16 halves
    int np;
    int paths[8];   // per dispatch slot: direction | output volume << 8
    int gstart[9];  // first workgroup of each slot, ascending
};

// Scanline `idx` of direction (du, dv): pixel at step i is
// (ub + su*i, vb + sv*i) for i in [i0, i1); empty when idx is past the end.
struct Line {
    int ub, vb, su, sv, i0, i1;
};

__device__ __forceinline__ Line line_geom(int idx, int du, int dv, int W, int H)
{
    Line L;
    if (dv == 0) {  // horizontal: one scanline per row
        L.vb = idx;
        L.sv = 0;
        L.su = du;
        L.ub = du > 0 ? 0 : W - 1;
        L.i0 = 0;
        L.i1 = idx < H ? W : 0;
        return L;
    }
    L.vb = dv > 0 ? 0 : H - 1;
    L.sv = dv;
    L.su = du;
    if (du == 0) {  // vertical: one scanline per column
        L.ub = idx;
        L.i0 = 0;
        L.i1 = idx < W ? H : 0;
        return L;
    }
    // diagonal: u = ell + du * i, indexed so that neighbouring idx are
    // neighbouring pixels of one row at every step
    const int nl = W + H - 1;
    const int ell = du > 0 ? idx - (H - 1) : idx;
    L.ub = ell;
    if (du > 0) {
        L.i0 = max(0, -ell);
        L.i1 = min(H, W - ell);
    } else {
        L.i0 = max(0, ell - (W - 1));
        L.i1 = min(H, ell + 1);
    }
    if (idx >= nl || L.i1 < L.i0) L.i1 = L.i0;
    return L;
}

// Buffer I/O for the aggregation loop.  Offsets at or beyond the end of a
// buffer are dropped by the hardware range check (loads return 0, stores
// are discarded), so scanlines outside the image need no branches.
constexpr uint32_t kOff = 0x80000000u;  // an offset outside every buffer
constexpr int kRsrcWord3 = 0x00020000;
// cache policy of the per-direction volume stores: non-temporal, so the
// streamed volumes do not evict the cost volume that every direction reads
constexpr int kStreamPolicy = 2;

typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v3u __attribute__((ext_vector_type(3)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kRsrcWord3);
}

// VPL cost bytes of one lane at byte offset `off` (kOff: none) plus the
// wave-uniform `soff`, which the range check may leave out: callers keep
// off + soff inside the buffer whenever off is
template <int VPL, bool ALIGNED>
__device__ __forceinline__ void buf_load_u8(Raw<VPL> &r, __amdgpu_buffer_rsrc_t rs, uint32_t off, int nvalid,
                                            uint32_t soff = 0)
{
    if constexpr (ALIGNED) {
        if constexpr (VPL == 2) {
            r.d[0] = __builtin_amdgcn_raw_buffer_load_b16(rs, off, soff, 0);
        } else if constexpr (VPL == 4) {
            r.d[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, soff, 0);
        } else if constexpr (VPL == 8) {
            const v2u t = __builtin_amdgcn_raw_buffer_load_b64(rs, off, soff, 0);
            r.d[0] = t.x;
            r.d[1] = t.y;
        } else if constexpr (VPL == 12) {
            const v3u t = __builtin_amdgcn_raw_buffer_load_b96(rs, off, soff, 0);
            r.d[0] = t.x;
            r.d[1] = t.y;
            r.d[2] = t.z;
        } else {
            const v4u t = __builtin_amdgcn_raw_buffer_load_b128(rs, off, soff, 0);
            r.d[0] = t.x;
            r.d[1] = t.y;
            r.d[2] = t.z;
            r.d[3] = t.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < Raw<VPL>::NW; ++i) r.d[i] = 0;
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const uint32_t o = (i < nvalid && off != kOff) ? off + i : kOff;
            r.d[i / 4] |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, o, soff, 0) << (8 * (i % 4));
        }
    }
}

// Inside the aggregation a lane keeps its VPL window values as NP = VPL/2
// packed pairs in a strided order: pair j holds (k0 + j, k0 + j + NP).  The
// k-1 neighbours of pair j are then pair j-1 and the k+1 neighbours pair
// j+1, so only the two end pairs need a shuffle (one alignbit each, fed by
// a DPP move from the neighbouring lane).
template <int VPL>
__device__ __forceinline__ uint32_t unpack_strided(const Raw<VPL> &r, int j)
{
    constexpr int NP = VPL / 2;
    const int blo = j, bhi = j + NP;
    const uint32_t sel = (uint32_t)(blo % 4) | (0x0Cu << 8) | ((uint32_t)(4 + bhi % 4) << 16) | (0x0Cu << 24);
    return __builtin_amdgcn_perm(r.d[bhi / 4], r.d[blo / 4], sel);
}

// strided pairs -> the lane's VPL bytes in window order, packed in dwords
template <int VPL>
__device__ __forceinline__ void pack_strided(const uint32_t (&p)[VPL / 2], uint32_t (&d)[(VPL + 3) / 4])
{
    constexpr int NP = VPL / 2;
    if constexpr (NP == 1) {
        d[0] = __builtin_amdgcn_perm(p[0], p[0], 0x0C0C0200u);
    } else if constexpr (NP == 2) {
        d[0] = __builtin_amdgcn_perm(p[1], p[0], 0x06020400u);
    } else {
        // t[q] = (p[2q].lo, p[2q+1].lo, p[2q].hi, p[2q+1].hi)
        uint32_t t[NP / 2];
#pragma unroll
        for (int q = 0; q < NP / 2; ++q) t[q] = __builtin_amdgcn_perm(p[2 * q + 1], p[2 * q], 0x06020400u);
        // byte b of the lane: b < NP -> low byte of pair b, else high of b-NP
        // = byte (b%2) + 2*(b >= NP) of t[(b % NP) / 2]
#pragma unroll
        for (int q = 0; q < (VPL + 3) / 4; ++q) {
            const int b0 = 4 * q, b2 = 4 * q + 2;
            const int ta = (b0 % NP) / 2, tb = (b2 % NP) / 2;
            const uint32_t sa = (uint32_t)((b0 >= NP) ? 2 : 0), sb = (uint32_t)((b2 >= NP) ? 2 : 0);
            // bytes b0, b0+1 come from t[ta], bytes b2, b2+1 from t[tb]
            const uint32_t sel = (sa) | ((sa + 1) << 8) | ((4 + sb) << 16) | ((5 + sb) << 24);
            d[q] = __builtin_amdgcn_perm(t[tb], t[ta], sel);
        }
    }
}

// stores of one lane's aggregated values (strided pairs) at element offset
// `off` of the output volume (kOff: dropped by the range check) plus the
// wave-uniform `soff` elements (as for buf_load_u8)
template <int VPL, bool ALIGNED, bool L8>
__device__ __forceinline__ void store_strided(const uint32_t (&v)[VPL / 2], __amdgpu_buffer_rsrc_t rs, uint32_t off,
                                              int nvalid, uint32_t soff = 0)
{
    constexpr int NP = VPL / 2;
    if constexpr (ALIGNED && L8) {
        uint32_t d[(VPL + 3) / 4];
        pack_strided<VPL>(v, d);
        if constexpr (VPL == 2) {
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)d[0], rs, off, soff, kStreamPolicy);
        } else if constexpr (VPL == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(d[0], rs, off, soff, kStreamPolicy);
        } else if constexpr (VPL == 8) {
            const v2u t = {d[0], d[1]};
            __builtin_amdgcn_raw_buffer_store_b64(t, rs, off, soff, kStreamPolicy);
        } else if constexpr (VPL == 12) {
            const v3u t = {d[0], d[1], d[2]};
            __builtin_amdgcn_raw_buffer_store_b96(t, rs, off, soff, kStreamPolicy);
        } else {
            const v4u t = {d[0], d[1], d[2], d[3]};
            __builtin_amdgcn_raw_buffer_store_b128(t, rs, off, soff, kStreamPolicy);
        }
    } else {
        // value i of the lane: pair i % NP, half i / NP
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
            const uint32_t val = (i < NP) ? (v[i] & 0xFFFFu) : (v[i - NP] >> 16);
            const bool ok = i < nvalid && off != kOff;
            if (L8)
                __builtin_amdgcn_raw_buffer_store_b8((unsigned char)val, rs, ok ? off + i : kOff, soff, kStreamPolicy);
            else
                __builtin_amdgcn_raw_buffer_store_b16((unsigned short)val, rs, ok ? 2 * (off + i) : kOff, 2 * soff,
                                                      kStreamPolicy);
        }
    }
}

// vector memory instructions issued per aggregation step (loads, stores)
template <int VPL, bool ALIGNED, bool L8>
struct VmemPerStep {
    static constexpr int loads = ALIGNED ? 1 : VPL;
    static constexpr int stores = (ALIGNED && L8) ? 1 : VPL;
    static constexpr int total = loads + stores;
};

// s_waitcnt immediate: wait until at most n vector memory operations are
// outstanding (gfx9 encoding; expcnt and lgkmcnt left at their maxima)
constexpr int vmcnt_imm(int n)
{
    return ((n > 63 ? 63 : n) & 0xF) | (0x7 << 4) | (0xF << 8) | (((n > 63 ? 63 : n) >> 4) << 14);
}

enum { kHorizontal = 0, kVertical = 1, kDiagonal = 2 };

// One workgroup's scanlines of one direction.  KIND selects the bookkeeping:
// horizontal and vertical scanlines cover the whole image edge to edge, so
// every lane is active at every step (tail lines past the last scanline
// repeat the last one, writing identical values to identical addresses);
// diagonal scanlines enter and leave the image at different steps, and
// only their loads and stores are masked.  Before a scanline enters the
// image its loads return 0, which keeps L' at 0, so the first in-image
// step computes L = C without any reset.
template <int G, int VPL, bool ALIGNED, bool PAD, bool L8, int PF, int KIND>
__device__ __forceinline__ void agg_scan(const AggParams &a, __amdgpu_buffer_rsrc_t rc, __amdgpu_buffer_rsrc_t ro,
                                         int du, int dv, int g)
{
    constexpr int NP = VPL / 2;
    constexpr int UNROLL = 2 * PF;  // steps per loop iteration
    constexpr int LPWAVE = 64 / G;  // scanlines per wave
    const int lane = threadIdx.x & (G - 1);
    const int lw = threadIdx.x / G;
    const int W = a.W, H = a.H, w = a.w;
    const int lpw = (int)blockDim.x / G;  // scanlines per workgroup

    int I0 = 0, I1;
    int idx = g * lpw + lw;
    if constexpr (KIND == kHorizontal) {
        idx = min(idx, H - 1);
        I1 = W;
    } else if constexpr (KIND == kVertical) {
        idx = min(idx, W - 1);
        I1 = H;
    } else {
        // the wave's step range: the union over its own scanlines
        I0 = 1 << 30;
        I1 = 0;
        const int first = g * lpw + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * LPWAVE;
        for (int l = 0; l < LPWAVE; ++l) {
            const Line t = line_geom(first + l, du, dv, W, H);
            if (t.i1 > t.i0) {
                I0 = min(I0, t.i0);
                I1 = max(I1, t.i1);
            }
        }
        if (I1 <= I0) return;
    }
    const Line ln = line_geom(idx, du, dv, W, H);
    const int kbase = lane * VPL;
    const int nvalid = min(max(w - kbase, 0), VPL);
    const bool has = nvalid > 0;
    // element offset of this lane's values at step i: off0 + i * stride
    // (wrapping 32-bit arithmetic; exact whenever the pixel is in the image);
    // lanes past the window never touch memory (offset stays kOff)
    const uint32_t stride = has ? (uint32_t)((ln.sv * W + ln.su) * w) : 0u;
    const uint32_t off0 = has ? (uint32_t)((ln.vb * W + ln.ub) * w + kbase) : kOff;
    const uint32_t li0 = (uint32_t)ln.i0, llen = (uint32_t)(ln.i1 - ln.i0);
    auto offset = [&](int i) -> uint32_t {
        const uint32_t o = off0 + (uint32_t)i * stride;
        if constexpr (KIND == kDiagonal)
            return ((uint32_t)i - li0 < llen) ? o : kOff;
        else
            return o;
    };

    // The end lanes of a group have no neighbour across the group edge:
    // the half they use of their DPP neighbour (0 at a row edge, another
    // scanline's value inside a row, at most kInf2 + P2) is raised to at
    // least kInf2, which acts as outside the window (kInf2 + P1 - m_q > P2).
    const uint32_t edge_l = lane == 0 ? kInf2 : 0u;
    const uint32_t edge_r = lane == G - 1 ? kInf2 : 0u;
    // narrow lanes (one dword of cost bytes): the pair unpacking and the
    // padding in one byte permutation, padded halves taking kInf2's bytes
    uint32_t psel[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const uint32_t lo = j >= nvalid ? 0x0504u : ((uint32_t)j | 0x0C00u);
        const uint32_t hi = j + NP >= nvalid ? 0x0706u : ((uint32_t)(j + NP) | 0x0C00u);
        psel[j] = lo | (hi << 16);
    }
    uint32_t padp[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        padp[j] = 0;
        if (PAD) {
            if (j >= nvalid) padp[j] |= kPad;
            if (j + NP >= nvalid) padp[j] |= kPad << 16;
        }
    }

    Raw<VPL> ring[PF];
#pragma unroll
    for (int s = 0; s < PF; ++s)
        buf_load_u8<VPL, ALIGNED>(ring[s], rc, (I0 + s < I1) ? offset(I0 + s) : kOff, nvalid);

    // Lq: the predecessor's L (as stored), mnq: its running pair minimum.
    // A scanline starts from Lq = 0 (then L = C + min(0, P1, P2) - 0 = C).
    uint32_t Lq[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) Lq[j] = 0;
    uint32_t mnq = 0;

    // one step: consume ring slot S (loaded PF steps ago), refill it for
    // step i + PF from offset lo (+ scalar lso), aggregate, store at so
    // (+ sso)
    auto step = [&](const int S, const uint32_t lo, const uint32_t lso, const uint32_t so,
                    const uint32_t sso) __attribute__((always_inline)) {
        // ring[S] was loaded PF steps ago; everything issued since may stay
        // in flight.  The scheduling fence keeps later steps' reads of the
        // ring below this wait.
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(VmemPerStep<VPL, ALIGNED, L8>::stores +
                                             (PF - 1) * VmemPerStep<VPL, ALIGNED, L8>::total));
        uint32_t c2[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            if constexpr (PAD && NP <= 2)
                c2[j] = __builtin_amdgcn_perm(kInf2, (uint32_t)ring[S].d[0], psel[j]);
            else
                c2[j] = unpack_strided(ring[S], j) | padp[j];
        }
        buf_load_u8<VPL, ALIGNED>(ring[S], rc, lo, nvalid, lso);
        // m_q = min_k L(q,k) in both u16 halves: the lane's pair minimum
        // (from the end of the previous step) folded over its halves, then
        // reduced over the group as 32-bit values (such doubled values order
        // as m_q does).  This chain is independent of the neighbour terms
        // below, which overlap it.
        const uint32_t mm = group_min<G>(pk_min_halves(mnq));
        // end neighbours across the lane edges (outside the window: 0x3FFF)
        // (e: only its high half is used, so a 32-bit maximum, which the
        // compiler folds into the DPP move; f: its low half, a packed one
        // unless the group is a whole row)
        const uint32_t e = max(dpp0<kRowShr1>(Lq[NP - 1]), edge_l);
        uint32_t f;
        if constexpr (G == 16)  // (edge lanes read the zero fill: a 32-bit maximum is exact)
            f = max(dpp0<kRowShl1>(Lq[0]), edge_r);
        else
            f = pk_max(dpp0<kRowShl1>(Lq[0]), edge_r);
        // L(p,k) = C(p,k) + min(L(q,k), L(q,k+-1) + P1, m_q + P2) - m_q
        //        = C(p,k) + min(t - m_q, P2),  t = min(L(q,k), L(q,k+-1) + P1) >= m_q,
        // so m_q enters only after t (no u16 value goes below 0 or past
        // 0x3FFF + P1 + P2)
        uint32_t Ln[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const uint32_t lft = j ? Lq[j - 1] : __builtin_amdgcn_alignbit(Lq[NP - 1], e, 16);
            const uint32_t rgt = j + 1 < NP ? Lq[j + 1] : __builtin_amdgcn_alignbit(f, Lq[0], 16);
            const uint32_t t = pk_min(Lq[j], pk_add(pk_min(lft, rgt), a.p1x2));
            Ln[j] = pk_add(pk_min(pk_sub(t, mm), a.p2x2), c2[j]);
        }
        const uint32_t mn = pk_min_tree<NP>(Ln);
        store_strided<VPL, ALIGNED, L8>(Ln, ro, so, nvalid, sso);
#pragma unroll
        for (int j = 0; j < NP; ++j) Lq[j] = Ln[j];
        mnq = mn;
    };

    // step i with its accesses checked against the scanline's end: a step
    // past it, or a prefetch past it, is dropped
    auto checked_step = [&](const int i, const int S) __attribute__((always_inline)) {
        step(S, i + PF < I1 ? offset(i + PF) : kOff, 0u, i < I1 ? offset(i) : kOff, 0u);
    };

    // The first turn of the ring runs outside the loops: at a loop head
    // every slot was then refilled by a step, exactly as on the back edge,
    // so the compiler sees the same loads in flight from both sides and
    // needs no deeper wait there than inside the loop.  The step count is
    // padded to PF + a multiple of UNROLL; padded steps load nothing and
    // store nothing.
#pragma unroll
    for (int S = 0; S < PF; ++S) checked_step(I0 + S, S);
    const int nblk = (I1 - I0 - PF + UNROLL - 1) / UNROLL;
    // Blocks whose steps and prefetches all lie before I1 (the last prefetch
    // of block blk is step I0 + 2 PF + (blk + 1) UNROLL - 1) need no range
    // checks.  Horizontal and vertical scanlines also share one stride
    // (every lane with values advances by it): such a block takes one
    // vector offset per access kind and puts the step's place in the block
    // into the scalar offset, never negative (a block walking down the
    // addresses is based at its last step), every access staying inside the
    // volume.
    const int nfull = min(nblk, max(0, (I1 - I0 - 2 * PF) / UNROLL));
    const int ustride = __builtin_amdgcn_readfirstlane((dv * W + du) * w);
    const int sb = ustride < 0 ? UNROLL - 1 : 0;
    for (int blk = 0; blk < nfull; ++blk) {
        const int ib = I0 + PF + blk * UNROLL;
        if constexpr (KIND == kDiagonal) {
#pragma unroll
            for (int s = 0; s < UNROLL; ++s) step(s % PF, offset(ib + s + PF), 0u, offset(ib + s), 0u);
        } else {
            const uint32_t vl = offset(ib + PF + sb), vs = offset(ib + sb);
#pragma unroll
            for (int s = 0; s < UNROLL; ++s) {
                const uint32_t so = (uint32_t)__builtin_amdgcn_readfirstlane((s - sb) * ustride);
                step(s % PF, vl, so, vs, so);
            }
        }
    }
    for (int blk = nfull; blk < nblk; ++blk) {
#pragma unroll
        for (int s = 0; s < UNROLL; ++s) checked_step(I0 + PF + blk * UNROLL + s, s % PF);
    }
}


// One workgroup-sized piece of the aggregation: direction r, scanline group g
// of the volume described by `a`, written to output volume `vol`.  The
// horizontal directions may take a lane mapping of their own (GH, VPLH,
// PADH, PFH): their scanlines are the longest dependency chains, which the
// widest groups run with the fewest dependent instructions per step.
template <int G, int VPL, bool ALIGNED, bool PAD, bool L8, int PF, int GH = G, int VPLH = VPL, bool PADH = PAD,
          int PFH = PF>
__device__ __forceinline__ void agg_item(const AggParams &a, int r, int vol, int g)
{
    const int du = __builtin_amdgcn_readfirstlane(dir_du(r)), dv = __builtin_amdgcn_readfirstlane(dir_dv(r));
    // buffer descriptors (scalar registers): the cost volume and this
    // direction's output volume
    const uint32_t nbytes = (uint32_t)a.W * (uint32_t)a.H * (uint32_t)a.w;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cost, nbytes);
    const __amdgpu_buffer_rsrc_t ro =
        L8 ? make_rsrc(static_cast<const uint8_t *>(a.out) + (size_t)vol * a.vstride, nbytes)
           : make_rsrc(static_cast<const uint16_t *>(a.out) + (size_t)vol * a.vstride, nbytes * 2u);
    if (dv == 0) {
        // the longest dependency chains: issue them first on a shared SIMD
        __builtin_amdgcn_s_setprio(2);
        agg_scan<GH, VPLH, ALIGNED, PADH, L8, PFH, kHorizontal>(a, rc, ro, du, dv, g);
        __builtin_amdgcn_s_setprio(0);
    } else if (du == 0) {
        agg_scan<G, VPL, ALIGNED, PAD, L8, PF, kVertical>(a, rc, ro, du, dv, g);
    } else {
        agg_scan<G, VPL, ALIGNED, PAD, L8, PF, kDiagonal>(a, rc, ro, du, dv, g);
    }
}

// ---------------------------------------------------------------------------
// winner-take-all, sub-pixel parabola, eq. (10) offset

template <int G, int VPL>
__device__ __forceinline__ void select_and_write(const uint32_t (&S)[VPL / 2], int kbase, int w, int lane,
                                                 int lo, long long pix, uint16_t *dint, float *dsub)
{
    constexpr int NP = VPL / 2;
    uint32_t best = 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = kbase + 2 * j;
        const uint32_t s0 = S[j] & 0xFFFFu, s1 = S[j] >> 16;
        if (k < w) best = min(best, (s0 << 8) | (uint32_t)k);
        if (k + 1 < w) best = min(best, (s1 << 8) | (uint32_t)(k + 1));
    }
    best = group_min<G>(best);
    const int ks = (int)(best & 0xFFu);
    const int s0 = (int)(best >> 8);
    uint32_t sm = 0, sp = 0;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = kbase + 2 * j;
        const uint32_t a = S[j] & 0xFFFFu, b = S[j] >> 16;
        if (k == ks - 1) sm = a;
        if (k + 1 == ks - 1) sm = b;
        if (k == ks + 1) sp = a;
        if (k + 1 == ks + 1) sp = b;
    }
    sm = group_max<G>(sm);
    sp = group_max<G>(sp);
    if (lane == 0) {
        dint[pix] = (uint16_t)(lo + ks);
        if (dsub) {
            float delta = 0.0f;
            if (ks > 0 && ks < w - 1) {
                const int num = (int)sm - (int)sp;
                const int den = 2 * ((int)sm - 2 * s0 + (int)sp);
                delta = __fdiv_rn((float)num, (float)den);
            }
            dsub[pix] = __fadd_rn((float)(lo + ks), delta);
        }
    }
}


// Selection on uint8 per-direction volumes: the byte sums are formed SWAR
// style, even and odd bytes of each dword accumulating in the two u16
// halves of separate registers (sums <= npaths * (Cmax + P2) <= 65535, so
// halves never carry).  ev[q] then holds S at window indices (4q, 4q+2) and
// od[q] at (4q+1, 4q+3) of the lane's range.
template <int G, int VPL>
__device__ __forceinline__ void select_swar(const uint32_t (&ev)[Raw<VPL>::NW], const uint32_t (&od)[Raw<VPL>::NW],
                                            int kbase, int w, int lane, int lo, long long pix, uint16_t *dint,
                                            float *dsub)
{
    constexpr int NW = Raw<VPL>::NW;
    uint32_t best = 0xFFFFFFFFu;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int k = kbase + 4 * q + h;
            const uint32_t sv = ((h & 1) ? od[q] : ev[q]) >> (16 * (h >> 1)) & 0xFFFFu;
            if (4 * q + h < VPL && k < w) best = min(best, (sv << 8) | (uint32_t)k);
        }
    }
    best = group_min<G>(best);
    const int ks = (int)(best & 0xFFu);
    const int s0 = (int)(best >> 8);
    uint32_t sm = 0, sp = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int k = kbase + 4 * q + h;
            const uint32_t sv = ((h & 1) ? od[q] : ev[q]) >> (16 * (h >> 1)) & 0xFFFFu;
            if (4 * q + h < VPL) {
                if (k == ks - 1) sm = sv;
                if (k == ks + 1) sp = sv;
            }
        }
    }
    sm = group_max<G>(sm);
    sp = group_max<G>(sp);
    if (lane == 0) {
        dint[pix] = (uint16_t)(lo + ks);
        if (dsub) {
            float delta = 0.0f;
            if (ks > 0 && ks < w - 1) {
                const int num = (int)sm - (int)sp;
                const int den = 2 * ((int)sm - 2 * s0 + (int)sp);
                delta = __fdiv_rn((float)num, (float)den);
            }
            dsub[pix] = __fadd_rn((float)(lo + ks), delta);
        }
    }
}


// selection for pixel group `pblock` (blockDim / G pixels, G lanes each) of
// one volume set
template <int G, int VPL, bool ALIGNED, bool L8>
__device__ __forceinline__ void wta_paths_group(const void *__restrict__ vols, long long vstride, int np,
                                                const int32_t *__restrict__ d_lo, int W, int H, int w,
                                                uint16_t *__restrict__ dint, float *__restrict__ dsub,
                                                long long pblock)
{
    constexpr int NP = VPL / 2;
    const int lane = threadIdx.x & (G - 1);
    const long long pix = pblock * (blockDim.x / G) + (threadIdx.x / G);
    if (pix >= (long long)W * H) return;
    const int kbase = lane * VPL;
    const int nvalid = min(max(w - kbase, 0), VPL);
    const int v = (int)(pix / W);
    if constexpr (L8 && VPL % 4 == 0) {
        constexpr int NW = Raw<VPL>::NW;
        uint32_t ev[NW], od[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) ev[q] = od[q] = 0;
        if (nvalid > 0 && np == 8) {
            // all eight volumes in flight at once
            const uint8_t *base = static_cast<const uint8_t *>(vols) + pix * w + kbase;
            Raw<VPL> x[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) load_u8<VPL, ALIGNED>(x[r], base + r * vstride, nvalid);
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    ev[q] += x[r].d[q] & 0x00FF00FFu;
                    od[q] += (x[r].d[q] >> 8) & 0x00FF00FFu;
                }
        } else if (nvalid > 0) {
            const uint8_t *base = static_cast<const uint8_t *>(vols) + pix * w + kbase;
            int r = 0;
            for (; r + 1 < np; r += 2) {
                Raw<VPL> x, y;
                load_u8<VPL, ALIGNED>(x, base + r * vstride, nvalid);
                load_u8<VPL, ALIGNED>(y, base + (r + 1) * vstride, nvalid);
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    ev[q] += (x.d[q] & 0x00FF00FFu) + (y.d[q] & 0x00FF00FFu);
                    od[q] += ((x.d[q] >> 8) & 0x00FF00FFu) + ((y.d[q] >> 8) & 0x00FF00FFu);
                }
            }
            if (r < np) {
                Raw<VPL> x;
                load_u8<VPL, ALIGNED>(x, base + r * vstride, nvalid);
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    ev[q] += x.d[q] & 0x00FF00FFu;
                    od[q] += (x.d[q] >> 8) & 0x00FF00FFu;
                }
            }
        }
        select_swar<G, VPL>(ev, od, kbase, w, lane, d_lo ? d_lo[v] : 0, pix, dint, dsub);
    } else {
        uint32_t S[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) S[j] = 0;
        if (nvalid > 0) {
            for (int r = 0; r < np; ++r) {
                if (L8) {
                    Raw<VPL> raw;
                    load_u8<VPL, ALIGNED>(raw, static_cast<const uint8_t *>(vols) + r * vstride + pix * w + kbase,
                                          nvalid);
#pragma unroll
                    for (int j = 0; j < NP; ++j) S[j] = pk_add(S[j], unpack_pair(raw, j));
                } else {
                    uint32_t t[NP];
                    load_u16_pairs<VPL, ALIGNED>(
                        t, static_cast<const uint16_t *>(vols) + r * vstride + pix * w + kbase, nvalid);
#pragma unroll
                    for (int j = 0; j < NP; ++j) S[j] = pk_add(S[j], t[j]);
                }
            }
        }
        select_and_write<G, VPL>(S, kbase, w, lane, d_lo ? d_lo[v] : 0, pix, dint, dsub);
    }
}


}  // namespace dev
}  // namespace sgm
