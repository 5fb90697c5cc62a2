// HIP kernels of the SGM hot path for gfx950 (CDNA4, wave64).
//
// Data layout (all row-major, disparity fastest):
//   census codes   uint64 [H][W]
//   cost C         uint8  [H][W][w]       (Sec. II-B, c(p,d); census + Hamming)
//   per-path L_r   uint8 or uint16 [H][W][w], one volume per direction
//   summed S       uint16 [H][W][w]       (eq. (9))
//
// Lane mapping of the aggregation (eq. (8)): a scanline of the path is
// carried by one 16-lane DPP row; lane j holds the VPL consecutive window
// indices [j*VPL, (j+1)*VPL) as VPL/2 packed u16 pairs.  One wave64 thus
// advances four scanlines, one workgroup of 256 threads sixteen.  Per step
// a lane
//   * loads its VPL cost bytes (prefetched PF steps ahead into registers),
//   * forms the k-1 / k+1 neighbour pairs with v_alignbit inside the lane
//     and one row_shr / row_shl DPP move across lanes,
//   * evaluates min(L'(k), min(L'(k-1), L'(k+1)) + P1, P2) + C with packed
//     u16 min/add (L' is the previous pixel's L minus its minimum, so the
//     "m_q + P2" term of eq. (8) becomes the constant P2),
//   * reduces the minimum over the window with four DPP steps and
//     subtracts it for the next step.
// Window indices k >= w (when 16*VPL > w) carry the cost 0x3FFF; their
// aggregated values then never win a minimum because Cmax + 2 P2 < 0x3FFF.
//
// Scanlines of every direction are independent, so all directions of a
// frame are aggregated by one launch; each writes its own L_r volume (uint8
// when Cmax + P2 <= 255) and the selection kernel sums them.  Vertical and
// diagonal scanlines are grouped so that 16 neighbouring scanlines sit on
// 16 neighbouring pixels of the same image row at every step (a sheared
// index for the diagonals), which keeps every wave's loads and stores on
// contiguous 512-byte runs.

#include "sgm_internal.h"

namespace sgm {
namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr uint32_t kInf2 = 0x3FFF3FFFu;  // pair of "outside the window" values
constexpr uint32_t kPad = 0x3FFFu;

__device__ __forceinline__ uint32_t pk_min(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
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

// DPP move: lanes whose source lies outside their 16-lane row keep `old`.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t src)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, CTRL, 0xF, 0xF, false);
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

template <int VPL>
struct Raw {
    static constexpr int NW = (VPL + 3) / 4;
    uint32_t d[NW];
};

template <int VPL, bool ALIGNED>
__device__ __forceinline__ void load_u8(Raw<VPL> &r, const uint8_t *p, int nvalid)
{
    if constexpr (ALIGNED) {
        if constexpr (VPL == 2) {
            r.d[0] = *reinterpret_cast<const uint16_t *>(p);
        } else if constexpr (VPL == 4) {
            r.d[0] = *reinterpret_cast<const uint32_t *>(p);
        } else if constexpr (VPL == 8) {
            const uint2 t = *reinterpret_cast<const uint2 *>(p);
            r.d[0] = t.x;
            r.d[1] = t.y;
        } else if constexpr (VPL == 12) {
            const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
            r.d[0] = q[0];
            r.d[1] = q[1];
            r.d[2] = q[2];
        } else {
            const uint4 t = *reinterpret_cast<const uint4 *>(p);
            r.d[0] = t.x;
            r.d[1] = t.y;
            r.d[2] = t.z;
            r.d[3] = t.w;
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

template <int N>
__global__ __launch_bounds__(256) void k_census(const uint8_t *__restrict__ img, int pitch, int W, int H,
                                                uint64_t *__restrict__ out)
{
    constexpr int R = N / 2, TW = 64, TH = 4, LW = TW + 2 * R, LH = TH + 2 * R;
    __shared__ uint8_t tile[LH][LW];
    const int u0 = blockIdx.x * TW, v0 = blockIdx.y * TH;
    for (int t = threadIdx.x; t < LH * LW; t += blockDim.x) {
        const int ty = t / LW, tx = t % LW;
        const int v = min(max(v0 + ty - R, 0), H - 1);
        const int u = min(max(u0 + tx - R, 0), W - 1);
        tile[ty][tx] = img[(size_t)v * pitch + u];
    }
    __syncthreads();
    const int tx = threadIdx.x % TW, ty = threadIdx.x / TW;
    const int u = u0 + tx, v = v0 + ty;
    if (u >= W || v >= H) return;
    const int c = tile[ty + R][tx + R];
    uint64_t bits = 0;
    int b = 0;
#pragma unroll
    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
            if (dx == 0 && dy == 0) continue;
            bits |= (uint64_t)(tile[ty + R + dy][tx + R + dx] < c) << b;
            ++b;
        }
    out[(size_t)v * W + u] = bits;
}

// ---------------------------------------------------------------------------
// matching cost: C(u,v,k) = popcount(cL(u,v) ^ cR(u - d_lo(v) - k, v))

template <int VPL, bool ALIGNED>
__global__ __launch_bounds__(256) void k_cost(const uint64_t *__restrict__ cl, const uint64_t *__restrict__ cr,
                                              const int32_t *__restrict__ d_lo, int W, int H, int w, int cmax,
                                              uint8_t *__restrict__ cost)
{
    __shared__ uint64_t s_cr[16 + 256];
    const int v = blockIdx.y;
    const int u0 = blockIdx.x * 16;
    const int lo = d_lo ? d_lo[v] : 0;
    const int first = u0 - lo - (w - 1);  // right column held in s_cr[0]
    for (int t = threadIdx.x; t < 15 + w; t += blockDim.x) {
        const int col = first + t;
        s_cr[t] = (col >= 0 && col < W) ? cr[(size_t)v * W + col] : 0ull;
    }
    __syncthreads();
    const int lane = threadIdx.x & 15;
    const int u = u0 + (threadIdx.x >> 4);
    const int kbase = lane * VPL;
    if (u >= W || kbase >= w) return;
    const int nvalid = min(VPL, w - kbase);
    const uint64_t a = cl[(size_t)v * W + u];
    uint32_t pairs[VPL / 2];
#pragma unroll
    for (int j = 0; j < VPL / 2; ++j) {
        uint32_t pr = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = kbase + 2 * j + h;
            const int col = u - lo - k;
            uint32_t c = (uint32_t)cmax;
            if (col >= 0 && k < w) c = (uint32_t)__popcll(a ^ s_cr[col - first]);
            pr |= c << (16 * h);
        }
        pairs[j] = pr;
    }
    store_u8_pairs<VPL, ALIGNED>(cost + ((size_t)v * W + u) * w + kbase, pairs, nvalid);
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
    int lines_per_wg;
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

typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v3u __attribute__((ext_vector_type(3)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kRsrcWord3);
}

// VPL cost bytes of one lane at byte offset `off` (kOff: none)
template <int VPL, bool ALIGNED>
__device__ __forceinline__ void buf_load_u8(Raw<VPL> &r, __amdgpu_buffer_rsrc_t rs, uint32_t off, int nvalid)
{
    if constexpr (ALIGNED) {
        if constexpr (VPL == 2) {
            r.d[0] = __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
        } else if constexpr (VPL == 4) {
            r.d[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
        } else if constexpr (VPL == 8) {
            const v2u t = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
            r.d[0] = t.x;
            r.d[1] = t.y;
        } else if constexpr (VPL == 12) {
            const v3u t = __builtin_amdgcn_raw_buffer_load_b96(rs, off, 0, 0);
            r.d[0] = t.x;
            r.d[1] = t.y;
            r.d[2] = t.z;
        } else {
            const v4u t = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
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
            r.d[i / 4] |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, o, 0, 0) << (8 * (i % 4));
        }
    }
}

// packed u16 pairs of one lane -> uint8 (L8) or uint16 values at element
// offset `off` of the buffer (kOff: none)
template <int VPL, bool ALIGNED, bool L8>
__device__ __forceinline__ void buf_store_pairs(const uint32_t (&v)[VPL / 2], __amdgpu_buffer_rsrc_t rs, uint32_t off,
                                                int nvalid)
{
    constexpr int NP = VPL / 2;
    if constexpr (ALIGNED && L8) {
        if constexpr (VPL == 2) {
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)__builtin_amdgcn_perm(v[0], v[0], 0x0C0C0200u), rs,
                                                  off, 0, 0);
        } else if constexpr (VPL == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(pack_bytes(v[0], v[1]), rs, off, 0, 0);
        } else if constexpr (VPL == 8) {
            const v2u t = {pack_bytes(v[0], v[1]), pack_bytes(v[2], v[3])};
            __builtin_amdgcn_raw_buffer_store_b64(t, rs, off, 0, 0);
        } else if constexpr (VPL == 12) {
            const v3u t = {pack_bytes(v[0], v[1]), pack_bytes(v[2], v[3]), pack_bytes(v[4], v[5])};
            __builtin_amdgcn_raw_buffer_store_b96(t, rs, off, 0, 0);
        } else {
            const v4u t = {pack_bytes(v[0], v[1]), pack_bytes(v[2], v[3]), pack_bytes(v[4], v[5]),
                           pack_bytes(v[6], v[7])};
            __builtin_amdgcn_raw_buffer_store_b128(t, rs, off, 0, 0);
        }
    } else if constexpr (ALIGNED) {
        const uint32_t bo = off == kOff ? kOff : off * 2;
        if constexpr (NP == 1) {
            __builtin_amdgcn_raw_buffer_store_b32(v[0], rs, bo, 0, 0);
        } else if constexpr (NP == 2) {
            const v2u t = {v[0], v[1]};
            __builtin_amdgcn_raw_buffer_store_b64(t, rs, bo, 0, 0);
        } else {
#pragma unroll
            for (int j = 0; j < NP; j += 2) {
                const v2u t = {v[j], v[j + 1]};
                __builtin_amdgcn_raw_buffer_store_b64(t, rs, bo == kOff ? kOff : bo + 4 * j, 0, 0);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < NP; ++j) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = 2 * j + h;
                const uint32_t val = h ? (v[j] >> 16) : (v[j] & 0xFFFFu);
                const bool ok = i < nvalid && off != kOff;
                if (L8)
                    __builtin_amdgcn_raw_buffer_store_b8((unsigned char)val, rs, ok ? off + i : kOff, 0, 0);
                else
                    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)val, rs, ok ? 2 * (off + i) : kOff, 0,
                                                          0);
            }
        }
    }
}

// vector memory instructions issued per aggregation step (loads, stores)
template <int VPL, bool ALIGNED, bool L8>
struct VmemPerStep {
    static constexpr int loads = ALIGNED ? 1 : VPL;
    static constexpr int stores = !ALIGNED ? VPL : (L8 ? 1 : (VPL / 2 <= 2 ? 1 : VPL / 4));
    static constexpr int total = loads + stores;
};

// s_waitcnt immediate that waits until at most n vector memory operations
// are outstanding (gfx9 encoding; expcnt and lgkmcnt left at their maxima)
constexpr int vmcnt_imm(int n)
{
    return (n > 63 ? 63 : n) < 0 ? 0x0F70 : (((n > 63 ? 63 : n) & 0xF) | (0x7 << 4) | (0xF << 8) | (((n > 63 ? 63 : n) >> 4) << 14));
}

template <int VPL, bool ALIGNED, bool PAD, bool L8, int PF>
__global__ __launch_bounds__(256) void k_aggregate(AggParams a)
{
    constexpr int NP = VPL / 2;
    const int lane = threadIdx.x & 15;
    const int lw = threadIdx.x >> 4;
    int slot = 0;
    while (slot + 1 < a.np && (int)blockIdx.x >= a.gstart[slot + 1]) ++slot;
    const int r = a.paths[slot] & 0xFF;
    const int vol = a.paths[slot] >> 8;
    const int g = (int)blockIdx.x - a.gstart[slot];
    const int du = dir_du(r), dv = dir_dv(r);
    const int W = a.W, H = a.H, w = a.w;

    // step range of the whole workgroup (uniform) and of this scanline
    int I0 = 1 << 30, I1 = 0;
    for (int l = 0; l < a.lines_per_wg; ++l) {
        const Line t = line_geom(g * a.lines_per_wg + l, du, dv, W, H);
        if (t.i1 > t.i0) {
            I0 = min(I0, t.i0);
            I1 = max(I1, t.i1);
        }
    }
    if (I1 <= I0) return;
    const Line ln = line_geom(g * a.lines_per_wg + lw, du, dv, W, H);
    const int kbase = lane * VPL;
    const int nvalid = min(max(w - kbase, 0), VPL);
    const int nlen = nvalid > 0 ? ln.i1 - ln.i0 : 0;  // steps this lane loads and stores
    // element offset of this lane's values at step i: off0 + i * stride
    // (wrapping 32-bit arithmetic; exact whenever the pixel is in the image)
    const uint32_t off0 = (uint32_t)((ln.vb * W + ln.ub) * w + kbase);
    const uint32_t stride = (uint32_t)((ln.sv * W + ln.su) * w);
    const uint32_t nbytes = (uint32_t)W * (uint32_t)H * (uint32_t)w;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cost, nbytes);
    const __amdgpu_buffer_rsrc_t ro =
        L8 ? make_rsrc(static_cast<const uint8_t *>(a.out) + (size_t)vol * a.vstride, nbytes)
           : make_rsrc(static_cast<const uint16_t *>(a.out) + (size_t)vol * a.vstride, nbytes * 2u);

    uint32_t padp[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        padp[j] = 0;
        if (PAD) {
            if (2 * j >= nvalid) padp[j] |= kPad;
            if (2 * j + 1 >= nvalid) padp[j] |= kPad << 16;
        }
    }

    Raw<VPL> ring[PF];
#pragma unroll
    for (int s = 0; s < PF; ++s) {
        const int i = I0 + s;
        const uint32_t o = (uint32_t)(i - ln.i0) < (uint32_t)nlen ? off0 + (uint32_t)i * stride : kOff;
        buf_load_u8<VPL, ALIGNED>(ring[s], rc, o, nvalid);
    }

    uint32_t Lp[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) Lp[j] = 0;

    // the step count is padded to a multiple of PF; padded steps are
    // inactive in every lane
    const int nblk = (I1 - I0 + PF - 1) / PF;
    for (int blk = 0; blk < nblk; ++blk) {
#pragma unroll
        for (int s = 0; s < PF; ++s) {
            const int i = I0 + blk * PF + s;
            const bool act = (uint32_t)(i - ln.i0) < (uint32_t)(ln.i1 - ln.i0);
            const bool io = (uint32_t)(i - ln.i0) < (uint32_t)nlen;
            // ring[s] was loaded PF steps ago; everything issued since then
            // may stay in flight.  The scheduling fence keeps later steps'
            // reads of the ring below this wait.
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(VmemPerStep<VPL, ALIGNED, L8>::stores +
                                                 (PF - 1) * VmemPerStep<VPL, ALIGNED, L8>::total));
            uint32_t c2[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j) c2[j] = unpack_pair(ring[s], j) | padp[j];
            {
                const int ip = i + PF;
                const uint32_t o =
                    (uint32_t)(ip - ln.i0) < (uint32_t)nlen ? off0 + (uint32_t)ip * stride : kOff;
                buf_load_u8<VPL, ALIGNED>(ring[s], rc, o, nvalid);
            }
            // neighbours across the lane edges (outside the window: 0x3FFF)
            const uint32_t le = dpp<kRowShr1>(kInf2, Lp[NP - 1]);
            const uint32_t re = dpp<kRowShl1>(kInf2, Lp[0]);
            uint32_t Ln[NP];
            uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const uint32_t lft = __builtin_amdgcn_alignbit(Lp[j], j ? Lp[j - 1] : le, 16);
                const uint32_t rgt = __builtin_amdgcn_alignbit(j + 1 < NP ? Lp[j + 1] : re, Lp[j], 16);
                uint32_t t = pk_add(pk_min(lft, rgt), a.p1x2);
                t = pk_min(pk_min(t, Lp[j]), a.p2x2);
                Ln[j] = pk_add(t, c2[j]);
                mn = pk_min(mn, Ln[j]);
            }
            const uint32_t m = row_min16(min(mn & 0xFFFFu, mn >> 16));
            const uint32_t mm = m | (m << 16);
            buf_store_pairs<VPL, ALIGNED, L8>(Ln, ro, io ? off0 + (uint32_t)i * stride : kOff, nvalid);
#pragma unroll
            for (int j = 0; j < NP; ++j) Lp[j] = act ? pk_sub(Ln[j], mm) : 0u;
        }
    }
}

// ---------------------------------------------------------------------------
// S = sum of per-path volumes

template <bool L8>
__global__ __launch_bounds__(256) void k_sum(const void *__restrict__ vols, long long vstride, int np,
                                             long long nvol, uint16_t *__restrict__ sum)
{
    const long long e0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * 8;
    if (e0 >= nvol) return;
    const bool vec = e0 + 8 <= nvol && ((reinterpret_cast<uintptr_t>(sum) & 15) == 0);
    if (vec) {
        uint32_t acc[4] = {0, 0, 0, 0};
        for (int r = 0; r < np; ++r) {
            if (L8) {
                const uint2 t = *reinterpret_cast<const uint2 *>(static_cast<const uint8_t *>(vols) +
                                                                 r * vstride + e0);
                acc[0] = pk_add(acc[0], __builtin_amdgcn_perm(t.x, t.x, 0x0C010C00u));
                acc[1] = pk_add(acc[1], __builtin_amdgcn_perm(t.x, t.x, 0x0C030C02u));
                acc[2] = pk_add(acc[2], __builtin_amdgcn_perm(t.y, t.y, 0x0C010C00u));
                acc[3] = pk_add(acc[3], __builtin_amdgcn_perm(t.y, t.y, 0x0C030C02u));
            } else {
                const uint4 t = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(vols) +
                                                                 r * vstride + e0);
                acc[0] = pk_add(acc[0], t.x);
                acc[1] = pk_add(acc[1], t.y);
                acc[2] = pk_add(acc[2], t.z);
                acc[3] = pk_add(acc[3], t.w);
            }
        }
        *reinterpret_cast<uint4 *>(sum + e0) = make_uint4(acc[0], acc[1], acc[2], acc[3]);
    } else {
        for (long long e = e0; e < nvol && e < e0 + 8; ++e) {
            uint32_t s = 0;
            for (int r = 0; r < np; ++r)
                s += L8 ? static_cast<const uint8_t *>(vols)[r * vstride + e]
                        : static_cast<const uint16_t *>(vols)[r * vstride + e];
            sum[e] = (uint16_t)s;
        }
    }
}

// ---------------------------------------------------------------------------
// winner-take-all, sub-pixel parabola, eq. (10) offset

template <int VPL>
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
    best = row_min16(best);
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
    sm = row_max16(sm);
    sp = row_max16(sp);
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

template <int VPL, bool ALIGNED>
__global__ __launch_bounds__(256) void k_wta_sum(const uint16_t *__restrict__ sum, const int32_t *__restrict__ d_lo,
                                                 int W, int H, int w, uint16_t *__restrict__ dint,
                                                 float *__restrict__ dsub)
{
    const int lane = threadIdx.x & 15;
    const long long pix = (long long)blockIdx.x * (blockDim.x >> 4) + (threadIdx.x >> 4);
    if (pix >= (long long)W * H) return;
    const int kbase = lane * VPL;
    const int nvalid = min(max(w - kbase, 0), VPL);
    uint32_t S[VPL / 2];
    if (nvalid > 0)
        load_u16_pairs<VPL, ALIGNED>(S, sum + pix * w + kbase, nvalid);
    else
#pragma unroll
        for (int j = 0; j < VPL / 2; ++j) S[j] = 0;
    const int v = (int)(pix / W);
    select_and_write<VPL>(S, kbase, w, lane, d_lo ? d_lo[v] : 0, pix, dint, dsub);
}

template <int VPL, bool ALIGNED, bool L8>
__global__ __launch_bounds__(256) void k_wta_paths(const void *__restrict__ vols, long long vstride, int np,
                                                   const int32_t *__restrict__ d_lo, int W, int H, int w,
                                                   uint16_t *__restrict__ dint, float *__restrict__ dsub)
{
    constexpr int NP = VPL / 2;
    const int lane = threadIdx.x & 15;
    const long long pix = (long long)blockIdx.x * (blockDim.x >> 4) + (threadIdx.x >> 4);
    if (pix >= (long long)W * H) return;
    const int kbase = lane * VPL;
    const int nvalid = min(max(w - kbase, 0), VPL);
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
                load_u16_pairs<VPL, ALIGNED>(t, static_cast<const uint16_t *>(vols) + r * vstride + pix * w + kbase,
                                             nvalid);
#pragma unroll
                for (int j = 0; j < NP; ++j) S[j] = pk_add(S[j], t[j]);
            }
        }
    }
    const int v = (int)(pix / W);
    select_and_write<VPL>(S, kbase, w, lane, d_lo ? d_lo[v] : 0, pix, dint, dsub);
}

// ---------------------------------------------------------------------------
// dispatch helpers

template <template <int> class F, typename... A>
hipError_t by_vpl(int vpl, A &&...args)
{
    switch (vpl) {
    case 2: return F<2>::run(args...);
    case 4: return F<4>::run(args...);
    case 8: return F<8>::run(args...);
    case 12: return F<12>::run(args...);
    case 16: return F<16>::run(args...);
    default: return hipErrorInvalidValue;
    }
}

constexpr int kPrefetch = 8;

template <int VPL>
struct AggLaunch {
    static hipError_t run(const KernelConfig &kc, bool l8, bool pad, const AggParams &p, dim3 grid, dim3 block,
                          hipStream_t s)
    {
        if (!kc.aligned) {
            if (l8) hipLaunchKernelGGL((k_aggregate<VPL, false, true, true, kPrefetch>), grid, block, 0, s, p);
            else hipLaunchKernelGGL((k_aggregate<VPL, false, true, false, kPrefetch>), grid, block, 0, s, p);
        } else if (pad) {
            if (l8) hipLaunchKernelGGL((k_aggregate<VPL, true, true, true, kPrefetch>), grid, block, 0, s, p);
            else hipLaunchKernelGGL((k_aggregate<VPL, true, true, false, kPrefetch>), grid, block, 0, s, p);
        } else {
            if (l8) hipLaunchKernelGGL((k_aggregate<VPL, true, false, true, kPrefetch>), grid, block, 0, s, p);
            else hipLaunchKernelGGL((k_aggregate<VPL, true, false, false, kPrefetch>), grid, block, 0, s, p);
        }
        return hipGetLastError();
    }
};

template <int VPL>
struct CostLaunch {
    static hipError_t run(const KernelConfig &kc, const Problem &pb, const uint64_t *cl, const uint64_t *cr,
                          const int32_t *d_lo, uint8_t *cost, hipStream_t s)
    {
        dim3 grid((pb.W + 15) / 16, pb.H), block(256);
        if (kc.aligned)
            hipLaunchKernelGGL((k_cost<VPL, true>), grid, block, 0, s, cl, cr, d_lo, pb.W, pb.H, pb.w, pb.cmax, cost);
        else
            hipLaunchKernelGGL((k_cost<VPL, false>), grid, block, 0, s, cl, cr, d_lo, pb.W, pb.H, pb.w, pb.cmax,
                               cost);
        return hipGetLastError();
    }
};

template <int VPL>
struct WtaSumLaunch {
    static hipError_t run(const KernelConfig &kc, const Problem &pb, const uint16_t *sum, const int32_t *d_lo,
                          uint16_t *dint, float *dsub, hipStream_t s)
    {
        const long long npix = (long long)pb.W * pb.H;
        dim3 grid((unsigned)((npix + 15) / 16)), block(256);
        if (kc.aligned)
            hipLaunchKernelGGL((k_wta_sum<VPL, true>), grid, block, 0, s, sum, d_lo, pb.W, pb.H, pb.w, dint, dsub);
        else
            hipLaunchKernelGGL((k_wta_sum<VPL, false>), grid, block, 0, s, sum, d_lo, pb.W, pb.H, pb.w, dint, dsub);
        return hipGetLastError();
    }
};

template <int VPL>
struct WtaPathsLaunch {
    static hipError_t run(const KernelConfig &kc, const Problem &pb, const void *vols, long long vstride, int np,
                          bool l8, const int32_t *d_lo, uint16_t *dint, float *dsub, hipStream_t s)
    {
        const long long npix = (long long)pb.W * pb.H;
        dim3 grid((unsigned)((npix + 15) / 16)), block(256);
        if (kc.aligned) {
            if (l8)
                hipLaunchKernelGGL((k_wta_paths<VPL, true, true>), grid, block, 0, s, vols, vstride, np, d_lo, pb.W,
                                   pb.H, pb.w, dint, dsub);
            else
                hipLaunchKernelGGL((k_wta_paths<VPL, true, false>), grid, block, 0, s, vols, vstride, np, d_lo, pb.W,
                                   pb.H, pb.w, dint, dsub);
        } else {
            if (l8)
                hipLaunchKernelGGL((k_wta_paths<VPL, false, true>), grid, block, 0, s, vols, vstride, np, d_lo, pb.W,
                                   pb.H, pb.w, dint, dsub);
            else
                hipLaunchKernelGGL((k_wta_paths<VPL, false, false>), grid, block, 0, s, vols, vstride, np, d_lo,
                                   pb.W, pb.H, pb.w, dint, dsub);
        }
        return hipGetLastError();
    }
};

long long volume_stride(const Problem &pb, bool l8)
{
    // each per-path volume starts on a 256-byte boundary
    const long long n = (long long)pb.W * pb.H * pb.w;
    const long long esz = l8 ? 1 : 2;
    return ((n * esz + 255) / 256 * 256) / esz;
}

}  // namespace

hipError_t launch_census(const Problem &pb, const uint8_t *img, int pitch, uint64_t *codes, hipStream_t s)
{
    dim3 grid((pb.W + 63) / 64, (pb.H + 3) / 4), block(256);
    switch (pb.n) {
    case 3: hipLaunchKernelGGL(k_census<3>, grid, block, 0, s, img, pitch, pb.W, pb.H, codes); break;
    case 5: hipLaunchKernelGGL(k_census<5>, grid, block, 0, s, img, pitch, pb.W, pb.H, codes); break;
    case 7: hipLaunchKernelGGL(k_census<7>, grid, block, 0, s, img, pitch, pb.W, pb.H, codes); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cost(const Problem &pb, const KernelConfig &kc, const uint64_t *cl, const uint64_t *cr,
                       const int32_t *d_lo, uint8_t *cost, hipStream_t s)
{
    return by_vpl<CostLaunch>(kc.vpl, kc, pb, cl, cr, d_lo, cost, s);
}

hipError_t launch_aggregate(const Problem &pb, const KernelConfig &kc, const uint8_t *cost, const int *paths, int np,
                            bool l8, void *out, hipStream_t s)
{
    AggParams p{};
    p.cost = cost;
    p.out = out;
    p.vstride = volume_stride(pb, l8);
    p.W = pb.W;
    p.H = pb.H;
    p.w = pb.w;
    p.p1x2 = (uint32_t)pb.p1 * 0x10001u;
    p.p2x2 = (uint32_t)pb.p2 * 0x10001u;
    p.np = np;
    p.lines_per_wg = kc.agg_block / 16;
    // Dispatch slots in order of scanline length (horizontal, diagonal,
    // vertical) so the longest dependency chains start first.  Slot o
    // aggregates direction paths[i] into output volume i: code = r | i << 8.
    int no = 0, acc = 0;
    for (int kind = 0; kind < 3; ++kind)
        for (int i = 0; i < np; ++i) {
            const int r = paths[i];
            const int k = (r <= 1) ? 0 : (r >= 4 ? 1 : 2);
            if (k != kind) continue;
            const int nl = (r <= 1) ? pb.H : (r <= 3 ? pb.W : pb.W + pb.H - 1);
            p.paths[no] = r | (i << 8);
            p.gstart[no] = acc;
            acc += (nl + p.lines_per_wg - 1) / p.lines_per_wg;
            ++no;
        }
    p.gstart[np] = acc;
    dim3 grid(acc), block(kc.agg_block);
    return by_vpl<AggLaunch>(kc.vpl, kc, l8, pb.w < 16 * kc.vpl, p, grid, block, s);
}

hipError_t launch_sum(const Problem &pb, const KernelConfig &kc, const void *vols, int np, bool l8, uint16_t *sum,
                      hipStream_t s)
{
    (void)kc;
    const long long nvol = (long long)pb.W * pb.H * pb.w;
    const long long threads = (nvol + 7) / 8;
    dim3 grid((unsigned)((threads + 255) / 256)), block(256);
    const long long vs = volume_stride(pb, l8);
    if (l8) hipLaunchKernelGGL(k_sum<true>, grid, block, 0, s, vols, vs, np, nvol, sum);
    else hipLaunchKernelGGL(k_sum<false>, grid, block, 0, s, vols, vs, np, nvol, sum);
    return hipGetLastError();
}

hipError_t launch_wta_sum(const Problem &pb, const KernelConfig &kc, const uint16_t *sum, const int32_t *d_lo,
                          uint16_t *dint, float *dsub, hipStream_t s)
{
    return by_vpl<WtaSumLaunch>(kc.vpl, kc, pb, sum, d_lo, dint, dsub, s);
}

hipError_t launch_wta_paths(const Problem &pb, const KernelConfig &kc, const void *vols, int np, bool l8,
                            const int32_t *d_lo, uint16_t *dint, float *dsub, hipStream_t s)
{
    return by_vpl<WtaPathsLaunch>(kc.vpl, kc, pb, vols, volume_stride(pb, l8), np, l8, d_lo, dint, dsub, s);
}

}  // namespace sgm
