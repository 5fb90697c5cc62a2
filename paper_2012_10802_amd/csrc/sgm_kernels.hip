// HIP kernels of the SGM hot path for gfx950 (CDNA4, wave64).
//
// Data layout (all row-major, disparity fastest):
//   census codes   uint64 [H][W]
//   cost C         uint8  [H][W][w]       (Sec. II-B, c(p,d); census + Hamming)
//   per-path L_r   uint8 or uint16 [H][W][w], one volume per direction
//   summed S       uint16 [H][W][w]       (eq. (9))
//
// Lane mapping of the aggregation (eq. (8)): a scanline of the path is
// carried by a group of G lanes (a 16-lane DPP row, or for the vertical and
// diagonal directions of windows up to 64 a half row or a quad); lane j
// holds the VPL consecutive window indices [j*VPL, (j+1)*VPL) as VPL/2
// packed u16 pairs.  With G = 16 one wave64 advances four scanlines, one
// workgroup of 256 threads sixteen.  Per step a lane
//   * loads its VPL cost bytes (prefetched PF steps ahead into registers),
//   * forms the k-1 / k+1 neighbour pairs with v_alignbit inside the lane
//     and one row_shr / row_shl DPP move across lanes,
//   * reduces the predecessor's minimum m_q over the window with DPP
//     steps (four for a row; independent of, and overlapped with, the
//     neighbour terms),
//   * evaluates C + min(L(k), min(L(k-1), L(k+1)) + P1, m_q + P2) - m_q with
//     packed u16 min/add/sub.
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

#include "sgm_device.h"
#include "sgm_internal.h"

namespace sgm {
namespace {

using namespace dev;

template <int N>
__global__ __launch_bounds__(256) void k_census(const uint8_t *__restrict__ img, int pitch, int W, int H,
                                                uint64_t *__restrict__ out)
{
    census_tile<N>(img, pitch, W, H, out, blockIdx.x, blockIdx.y);
}

// both images of a pair in one launch (blockIdx.z: 0 left, 1 right)
template <int N>
__global__ __launch_bounds__(256) void k_census_lr(const uint8_t *__restrict__ left,
                                                   const uint8_t *__restrict__ right, int pitch, int W, int H,
                                                   uint64_t *__restrict__ out_l, uint64_t *__restrict__ out_r)
{
    const bool r = blockIdx.z != 0;
    census_tile<N>(r ? right : left, pitch, W, H, r ? out_r : out_l, blockIdx.x, blockIdx.y);
}

template <int CH>
__global__ __launch_bounds__(256) void k_cost(const uint64_t *__restrict__ cl, const uint64_t *__restrict__ cr,
                                              const int32_t *__restrict__ d_lo, int W, int H, int w, int cmax,
                                              uint8_t *__restrict__ cost)
{
    __shared__ CostLds lds;
    cost_tile<CH>(cl, cr, d_lo, W, H, w, cmax, cost, blockIdx.x, blockIdx.y, lds);
}

template <int G, int VPL, bool ALIGNED, bool PAD, bool L8, int PF, int GH, int VPLH, bool PADH, int PFH>
__global__ __launch_bounds__(256) void k_aggregate(AggParams a)
{
    int slot = 0;
    while (slot + 1 < a.np && (int)blockIdx.x >= a.gstart[slot + 1]) ++slot;
    // workgroup-uniform by construction; say so, so that the buffer
    // descriptors built from them stay in scalar registers
    slot = __builtin_amdgcn_readfirstlane(slot);
    const int r = __builtin_amdgcn_readfirstlane(a.paths[slot] & 0xFF);
    const int vol = __builtin_amdgcn_readfirstlane(a.paths[slot] >> 8);
    const int g = __builtin_amdgcn_readfirstlane((int)blockIdx.x - a.gstart[slot]);
    agg_item<G, VPL, ALIGNED, PAD, L8, PF, GH, VPLH, PADH, PFH>(a, r, vol, g);
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
    select_and_write<16, VPL>(S, kbase, w, lane, d_lo ? d_lo[v] : 0, pix, dint, dsub);
}

template <int G, int VPL, bool ALIGNED, bool L8>
__global__ __launch_bounds__(256) void k_wta_paths(const void *__restrict__ vols, long long vstride, int np,
                                                   const int32_t *__restrict__ d_lo, int W, int H, int w,
                                                   uint16_t *__restrict__ dint, float *__restrict__ dsub)
{
    wta_paths_group<G, VPL, ALIGNED, L8>(vols, vstride, np, d_lo, W, H, w, dint, dsub, blockIdx.x);
}

// ---------------------------------------------------------------------------
// dispatch helpers

// Lane mappings compiled for the volume kernels: G lanes carry one scanline
// (aggregation) or one pixel (selection), each holding VPL window values.
// G = 16 serves every window width (with any w % VPL); the narrower groups
// serve w <= 64 when w is a multiple of VPL.
template <template <int, int> class F, typename... A>
hipError_t by_mapping(int g, int vpl, A &&...args)
{
    switch (g * 256 + vpl) {
    case 16 * 256 + 2: return F<16, 2>::run(args...);
    case 16 * 256 + 4: return F<16, 4>::run(args...);
    case 16 * 256 + 8: return F<16, 8>::run(args...);
    case 16 * 256 + 12: return F<16, 12>::run(args...);
    case 16 * 256 + 16: return F<16, 16>::run(args...);
    case 8 * 256 + 4: return F<8, 4>::run(args...);
    case 8 * 256 + 8: return F<8, 8>::run(args...);
    case 4 * 256 + 4: return F<4, 4>::run(args...);
    case 4 * 256 + 8: return F<4, 8>::run(args...);
    case 4 * 256 + 12: return F<4, 12>::run(args...);
    case 4 * 256 + 16: return F<4, 16>::run(args...);
    default: return hipErrorInvalidValue;
    }
}

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

// Steps of cost prefetched ahead by each scanline.  Measured on 1280x720,
// w = 128 (four u16 pairs per lane): 24 steps stream the cost 11 % faster
// than 8 (20 and 32 do not), so that width takes 24; the others keep 8,
// where deeper rings only add registers.
constexpr int prefetch_steps(int g, int vpl) { return (g == 16 && vpl == 8) ? 24 : 8; }

// The horizontal directions always run on 16 lanes per scanline (see
// agg_item): a narrower mapping (w <= 64) pairs with the 16-lane one of the
// same widths, whose lanes hold 2 values up to w = 32 and 4 up to 64, padded
// whenever its 16 * VPLH slots exceed the narrow mapping's G * VPL.
template <int G, int VPL>
struct HorizontalMapping {
    static constexpr int VPLH = G == 16 ? VPL : (G * VPL <= 32 ? 2 : 4);
    static constexpr int PFH = prefetch_steps(16, VPLH);
    template <bool PAD>
    static constexpr bool padh() { return PAD || 16 * VPLH != G * VPL; }
};

template <int G, int VPL>
struct AggLaunch {
    static constexpr int PF = prefetch_steps(G, VPL);
    static constexpr int VPLH = HorizontalMapping<G, VPL>::VPLH;
    static constexpr int PFH = HorizontalMapping<G, VPL>::PFH;
    template <bool ALIGNED, bool PAD, bool L8>
    static void launch(const AggParams &p, dim3 grid, dim3 block, hipStream_t s)
    {
        constexpr bool PADH = HorizontalMapping<G, VPL>::template padh<PAD>();
        hipLaunchKernelGGL((k_aggregate<G, VPL, ALIGNED, PAD, L8, PF, 16, VPLH, PADH, PFH>), grid, block, 0, s, p);
    }
    static hipError_t run(const KernelConfig &kc, bool l8, bool pad, const AggParams &p, dim3 grid, dim3 block,
                          hipStream_t s)
    {
        if constexpr (G == 16) {
            if (!kc.aligned) {
                if (l8) launch<false, true, true>(p, grid, block, s);
                else launch<false, true, false>(p, grid, block, s);
                return hipGetLastError();
            }
        } else {
            if (!kc.aligned) return hipErrorInvalidValue;
        }
        if (pad) {
            if (l8) launch<true, true, true>(p, grid, block, s);
            else launch<true, true, false>(p, grid, block, s);
        } else {
            if (l8) launch<true, false, true>(p, grid, block, s);
            else launch<true, false, false>(p, grid, block, s);
        }
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

template <int G, int VPL>
struct WtaPathsLaunch {
    static hipError_t run(const KernelConfig &kc, const Problem &pb, const void *vols, long long vstride, int np,
                          bool l8, const int32_t *d_lo, uint16_t *dint, float *dsub, hipStream_t s)
    {
        const long long npix = (long long)pb.W * pb.H;
        constexpr int PPB = 256 / G;  // pixels per workgroup
        dim3 grid((unsigned)((npix + PPB - 1) / PPB)), block(256);
        if constexpr (G == 16) {
            if (!kc.aligned) {
                if (l8)
                    hipLaunchKernelGGL((k_wta_paths<G, VPL, false, true>), grid, block, 0, s, vols, vstride, np,
                                       d_lo, pb.W, pb.H, pb.w, dint, dsub);
                else
                    hipLaunchKernelGGL((k_wta_paths<G, VPL, false, false>), grid, block, 0, s, vols, vstride, np,
                                       d_lo, pb.W, pb.H, pb.w, dint, dsub);
                return hipGetLastError();
            }
        } else {
            if (!kc.aligned) return hipErrorInvalidValue;
        }
        if (l8)
            hipLaunchKernelGGL((k_wta_paths<G, VPL, true, true>), grid, block, 0, s, vols, vstride, np, d_lo, pb.W,
                               pb.H, pb.w, dint, dsub);
        else
            hipLaunchKernelGGL((k_wta_paths<G, VPL, true, false>), grid, block, 0, s, vols, vstride, np, d_lo, pb.W,
                               pb.H, pb.w, dint, dsub);
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
    dim3 grid((pb.W + kCensusTW - 1) / kCensusTW, (pb.H + kCensusTH - 1) / kCensusTH), block(256);
    switch (pb.n) {
    case 3: hipLaunchKernelGGL(k_census<3>, grid, block, 0, s, img, pitch, pb.W, pb.H, codes); break;
    case 5: hipLaunchKernelGGL(k_census<5>, grid, block, 0, s, img, pitch, pb.W, pb.H, codes); break;
    case 7: hipLaunchKernelGGL(k_census<7>, grid, block, 0, s, img, pitch, pb.W, pb.H, codes); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_census_lr(const Problem &pb, const uint8_t *left, const uint8_t *right, int pitch, uint64_t *cl,
                            uint64_t *cr, hipStream_t s)
{
    dim3 grid((pb.W + kCensusTW - 1) / kCensusTW, (pb.H + kCensusTH - 1) / kCensusTH, 2), block(256);
    switch (pb.n) {
    case 3: hipLaunchKernelGGL(k_census_lr<3>, grid, block, 0, s, left, right, pitch, pb.W, pb.H, cl, cr); break;
    case 5: hipLaunchKernelGGL(k_census_lr<5>, grid, block, 0, s, left, right, pitch, pb.W, pb.H, cl, cr); break;
    case 7: hipLaunchKernelGGL(k_census_lr<7>, grid, block, 0, s, left, right, pitch, pb.W, pb.H, cl, cr); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cost(const Problem &pb, const KernelConfig &kc, const uint64_t *cl, const uint64_t *cr,
                       const int32_t *d_lo, uint8_t *cost, hipStream_t s)
{
    (void)kc;
    dim3 grid((pb.W + kCostTile - 1) / kCostTile, pb.H), block(256);
    // 16-byte (8-byte) stores need w % 16 == 0 (w % 8 == 0) and a volume
    // aligned to them
    const uintptr_t a = reinterpret_cast<uintptr_t>(cost);
    if ((pb.w % 16) == 0 && (a % 16) == 0)
        hipLaunchKernelGGL(k_cost<16>, grid, block, 0, s, cl, cr, d_lo, pb.W, pb.H, pb.w, pb.cmax, cost);
    else if ((pb.w % 8) == 0 && (a % 8) == 0)
        hipLaunchKernelGGL(k_cost<8>, grid, block, 0, s, cl, cr, d_lo, pb.W, pb.H, pb.w, pb.cmax, cost);
    else
        hipLaunchKernelGGL(k_cost<4>, grid, block, 0, s, cl, cr, d_lo, pb.W, pb.H, pb.w, pb.cmax, cost);
    return hipGetLastError();
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
    // Dispatch slots: the horizontal directions first (the longest
    // dependency chains), then diagonal and vertical (agg_order 0) or
    // vertical and diagonal (1), the better one depending on the frame and
    // lane count (a tuned launch choice).  Slot o
    // aggregates direction paths[i] into output volume i: code = r | i << 8.
    // A workgroup carries agg_block / lanes scanlines, the horizontal ones
    // on 16 lanes each.
    int no = 0, acc = 0;
    for (int kind = 0; kind < 3; ++kind)
        for (int i = 0; i < np; ++i) {
            const int r = paths[i];
            const int k = (r <= 1) ? 0 : ((r >= 4) == (kc.agg_order == 0) ? 1 : 2);
            if (k != kind) continue;
            const int nl = (r <= 1) ? pb.H : (r <= 3 ? pb.W : pb.W + pb.H - 1);
            const int lpw = kc.agg_block / (k == 0 ? 16 : kc.lanes);
            p.paths[no] = r | (i << 8);
            p.gstart[no] = acc;
            acc += (nl + lpw - 1) / lpw;
            ++no;
        }
    p.gstart[np] = acc;
    dim3 grid(acc), block(kc.agg_block);
    return by_mapping<AggLaunch>(kc.lanes, kc.vpl, kc, l8, pb.w < kc.lanes * kc.vpl, p, grid, block, s);
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
    // the materialised sum is read by 16 lanes per pixel
    const Mapping m = choose_mapping(pb.w, 16);
    return by_vpl<WtaSumLaunch>(m.vpl, kc, pb, sum, d_lo, dint, dsub, s);
}

hipError_t launch_wta_paths(const Problem &pb, const KernelConfig &kc, const void *vols, int np, bool l8,
                            const int32_t *d_lo, uint16_t *dint, float *dsub, hipStream_t s)
{
    return by_mapping<WtaPathsLaunch>(kc.wta_lanes, kc.wta_vpl, kc, pb, vols, volume_stride(pb, l8), np, l8, d_lo,
                                      dint, dsub, s);
}

}  // namespace sgm
