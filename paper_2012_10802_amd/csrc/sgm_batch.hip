// Batched kernels: every pair of a batch in one grid per stage, and one
// persistent aggregation launch for all pairs and directions.
//
// Stage grids are the concatenation of the single-pair grids; a workgroup
// finds its pair by binary search over the per-pair start indices.  The
// aggregation is persistent: each workgroup is one wave that repeatedly
// takes the next item (pair, direction, group of 64 / lanes scanlines, 4 for
// the horizontal directions, which always run on 16 lanes) from a
// queue in the workspace with one atomic add, runs it, and stops when the
// queue is empty (every wave reaches that exit).  The queue order is laid
// out on the host (longest scanlines first by default), which balances
// pairs of very different sizes without any inter-wave waiting.

#include "sgm_device.h"
#include "sgm_internal.h"

namespace sgm {
namespace {

using namespace dev;

__device__ __forceinline__ int find_pair(const BatchDev &b, int block, int PairDev::*start)
{
    int lo = 0, hi = b.npairs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.pairs[mid].*start <= block) lo = mid;
        else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

__global__ void k_batch_reset(uint32_t *counter) { *counter = 0u; }

template <int N>
__global__ __launch_bounds__(256) void k_census_batch(BatchDev b)
{
    const int blk = blockIdx.x;
    const int pi = find_pair(b, blk, &PairDev::census_start);
    const PairDev &P = b.pairs[pi];
    const int local = blk - P.census_start;
    const int per = P.census_tx * P.census_ty;
    const int img = local / per, t = local - img * per;
    uint64_t *out = reinterpret_cast<uint64_t *>(b.ws + (img ? P.off_codes_r : P.off_codes_l));
    census_tile<N>(img ? P.right : P.left, P.pitch, P.W, P.H, out, t % P.census_tx, t / P.census_tx);
}

__global__ __launch_bounds__(256) void k_cost_batch(BatchDev b)
{
    const int blk = blockIdx.x;
    const int pi = find_pair(b, blk, &PairDev::cost_start);
    const PairDev &P = b.pairs[pi];
    const int local = blk - P.cost_start;
    const uint64_t *cl = reinterpret_cast<const uint64_t *>(b.ws + P.off_codes_l);
    const uint64_t *cr = reinterpret_cast<const uint64_t *>(b.ws + P.off_codes_r);
    uint8_t *cost = b.ws + P.off_cost;
    const int bx = local % P.cost_tx, v = local / P.cost_tx;
    __shared__ CostLds lds;  // one for every piece width
    if (P.w % 16 == 0)
        cost_tile<16>(cl, cr, P.d_lo, P.W, P.H, P.w, b.cmax, cost, bx, v, lds);
    else if (P.w % 8 == 0)
        cost_tile<8>(cl, cr, P.d_lo, P.W, P.H, P.w, b.cmax, cost, bx, v, lds);
    else
        cost_tile<4>(cl, cr, P.d_lo, P.W, P.H, P.w, b.cmax, cost, bx, v, lds);
}

constexpr int kBatchPrefetch = 8;

template <bool L8>
__global__ __launch_bounds__(64) void k_aggregate_batch(BatchDev b)
{
    for (;;) {
        uint32_t item = 0;
        if (threadIdx.x == 0) item = atomicAdd(b.counter, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if ((int)item >= b.nitems) break;
        const uint32_t w0 = __builtin_amdgcn_readfirstlane(b.items[2 * item]);
        const int g = __builtin_amdgcn_readfirstlane((int)b.items[2 * item + 1]);
        const int pi = (int)(w0 >> 8), r = (int)(w0 & 0xFFu);
        const PairDev &P = b.pairs[pi];
        AggParams a;
        a.cost = b.ws + P.off_cost;
        a.out = b.ws + P.off_vols;
        a.vstride = P.vstride;
        a.W = P.W;
        a.H = P.H;
        a.w = P.w;
        a.p1x2 = b.p1x2;
        a.p2x2 = b.p2x2;
        a.np = b.npaths;
        // (lanes, values per lane, padded window) of the pair's mapping; the
        // horizontal directions take the pair's 16-lane one
        const bool horiz = r <= 1;
        const int variant = __builtin_amdgcn_readfirstlane(horiz ? 16 * 512 + P.h_vpl * 2 + P.h_pad
                                                                 : P.lanes * 512 + P.vpl * 2 + P.pad);
        switch (variant) {
        case 16 * 512 + 4: agg_item<16, 2, true, false, L8, kBatchPrefetch>(a, r, r, g); break;
        case 16 * 512 + 5: agg_item<16, 2, true, true, L8, kBatchPrefetch>(a, r, r, g); break;
        case 16 * 512 + 8: agg_item<16, 4, true, false, L8, kBatchPrefetch>(a, r, r, g); break;
        case 16 * 512 + 9: agg_item<16, 4, true, true, L8, kBatchPrefetch>(a, r, r, g); break;
        case 16 * 512 + 16: agg_item<16, 8, true, false, L8, kBatchPrefetch>(a, r, r, g); break;
        case 16 * 512 + 17: agg_item<16, 8, true, true, L8, kBatchPrefetch>(a, r, r, g); break;
        case 16 * 512 + 24: agg_item<16, 12, true, false, L8, kBatchPrefetch>(a, r, r, g); break;
        case 16 * 512 + 25: agg_item<16, 12, true, true, L8, kBatchPrefetch>(a, r, r, g); break;
        case 16 * 512 + 32: agg_item<16, 16, true, false, L8, kBatchPrefetch>(a, r, r, g); break;
        case 16 * 512 + 33: agg_item<16, 16, true, true, L8, kBatchPrefetch>(a, r, r, g); break;
        case 8 * 512 + 8: agg_item<8, 4, true, false, L8, kBatchPrefetch>(a, r, r, g); break;
        case 8 * 512 + 9: agg_item<8, 4, true, true, L8, kBatchPrefetch>(a, r, r, g); break;
        case 8 * 512 + 16: agg_item<8, 8, true, false, L8, kBatchPrefetch>(a, r, r, g); break;
        case 8 * 512 + 17: agg_item<8, 8, true, true, L8, kBatchPrefetch>(a, r, r, g); break;
        case 4 * 512 + 8: agg_item<4, 4, true, false, L8, kBatchPrefetch>(a, r, r, g); break;
        case 4 * 512 + 9: agg_item<4, 4, true, true, L8, kBatchPrefetch>(a, r, r, g); break;
        case 4 * 512 + 16: agg_item<4, 8, true, false, L8, kBatchPrefetch>(a, r, r, g); break;
        case 4 * 512 + 17: agg_item<4, 8, true, true, L8, kBatchPrefetch>(a, r, r, g); break;
        case 4 * 512 + 24: agg_item<4, 12, true, false, L8, kBatchPrefetch>(a, r, r, g); break;
        case 4 * 512 + 25: agg_item<4, 12, true, true, L8, kBatchPrefetch>(a, r, r, g); break;
        case 4 * 512 + 32: agg_item<4, 16, true, false, L8, kBatchPrefetch>(a, r, r, g); break;
        default: agg_item<4, 16, true, true, L8, kBatchPrefetch>(a, r, r, g); break;
        }
    }
}

template <bool L8>
__global__ __launch_bounds__(256) void k_wta_batch(BatchDev b)
{
    const int blk = blockIdx.x;
    const int pi = find_pair(b, blk, &PairDev::wta_start);
    const PairDev &P = b.pairs[pi];
    const long long local = blk - P.wta_start;
    const void *vols = b.ws + P.off_vols;
    switch (__builtin_amdgcn_readfirstlane(P.wta_lanes * 256 + P.wta_vpl)) {
    case 16 * 256 + 2: wta_paths_group<16, 2, true, L8>(vols, P.vstride, b.npaths, P.d_lo, P.W, P.H, P.w, P.dint, P.dsub, local); break;
    case 16 * 256 + 4: wta_paths_group<16, 4, true, L8>(vols, P.vstride, b.npaths, P.d_lo, P.W, P.H, P.w, P.dint, P.dsub, local); break;
    case 16 * 256 + 8: wta_paths_group<16, 8, true, L8>(vols, P.vstride, b.npaths, P.d_lo, P.W, P.H, P.w, P.dint, P.dsub, local); break;
    case 16 * 256 + 12: wta_paths_group<16, 12, true, L8>(vols, P.vstride, b.npaths, P.d_lo, P.W, P.H, P.w, P.dint, P.dsub, local); break;
    case 8 * 256 + 4: wta_paths_group<8, 4, true, L8>(vols, P.vstride, b.npaths, P.d_lo, P.W, P.H, P.w, P.dint, P.dsub, local); break;
    case 8 * 256 + 8: wta_paths_group<8, 8, true, L8>(vols, P.vstride, b.npaths, P.d_lo, P.W, P.H, P.w, P.dint, P.dsub, local); break;
    case 4 * 256 + 4: wta_paths_group<4, 4, true, L8>(vols, P.vstride, b.npaths, P.d_lo, P.W, P.H, P.w, P.dint, P.dsub, local); break;
    case 4 * 256 + 8: wta_paths_group<4, 8, true, L8>(vols, P.vstride, b.npaths, P.d_lo, P.W, P.H, P.w, P.dint, P.dsub, local); break;
    case 4 * 256 + 12: wta_paths_group<4, 12, true, L8>(vols, P.vstride, b.npaths, P.d_lo, P.W, P.H, P.w, P.dint, P.dsub, local); break;
    case 4 * 256 + 16: wta_paths_group<4, 16, true, L8>(vols, P.vstride, b.npaths, P.d_lo, P.W, P.H, P.w, P.dint, P.dsub, local); break;
    default: wta_paths_group<16, 16, true, L8>(vols, P.vstride, b.npaths, P.d_lo, P.W, P.H, P.w, P.dint, P.dsub, local); break;
    }
}

}  // namespace

hipError_t launch_batch(const BatchDev &b, const BatchGrids &g, int census_n, bool l8, int agg_waves, hipStream_t s,
                        const hipEvent_t *ev)
{
    if (census_n != 3 && census_n != 5 && census_n != 7) return hipErrorInvalidValue;
    auto mark = [&](int i) {
        if (ev && ev[i]) hipEventRecord(ev[i], s);
    };
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, b.counter);
    mark(0);
    switch (census_n) {
    case 3: hipLaunchKernelGGL(k_census_batch<3>, dim3(g.census), dim3(256), 0, s, b); break;
    case 5: hipLaunchKernelGGL(k_census_batch<5>, dim3(g.census), dim3(256), 0, s, b); break;
    default: hipLaunchKernelGGL(k_census_batch<7>, dim3(g.census), dim3(256), 0, s, b); break;
    }
    mark(1);
    hipLaunchKernelGGL(k_cost_batch, dim3(g.cost), dim3(256), 0, s, b);
    mark(2);
    if (l8) hipLaunchKernelGGL(k_aggregate_batch<true>, dim3(agg_waves), dim3(64), 0, s, b);
    else hipLaunchKernelGGL(k_aggregate_batch<false>, dim3(agg_waves), dim3(64), 0, s, b);
    mark(3);
    if (l8) hipLaunchKernelGGL(k_wta_batch<true>, dim3(g.wta), dim3(256), 0, s, b);
    else hipLaunchKernelGGL(k_wta_batch<false>, dim3(g.wta), dim3(256), 0, s, b);
    mark(4);
    return hipGetLastError();
}

}  // namespace sgm
