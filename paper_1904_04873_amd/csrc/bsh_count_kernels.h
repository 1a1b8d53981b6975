// The stage-1 count kernels (plain launch, one block per queued unit, persistent blocks) and
// their launch helpers, as templates over (kernel mode, chunk).  Each mode is instantiated in
// one source only: the select variants in bsh_count.hip / bsh_count_batch.hip, the table variant
// in bsh_count_table.hip.  Internal to libbsh.
#pragma once

#include "bsh_count_tile.h"

namespace bsh {

// Plain launch form (bsh_hough_count): one block per tile of one work item.
template <int kMode, int kChunk>
__global__ __launch_bounds__(kMaxLanes, min_blocks<kMode>()) void hough_count_kernel(const PlainLaunch p)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int blk = blockIdx.x;
    const int s = blk / p.tiles_per_sky;
    const int t = blk - s * p.tiles_per_sky;
    int lo = 0, hi = p.d.n_per;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (p.tile_start[mid] <= t) lo = mid; else hi = mid;
    }
    run_tile<kMode, kChunk>(p.d, s, lo, t - p.tile_start[lo], smem);
}

// The batched plan's launch forms over a queue of (item, pixel, period, tile) units: one block
// per unit, dispatched in queue order (the default), or persistent blocks that pull units from
// an atomic queue counter until it is empty.  Both run the same tile body and give the same
// maps.  Measured on the table variant: the persistent loop keeps the tile's loop-invariant
// values live across units and takes more registers (two waves per SIMD where one unit per block
// fits three), and the hardware dispatcher hands blocks to CUs in queue order as earlier ones
// finish, which is the balance the queue counter gives.
template <int kMode, int kChunk>
__global__ __launch_bounds__(kMaxLanes, min_blocks<kMode>()) void hough_batch_kernel(const ItemDesc* __restrict__ items,
                                                               const WorkUnit* __restrict__ units,
                                                               int64_t n_units, uint32_t* counter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t next;
    for (;;) {
        if (threadIdx.x == 0) next = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        // the unit index is the block's: read as a wave-uniform value, so that the unit and its
        // item descriptor load into scalar registers
        const int64_t u = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)next);
        __syncthreads();
        if (u >= n_units) break;
        const WorkUnit w = units[u];
        const ItemDesc d = items[w.item];
        run_tile<kMode, kChunk>(d, w.sky, w.ip, w.tile, smem);
    }
}

template <int kMode, int kChunk>
__global__ __launch_bounds__(kMaxLanes, min_blocks<kMode>()) void hough_unit_kernel(const ItemDesc* __restrict__ items,
                                                              const WorkUnit* __restrict__ units)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const WorkUnit w = units[blockIdx.x];
    const ItemDesc d = items[w.item];
    run_tile<kMode, kChunk>(d, w.sky, w.ip, w.tile, smem);
}

template <int kMode, int kChunk>
int launch_plain_mc(const PlainLaunch& p, int64_t blocks, int lanes, size_t lds, hipStream_t stream)
{
    const int rc = allow_lds((const void*)hough_count_kernel<kMode, kChunk>, lds);
    if (rc) return rc;
    hipLaunchKernelGGL((hough_count_kernel<kMode, kChunk>), dim3((unsigned)blocks), dim3(lanes), lds, stream, p);
    return BSH_OK;
}

template <int kMode, int kChunk>
int launch_batch_mc(const ItemDesc* items, const WorkUnit* units, int64_t n_units, uint32_t* counter, int blocks,
                    int lanes, size_t lds, bool persistent, hipStream_t stream)
{
    if (persistent) {
        const int rc = allow_lds((const void*)hough_batch_kernel<kMode, kChunk>, lds);
        if (rc) return rc;
        hipLaunchKernelGGL((hough_batch_kernel<kMode, kChunk>), dim3(blocks), dim3(lanes), lds, stream, items, units,
                           n_units, counter);
    } else {
        const int rc = allow_lds((const void*)hough_unit_kernel<kMode, kChunk>, lds);
        if (rc) return rc;
        hipLaunchKernelGGL((hough_unit_kernel<kMode, kChunk>), dim3((unsigned)n_units), dim3(lanes), lds, stream,
                           items, units);
    }
    return BSH_OK;
}

// Resident blocks per CU of the persistent form, or of the one-block-per-unit form (0 when the
// occupancy query fails).
template <int kMode, int kChunk>
int occupancy_mc(int lanes, size_t lds, bool persistent)
{
    int n = 0;
    const void* k = persistent ? (const void*)hough_batch_kernel<kMode, kChunk> : (const void*)hough_unit_kernel<kMode, kChunk>;
    if (allow_lds(k, lds) != BSH_OK) return 0;
    const hipError_t e = persistent
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, hough_batch_kernel<kMode, kChunk>, lanes, lds)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, hough_unit_kernel<kMode, kChunk>, lanes, lds);
    return e == hipSuccess ? n : 0;
}

}  // namespace bsh
