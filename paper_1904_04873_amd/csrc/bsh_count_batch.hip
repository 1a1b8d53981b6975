// Stage-1 weighted number count, the batched plan's launch forms over a queue of (item, pixel,
// period, tile) units: one block per unit, dispatched in queue order (the default), or
// persistent blocks that pull units from an atomic queue counter until it is empty.  Both run
// the same tile body (bsh_count_tile.h) and give the same maps.  Measured on the table variant:
// the persistent loop keeps the tile's loop-invariant values live across units and takes 212
// registers (two waves per SIMD), one unit per block takes about 160 (three waves), and the
// hardware dispatcher hands blocks to CUs in queue order as earlier ones finish, which is the
// balance the queue counter gives.
#include "bsh_count_tile.h"

namespace bsh {

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

int launch_batch(const ItemDesc* items, const WorkUnit* units, int64_t n_units, uint32_t* counter,
                 int blocks, int lanes, int chunk, int mode, int n_words, bool persistent, hipStream_t stream)
{
    const size_t lds = smem_bytes_of(mode, chunk, n_words);
    int rc = BSH_OK;
    if (!persistent && n_units > 0x7fffffff) return fail_inval("more than 2^31 - 1 units in one pass");
#define BSH_LAUNCH_BATCH(M, C)                                                                \
    if (persistent) {                                                                         \
        rc = allow_lds((const void*)hough_batch_kernel<M, C>, lds);                            \
        if (rc) return rc;                                                                    \
        hipLaunchKernelGGL((hough_batch_kernel<M, C>), dim3(blocks), dim3(lanes), lds, stream, items, units, \
                           n_units, counter);                                                 \
    } else {                                                                                  \
        rc = allow_lds((const void*)hough_unit_kernel<M, C>, lds);                             \
        if (rc) return rc;                                                                    \
        hipLaunchKernelGGL((hough_unit_kernel<M, C>), dim3((unsigned)n_units), dim3(lanes), lds, stream, items, \
                           units);                                                            \
    }
    BSH_DISPATCH(mode, chunk, BSH_LAUNCH_BATCH)
#undef BSH_LAUNCH_BATCH
    return check_launch("batched count");
}

int batch_blocks_per_cu(int lanes, int chunk, int mode, int n_words)
{
    int n = 0;
    hipError_t e = hipSuccess;
    const size_t lds = smem_bytes_of(mode, chunk, n_words);
#define BSH_OCC(M, C)                                                                         \
    if (allow_lds((const void*)hough_batch_kernel<M, C>, lds) == BSH_OK)                       \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, hough_batch_kernel<M, C>, lanes, lds)
    switch (mode * 1000 + chunk) {
    case 128: BSH_OCC(0, 128); break;
    case 256: BSH_OCC(0, 256); break;
    case 512: BSH_OCC(0, 512); break;
    case 1128: BSH_OCC(1, 128); break;
    case 1256: BSH_OCC(1, 256); break;
    case 1512: BSH_OCC(1, 512); break;
    case 2128: BSH_OCC(2, 128); break;
    case 2256: BSH_OCC(2, 256); break;
    case 2512: BSH_OCC(2, 512); break;
    case 3128: BSH_OCC(3, 128); break;
    case 3256: BSH_OCC(3, 256); break;
    case 3512: BSH_OCC(3, 512); break;
    case 4128: BSH_OCC(4, 128); break;
    case 4256: BSH_OCC(4, 256); break;
    case 4512: BSH_OCC(4, 512); break;
    case 5128: BSH_OCC(5, 128); break;
    case 5256: BSH_OCC(5, 256); break;
    case 5512: BSH_OCC(5, 512); break;
    default: break;
    }
#undef BSH_OCC
    if (e != hipSuccess || n < 1) n = 1;
    return n;
}

}  // namespace bsh
