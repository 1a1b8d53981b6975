// Stage-1 weighted number count, persistent launch form of the batched plan: blocks pull
// (item, pixel, period, tile) units from a queue until it is empty.  The tile body is in
// bsh_count_tile.h.
#include "bsh_count_tile.h"

namespace bsh {

template <int kMode, int kChunk>
__global__ __launch_bounds__(kMaxLanes, min_blocks<kMode>()) void hough_batch_kernel(const ItemDesc* __restrict__ items,
                                                               const WorkUnit* __restrict__ units,
                                                               int64_t n_units, uint32_t* counter)
{
    __shared__ __align__(16) unsigned char smem[smem_bytes<kMode, kChunk>()];
    __shared__ int64_t next;
    for (;;) {
        if (threadIdx.x == 0) next = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t u = next;
        __syncthreads();
        if (u >= n_units) break;
        const WorkUnit w = units[u];
        const ItemDesc d = items[w.item];
        run_tile<kMode, kChunk>(d, w.sky, w.ip, w.tile, smem);
    }
}

int launch_batch(const ItemDesc* items, const WorkUnit* units, int64_t n_units, uint32_t* counter,
                 int blocks, int lanes, int chunk, int mode, hipStream_t stream)
{
#define BSH_LAUNCH_BATCH(M, C)                                                                \
    hipLaunchKernelGGL((hough_batch_kernel<M, C>), dim3(blocks), dim3(lanes), 0, stream, items, units, \
                       n_units, counter)
    BSH_DISPATCH(mode, chunk, BSH_LAUNCH_BATCH)
#undef BSH_LAUNCH_BATCH
    return check_launch("batched count");
}

int batch_blocks_per_cu(int lanes, int chunk, int mode)
{
    int n = 0;
    hipError_t e = hipSuccess;
#define BSH_OCC(M, C) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, hough_batch_kernel<M, C>, lanes, 0)
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
