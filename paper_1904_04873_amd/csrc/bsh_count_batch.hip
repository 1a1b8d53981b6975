// Stage-1 weighted number count, the batched plan's launch forms (hough_unit_kernel, one block
// per queued unit, and the persistent hough_batch_kernel; bsh_count_kernels.h).  The select
// variants are instantiated here, the table variant in bsh_count_table.hip.
#include "bsh_count_kernels.h"

namespace bsh {

int launch_batch(const ItemDesc* items, const WorkUnit* units, int64_t n_units, uint32_t* counter,
                 int blocks, int lanes, int chunk, int mode, int n_words, bool persistent, hipStream_t stream)
{
    const size_t lds = smem_bytes_of(mode, chunk, n_words);
    if (!persistent && n_units > 0x7fffffff) return fail_inval("more than 2^31 - 1 units in one pass");
    int rc = BSH_OK;
    if (is_table_mode(mode)) {
        rc = launch_batch_table(items, units, n_units, counter, blocks, lanes, chunk, mode, lds, persistent, stream);
    } else {
#define BSH_LAUNCH_BATCH(M, C) rc = launch_batch_mc<M, C>(items, units, n_units, counter, blocks, lanes, lds, persistent, stream)
        BSH_DISPATCH_SELECT(mode, chunk, BSH_LAUNCH_BATCH)
#undef BSH_LAUNCH_BATCH
    }
    if (rc) return rc;
    return check_launch("batched count");
}

static int occupancy_select(int lanes, int chunk, int mode, size_t lds, bool persistent)
{
    int n = 0;
#define BSH_OCC(M, C) n = occupancy_mc<M, C>(lanes, lds, persistent)
    BSH_DISPATCH_SELECT(mode, chunk, BSH_OCC)
#undef BSH_OCC
    return n;
}

int batch_blocks_per_cu(int lanes, int chunk, int mode, int n_words, bool persistent)
{
    const size_t lds = smem_bytes_of(mode, chunk, n_words);
    const int n = is_table_mode(mode) ? occupancy_table(lanes, chunk, mode, lds, persistent)
                                      : occupancy_select(lanes, chunk, mode, lds, persistent);
    return n < 1 ? 1 : n;
}

}  // namespace bsh
