// The table variant of the stage-1 count (subset-sum tables, lane pairs; count_tile_pair in
// bsh_count_tile.h) in all three launch forms.  It is compiled on its own, with the instruction
// scheduler that favours independent instructions: the group loop's 46 table reads then issue in
// longer runs ahead of their adds, at the same three waves per SIMD (measured 3.8 % faster on the
// 200 Hz band, 5.2 % on the batched launch); the select variants, compiled elsewhere, would spill
// under it.
#include "bsh_count_kernels.h"

namespace bsh {

int launch_plain_table(const PlainLaunch& p, int64_t blocks, int lanes, int chunk, int mode, size_t lds,
                       hipStream_t stream)
{
    int rc = BSH_OK;
#define BSH_LAUNCH_PLAIN(M, C) rc = launch_plain_mc<M, C>(p, blocks, lanes, lds, stream)
    BSH_DISPATCH_TABLE(mode, chunk, BSH_LAUNCH_PLAIN)
#undef BSH_LAUNCH_PLAIN
    return rc;
}

int launch_batch_table(const ItemDesc* items, const WorkUnit* units, int64_t n_units, uint32_t* counter, int blocks,
                       int lanes, int chunk, int mode, size_t lds, bool persistent, hipStream_t stream)
{
    int rc = BSH_OK;
#define BSH_LAUNCH_BATCH(M, C) rc = launch_batch_mc<M, C>(items, units, n_units, counter, blocks, lanes, lds, persistent, stream)
    BSH_DISPATCH_TABLE(mode, chunk, BSH_LAUNCH_BATCH)
#undef BSH_LAUNCH_BATCH
    return rc;
}

int occupancy_table(int lanes, int chunk, int mode, size_t lds, bool persistent)
{
    int n = 0;
#define BSH_OCC(M, C) n = occupancy_mc<M, C>(lanes, lds, persistent)
    BSH_DISPATCH_TABLE(mode, chunk, BSH_OCC)
#undef BSH_OCC
    return n;
}

}  // namespace bsh
