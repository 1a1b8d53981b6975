// Stage-1 weighted number count, plain launch form (bsh_hough_count): one block per tile of
// one work item.  The tile body is in bsh_count_tile.h.
#include <cstring>

#include "bsh_count_tile.h"

namespace bsh {

template <int kMode, int kChunk>
__global__ __launch_bounds__(kMaxLanes, kMode == 2 ? 2 : 1) void hough_count_kernel(const PlainLaunch p)
{
    __shared__ __align__(16) unsigned char smem[smem_bytes<kMode, kChunk>()];
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

// Tiles of each period group of one item, in tile_start form.
int64_t plan_tiles(const bsh_grid* g, int lanes, int32_t* tile_start, int64_t* group_sizes)
{
    int64_t tiles = 0;
    for (int32_t ip = 0; ip < g->n_per; ++ip) {
        int64_t group = 0;
        for (int32_t ia = 0; ia < g->n_ap; ++ia) {
            const int64_t c = (int64_t)ia * g->n_per + ip;
            group += g->tasc_off_host[c + 1] - g->tasc_off_host[c];
        }
        if (tile_start) tile_start[ip] = (int32_t)tiles;
        if (group_sizes) group_sizes[ip] = group;
        tiles += (group + lanes - 1) / lanes;
    }
    if (tile_start)
        for (int32_t ip = g->n_per; ip <= BSH_MAX_PER; ++ip) tile_start[ip] = (int32_t)tiles;
    return tiles;
}

void fill_desc(ItemDesc& d, const bsh_segments* seg, const bsh_grid* grid, int32_t sky_lo,
               int32_t n_sky, uint32_t* count_out, float* wsum_out, int32_t* status)
{
    std::memset(&d, 0, sizeof(d));
    d.t_mid = seg->t_mid;
    d.v = seg->v_over_c;
    d.w = seg->weight;
    d.bits = seg->peak_bits;
    d.sky = grid->sky;
    d.a_p = grid->a_p;
    d.period = grid->period;
    d.tasc_off = grid->tasc_off;
    d.t_asc = grid->t_asc;
    d.count_out = count_out;
    d.wsum_out = wsum_out;
    d.status = status;
    d.n_seg = seg->n_seg;
    d.k_lo = seg->k_lo;
    d.k0 = grid->k0;
    d.w_per_sky = seg->weight_per_sky;
    d.n_words = words_for(seg->n_bins);
    d.n_bins = seg->n_bins;
    d.n_f0 = grid->n_f0;
    d.n_ap = grid->n_ap;
    d.n_per = grid->n_per;
    d.sky_lo = sky_lo;
    d.n_sky = n_sky;
    d.n_bin = grid->tasc_off_host[(int64_t)grid->n_ap * grid->n_per];
}

__global__ void fill_zero_kernel(uint32_t* p, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

int zero_words(void* p, int64_t n_words, hipStream_t stream)
{
    if (n_words <= 0 || !p) return BSH_OK;
    int64_t blocks = (n_words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (uint32_t*)p, n_words);
    return check_launch("zero fill");
}

int launch_plain(const PlainLaunch& p, int64_t blocks, int lanes, int chunk, int mode, hipStream_t stream)
{
#define BSH_LAUNCH_PLAIN(M, C)                                                                \
    hipLaunchKernelGGL((hough_count_kernel<M, C>), dim3((unsigned)blocks), dim3(lanes), 0, stream, p)
    BSH_DISPATCH(mode, chunk, BSH_LAUNCH_PLAIN)
#undef BSH_LAUNCH_PLAIN
    return check_launch("bsh_hough_count");
}

int kernel_mode(int variant, bool with_count)
{
    if (with_count) return 1;
    return variant == BSH_VARIANT_SELECT ? 0 : 2;
}

bool valid_tile_shape(int lanes, int chunk)
{
    return (lanes == 64 || lanes == 128 || lanes == 256 || lanes == 512) && (chunk == 128 || chunk == 256 || chunk == 512);
}

}  // namespace bsh

using namespace bsh;

extern "C" int bsh_hough_count_ex(const bsh_segments* seg, const bsh_grid* grid, int32_t lanes,
                                  int32_t chunk, int32_t variant, uint32_t* count_out, float* wsum_out,
                                  int32_t* status, bsh_stream stream)
{
    clear_error();
    int rc = check_segments(seg, true, false);
    if (rc) return rc;
    rc = check_grid(grid);
    if (rc) return rc;
    if (!count_out && !wsum_out) return fail_inval("both outputs are NULL");
    if (!valid_tile_shape(lanes, chunk)) return fail_inval("tile shape: lanes 64/128/256/512, chunk 128/256/512");
    if (variant < BSH_VARIANT_AUTO || variant > BSH_VARIANT_TABLE) return fail_inval("variant");
    rc = check_window(seg, grid);
    if (rc) return rc;

    PlainLaunch p;
    std::memset(&p, 0, sizeof(p));
    fill_desc(p.d, seg, grid, 0, grid->n_sky, count_out, wsum_out, status);
    const int64_t tiles = plan_tiles(grid, lanes, p.tile_start, nullptr);
    p.tiles_per_sky = (int32_t)tiles;
    const int64_t blocks = tiles * grid->n_sky;
    if (tiles == 0 || p.d.n_bin == 0) return BSH_OK;
    if (blocks > 0x7fffffff) return fail_inval("grid too large for one launch");
    hipStream_t s = (hipStream_t)stream;
    if (seg->n_seg == 0) {
        // no segments: every count is zero
        const int64_t n_t = (int64_t)grid->n_sky * p.d.n_bin * grid->n_f0;
        rc = zero_words(wsum_out, wsum_out ? n_t : 0, s);
        if (rc) return rc;
        return zero_words(count_out, count_out ? n_t : 0, s);
    }
    return launch_plain(p, blocks, lanes, chunk, kernel_mode(variant, count_out != nullptr), s);
}

extern "C" int bsh_hough_count(const bsh_segments* seg, const bsh_grid* grid, uint32_t* count_out,
                               float* wsum_out, int32_t* status, bsh_stream stream)
{
    return bsh_hough_count_ex(seg, grid, kDefaultLanes, kDefaultChunk, BSH_VARIANT_AUTO, count_out, wsum_out,
                              status, stream);
}
