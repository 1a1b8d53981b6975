// Stage-1 weighted number count, plain launch form (bsh_hough_count): one block per tile of
// one work item.  The tile body is in bsh_count_tile.h, the kernels in bsh_count_kernels.h; the
// select variants are instantiated here, the table variant in bsh_count_table.hip.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "bsh_count_kernels.h"

namespace bsh {

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
    d.ec = grid->ecc_c;
    d.es = grid->ecc_s;
    d.n_bin = grid->tasc_off_host[(int64_t)grid->n_ap * grid->n_per];
}

__global__ void fill_zero_kernel(uint32_t* p, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

// In place: the exact integer-valued floats of a unit-weight count become uint32 counts.
__global__ void floats_to_counts_kernel(uint32_t* p, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = (uint32_t)__uint_as_float(p[e]);
}

int floats_to_counts(uint32_t* p, int64_t n, hipStream_t stream)
{
    if (n <= 0) return BSH_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(floats_to_counts_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
    return check_launch("count conversion");
}

int zero_words(void* p, int64_t n_words, hipStream_t stream)
{
    if (n_words <= 0 || !p) return BSH_OK;
    int64_t blocks = (n_words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (uint32_t*)p, n_words);
    return check_launch("zero fill");
}

int launch_plain(const PlainLaunch& p, int64_t blocks, int lanes, int chunk, int mode, int n_words,
                 hipStream_t stream)
{
    const size_t lds = smem_bytes_of(mode, chunk, n_words);
    int rc = BSH_OK;
    if (is_table_mode(mode)) {
        rc = launch_plain_table(p, blocks, lanes, chunk, mode, lds, stream);
    } else {
#define BSH_LAUNCH_PLAIN(M, C) rc = launch_plain_mc<M, C>(p, blocks, lanes, lds, stream)
        BSH_DISPATCH_SELECT(mode, chunk, BSH_LAUNCH_PLAIN)
#undef BSH_LAUNCH_PLAIN
    }
    if (rc) return rc;
    return check_launch("bsh_hough_count");
}

// Dynamic LDS above the default per-block limit has to be allowed per kernel; each kernel is
// raised once to the largest size asked for so far (so a launch under stream capture, after the
// plan has sized its blocks, makes no runtime call).
int allow_lds(const void* kernel, size_t bytes)
{
    if (bytes <= 64 * 1024) return BSH_OK;
    static std::mutex mu;
    static std::unordered_map<const void*, size_t> allowed;
    std::lock_guard<std::mutex> lock(mu);
    size_t& have = allowed[kernel];
    if (bytes <= have) return BSH_OK;
    const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) {
        set_error("allowing %zu bytes of LDS: %s", bytes, hipGetErrorString(e));
        return BSH_EHIP;
    }
    have = bytes;
    return BSH_OK;
}

int kernel_mode(int variant, bool with_count)
{
    if (with_count) return 1;
    return variant == BSH_VARIANT_SELECT ? 0 : 2;
}

int ecc_mode(const bsh_grid* g) { return (g->ecc_c != 0.0 || g->ecc_s != 0.0) ? kEccMode : 0; }

bool prove_item(int mode, ItemDesc& d, const bsh_segments* seg, const bsh_grid* grid)
{
    double v, apw;
    if (!mode_table(mode) || !proven_window(seg, grid, &v, &apw)) return false;
    d.v_claim = v;
    d.apw_claim = apw;
    return true;
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
    // Counts from the table variant: the weighted count with every weight one, whose sums of small
    // integers are exact in FP32 (below 2^24), written as floats into count_out and converted there
    // (a second launch when the weighted sums are asked for too); the select variant, whose
    // partial sums and counts take more registers than a wave has, counts on request.
    const bool table_counts = count_out && variant != BSH_VARIANT_SELECT && seg->n_seg < ((int64_t)1 << 24);
    fill_desc(p.d, seg, grid, 0, grid->n_sky, table_counts ? nullptr : count_out, wsum_out, status);
    int mode = (table_counts ? kernel_mode(BSH_VARIANT_TABLE, false) : kernel_mode(variant, count_out != nullptr)) +
               ecc_mode(grid);
    if (prove_item(mode, p.d, seg, grid)) mode += kProvenMode;
    const int64_t tiles = plan_tiles(grid, tile_templates(mode, lanes), p.tile_start, nullptr);
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
    if (!table_counts) return launch_plain(p, blocks, lanes, chunk, mode, p.d.n_words, s);
    if (wsum_out) {
        rc = launch_plain(p, blocks, lanes, chunk, mode, p.d.n_words, s);
        if (rc) return rc;
    }
    PlainLaunch pc = p;
    pc.d.w = nullptr;
    pc.d.w_per_sky = 0;
    pc.d.wsum_out = reinterpret_cast<float*>(count_out);
    rc = launch_plain(pc, blocks, lanes, chunk, mode, pc.d.n_words, s);
    if (rc) return rc;
    return floats_to_counts(count_out, (int64_t)grid->n_sky * p.d.n_bin * grid->n_f0, s);
}

extern "C" int32_t bsh_count_window_proven(const bsh_segments* seg, const bsh_grid* grid)
{
    clear_error();
    int rc = check_segments(seg, false, false);
    if (rc) return rc;
    rc = check_grid(grid);
    if (rc) return rc;
    double v, apw;
    return proven_window(seg, grid, &v, &apw) ? 1 : 0;
}

extern "C" int bsh_hough_count(const bsh_segments* seg, const bsh_grid* grid, uint32_t* count_out,
                               float* wsum_out, int32_t* status, bsh_stream stream)
{
    return bsh_hough_count_ex(seg, grid, kDefaultLanes, kDefaultChunk, BSH_VARIANT_AUTO, count_out, wsum_out,
                              status, stream);
}

// ---------------------------------------------------------------- stage 1 with a bounded top-k

namespace {

struct CountTopkLayout {
    size_t map, merge_score, merge_index, tmp_score, tmp_index, topk, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

CountTopkLayout count_topk_layout(int64_t pass_templates, int32_t k)
{
    CountTopkLayout l;
    size_t at = 0;
    l.map = at;
    at += align256(sizeof(float) * (size_t)pass_templates);
    l.merge_score = at;
    at += align256(sizeof(float) * 2 * (size_t)k);
    l.merge_index = at;
    at += align256(sizeof(int64_t) * 2 * (size_t)k);
    l.tmp_score = at;
    at += align256(sizeof(float) * (size_t)k);
    l.tmp_index = at;
    at += align256(sizeof(int64_t) * (size_t)k);
    l.topk = at;
    at += align256(topk_workspace_bytes(1, k));
    l.total = at;
    return l;
}

__global__ void copy_list_kernel(const float* __restrict__ src_s, const int64_t* __restrict__ src_i,
                                 float* __restrict__ dst_s, int64_t* __restrict__ dst_i, int32_t k)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < k) {
        dst_s[e] = src_s[e];
        dst_i[e] = src_i[e];
    }
}

int copy_list(const float* ss, const int64_t* si, float* ds, int64_t* di, int32_t k, hipStream_t s)
{
    hipLaunchKernelGGL(copy_list_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, ss, si, ds, di, k);
    return check_launch("list copy");
}

int64_t pass_sky(const bsh_grid* grid, int32_t sky_per_pass)
{
    return sky_per_pass > 0 ? std::min<int64_t>(sky_per_pass, grid->n_sky) : grid->n_sky;
}

}  // namespace

extern "C" size_t bsh_hough_count_topk_workspace(const bsh_grid* grid, const bsh_topk_spec* spec)
{
    if (!grid || !spec || spec->k < 1 || grid->n_sky < 1 || !grid->tasc_off_host) return 0;
    const int64_t per_sky = grid->tasc_off_host[(int64_t)grid->n_ap * grid->n_per] * grid->n_f0;
    return count_topk_layout(pass_sky(grid, spec->sky_per_pass) * per_sky, spec->k).total;
}

extern "C" int bsh_hough_count_topk(const bsh_segments* seg, const bsh_grid* grid, const bsh_topk_spec* spec,
                                    float* out_score, int64_t* out_index, void* ws, size_t ws_bytes,
                                    int32_t* status, bsh_stream stream)
{
    clear_error();
    int rc = check_segments(seg, true, false);
    if (rc) return rc;
    rc = check_grid(grid);
    if (rc) return rc;
    if (!spec) return fail_inval("topk spec is NULL");
    if (spec->k < 1) return fail_inval("k < 1");
    if (spec->sky_per_pass < 0) return fail_inval("sky_per_pass < 0");
    if (!out_score || !out_index) return fail_inval("NULL output");
    if (!ws) return fail_inval("workspace is NULL");
    rc = check_window(seg, grid);
    if (rc) return rc;
    const int32_t k = spec->k;
    const int64_t n_bin = grid->tasc_off_host[(int64_t)grid->n_ap * grid->n_per];
    const int64_t per_sky = n_bin * grid->n_f0;
    const int64_t np = pass_sky(grid, spec->sky_per_pass);
    if (np * per_sky >= (int64_t)0xffffffff) return fail_inval("a pass holds 2^32 - 1 templates or more");
    const CountTopkLayout L = count_topk_layout(np * per_sky, k);
    if (ws_bytes < L.total) {
        set_error("workspace %zu < %zu bytes", ws_bytes, L.total);
        return BSH_ENOMEM;
    }
    if (np < grid->n_sky && np * per_sky < k) return fail_inval("a pass must hold at least k templates");
    char* base = (char*)ws;
    float* map = (float*)(base + L.map);
    float* m_s = (float*)(base + L.merge_score);
    int64_t* m_i = (int64_t*)(base + L.merge_index);
    float* t_s = (float*)(base + L.tmp_score);
    int64_t* t_i = (int64_t*)(base + L.tmp_index);
    void* tws = base + L.topk;
    const size_t tws_bytes = L.total - L.topk;
    hipStream_t s = (hipStream_t)stream;
    const bool single = np >= grid->n_sky;

    const int32_t lanes = kDefaultLanes, chunk = kDefaultChunk;
    const int mode = kernel_mode(BSH_VARIANT_AUTO, false) + ecc_mode(grid);
    PlainLaunch p;
    for (int64_t c0 = 0; c0 < grid->n_sky; c0 += np) {
        const int32_t nc = (int32_t)std::min<int64_t>(np, grid->n_sky - c0);
        const int64_t n_t = nc * per_sky;
        std::memset(&p, 0, sizeof(p));
        fill_desc(p.d, seg, grid, (int32_t)c0, nc, nullptr, map, status);
        if (seg->weight_per_sky) p.d.w = seg->weight + c0 * seg->n_seg;
        const int pmode = prove_item(mode, p.d, seg, grid) ? mode + kProvenMode : mode;
        const int64_t tiles = plan_tiles(grid, tile_templates(mode, lanes), p.tile_start, nullptr);
        p.tiles_per_sky = (int32_t)tiles;
        if (seg->n_seg == 0 || tiles == 0)
            rc = zero_words(map, n_t, s);
        else
            rc = launch_plain(p, tiles * nc, lanes, chunk, pmode, p.d.n_words, s);
        if (rc) return rc;
        const int64_t first = c0 * per_sky;
        if (single)
            return topk_segmented(map, nullptr, nullptr, 1, n_t, 0, k, out_score, out_index, tws, tws_bytes, s, first);
        // this pass's list goes after the running list; the two are merged into the running list
        const bool opening = c0 == 0;
        rc = topk_segmented(map, nullptr, nullptr, 1, n_t, 0, k, opening ? m_s : m_s + k, opening ? m_i : m_i + k,
                            tws, tws_bytes, s, first);
        if (rc) return rc;
        if (!opening) {
            rc = topk_segmented(m_s, m_i, nullptr, 1, 2 * (int64_t)k, 0, k, t_s, t_i, tws, tws_bytes, s);
            if (!rc) rc = copy_list(t_s, t_i, m_s, m_i, k, s);
            if (rc) return rc;
        }
    }
    return copy_list(m_s, m_i, out_score, out_index, k, s);
}
