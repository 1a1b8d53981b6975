// Batched stage 1 over many work items (sky patches x bands) with uneven sizes: one
// persistent launch whose blocks pull (item, pixel, period, tile) units from a queue ordered
// longest-first, then per-item and per-band top-lists, all captured in one HIP graph.
//
// The paper splits a search into independent band x sky-patch x binary-block jobs (eq:cost)
// and notes that the GPU idles while the host prepares the next job; here the whole set of
// jobs is one device-side queue, so the tail of one item overlaps the start of the next.
#include <algorithm>
#include <cstring>
#include <vector>

#include "bsh_count.h"

struct bsh_plan {
    int32_t n_items = 0, n_bands = 0, k_item = 0, k_band = 0;
    int32_t lanes = bsh::kDefaultLanes, chunk = bsh::kDefaultChunk, blocks = 0;
    bool use_graph = false;
    int32_t mode = 2;
    int64_t n_units = 0, max_item_len = 0, max_band_len = 0;
    std::vector<bsh::ItemDesc> items;            // host copies (plain mode)
    std::vector<bsh::PlainLaunch> plain;          // per-item plain launch parameters
    std::vector<int64_t> plain_blocks;
    std::vector<int64_t> item_off, band_off;      // host offsets
    bsh::ItemDesc* d_items = nullptr;
    bsh::WorkUnit* d_units = nullptr;
    uint32_t* d_counter = nullptr;
    int64_t* d_item_off = nullptr;
    int64_t* d_band_off = nullptr;
    float* d_item_score = nullptr;
    int64_t* d_item_index = nullptr;
    void* d_ws_item = nullptr;
    void* d_ws_band = nullptr;
    size_t ws_item = 0, ws_band = 0;
    float* maps = nullptr;
    float* band_score = nullptr;
    int64_t* band_index = nullptr;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

using namespace bsh;

constexpr int kItemShift = 40;    // global index = (item << 40) | index inside the item's map

int check_items(const bsh_item* items, int32_t n_items, const bsh_grid* grids, int32_t n_grids,
                int32_t n_bands)
{
    if (!items || n_items < 1) return fail_inval("no items");
    if (!grids || n_grids < 1) return fail_inval("no grids");
    if (n_bands < 1) return fail_inval("n_bands < 1");
    for (int32_t g = 0; g < n_grids; ++g) {
        int rc = check_grid(&grids[g]);
        if (rc) return rc;
    }
    int32_t prev_band = 0;
    for (int32_t i = 0; i < n_items; ++i) {
        const bsh_item& it = items[i];
        int rc = check_segments(&it.seg, true, false);
        if (rc) return rc;
        if (it.grid < 0 || it.grid >= n_grids) return fail_inval("item grid index");
        if (it.band < 0 || it.band >= n_bands) return fail_inval("item band index");
        if (it.band < prev_band) return fail_inval("items must be ordered by band");
        prev_band = it.band;
        const bsh_grid& g = grids[it.grid];
        if (it.n_sky < 1 || it.sky_lo < 0 || it.sky_lo + it.n_sky > g.n_sky)
            return fail_inval("item sky range");
        if (it.seg.weight_per_sky && it.n_sky < 1) return fail_inval("per-sky weights");
        rc = check_window(&it.seg, &g);
        if (rc) return rc;
    }
    return BSH_OK;
}

int64_t item_templates(const bsh_item& it, const bsh_grid& g)
{
    return (int64_t)it.n_sky * g.tasc_off_host[(int64_t)g.n_ap * g.n_per] * g.n_f0;
}

template <typename T>
int dev_alloc(T** p, size_t n)
{
    if (n == 0) n = 1;
    if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) {
        set_error("hipMalloc of %zu bytes failed", n * sizeof(T));
        return BSH_ENOMEM;
    }
    return BSH_OK;
}

__global__ void tag_kernel(int64_t* idx, int64_t n, int32_t k, int32_t shift)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n && idx[e] >= 0) idx[e] |= (e / k) << shift;
}

int enqueue_batched(bsh_plan* p, hipStream_t s)
{
    int rc = zero_words(p->d_counter, 1, s);
    if (rc) return rc;
    rc = launch_batch(p->d_items, p->d_units, p->n_units, p->d_counter, p->blocks, p->lanes, p->chunk,
                      p->mode, s);
    if (rc) return rc;
    if (p->k_item > 0) {
        rc = topk_segmented(p->maps, nullptr, p->d_item_off, p->n_items, p->max_item_len, kItemShift,
                            p->k_item, p->d_item_score, p->d_item_index, p->d_ws_item, p->ws_item, s);
        if (rc) return rc;
        if (p->k_band > 0)
            rc = topk_segmented(p->d_item_score, p->d_item_index, p->d_band_off, p->n_bands,
                                p->max_band_len, 0, p->k_band, p->band_score, p->band_index,
                                p->d_ws_band, p->ws_band, s);
    }
    return rc;
}

}  // namespace

extern "C" int64_t bsh_items_map_floats(const bsh_item* items, int32_t n_items, const bsh_grid* grids,
                                        int32_t n_grids)
{
    clear_error();
    if (!items || !grids || n_items < 1 || n_grids < 1) return -1;
    int64_t tot = 0;
    for (int32_t i = 0; i < n_items; ++i) {
        if (items[i].grid < 0 || items[i].grid >= n_grids) return -1;
        tot += item_templates(items[i], grids[items[i].grid]);
    }
    return tot;
}

static hipError_t release_plan(bsh_plan* p);

extern "C" int bsh_plan_create(const bsh_item* items, int32_t n_items, const bsh_grid* grids,
                               int32_t n_grids, int32_t n_bands, const bsh_plan_opts* opts,
                               float* maps, int64_t maps_floats, float* item_score,
                               int64_t* item_index, float* band_score, int64_t* band_index,
                               int32_t* status, bsh_plan** out)
{
    clear_error();
    if (!out) return fail_inval("plan pointer is NULL");
    *out = nullptr;
    int rc = check_items(items, n_items, grids, n_grids, n_bands);
    if (rc) return rc;
    bsh_plan_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    const int lanes = o.lanes ? o.lanes : kDefaultLanes;
    const int chunk = o.chunk ? o.chunk : kDefaultChunk;
    if (!valid_tile_shape(lanes, chunk)) return fail_inval("tile shape: lanes 64/128/256/512, chunk 128/256/512");
    if (o.variant < BSH_VARIANT_AUTO || o.variant > BSH_VARIANT_TABLE) return fail_inval("variant");
    if (o.k_item < 0 || o.k_band < 0) return fail_inval("k_item / k_band < 0");
    if (o.k_band > 0 && o.k_item == 0) return fail_inval("band lists need item lists");
    if (o.k_band > 0 && (!band_score || !band_index)) return fail_inval("band outputs are NULL");
    if (o.k_item > 0 && (!item_score || !item_index)) return fail_inval("item outputs are NULL");
    if (!maps) return fail_inval("maps is NULL");
    const int64_t need = bsh_items_map_floats(items, n_items, grids, n_grids);
    if (maps_floats < need) {
        set_error("maps holds %lld floats, %lld needed", (long long)maps_floats, (long long)need);
        return BSH_ENOMEM;
    }

    bsh_plan* p = new bsh_plan();
    p->n_items = n_items;
    p->n_bands = n_bands;
    p->k_item = o.k_item;
    p->k_band = o.k_band;
    p->lanes = lanes;
    p->chunk = chunk;
    p->mode = kernel_mode(o.variant, false);
    p->use_graph = o.use_graph != 0;
    p->maps = maps;
    p->band_score = band_score;
    p->band_index = band_index;
    p->d_item_score = item_score;
    p->d_item_index = item_index;

    // item descriptors, map offsets and the unit queue
    std::vector<WorkUnit> units;
    std::vector<int64_t> unit_cost;
    p->items.resize(n_items);
    p->plain.resize(n_items);
    p->plain_blocks.resize(n_items);
    p->item_off.assign(n_items + 1, 0);
    p->band_off.assign(n_bands + 1, 0);
    std::vector<int32_t> tile_start(BSH_MAX_PER + 1);
    for (int32_t i = 0; i < n_items; ++i) {
        const bsh_item& it = items[i];
        const bsh_grid& g = grids[it.grid];
        const int64_t n_t = item_templates(it, g);
        fill_desc(p->items[i], &it.seg, &g, it.sky_lo, it.n_sky, nullptr, maps + p->item_off[i], status);
        p->item_off[i + 1] = p->item_off[i] + n_t;
        p->max_item_len = std::max(p->max_item_len, n_t);
        std::vector<int64_t> groups(g.n_per);
        const int64_t tiles = plan_tiles(&g, lanes, tile_start.data(), groups.data());
        PlainLaunch& pl = p->plain[i];
        std::memset(&pl, 0, sizeof(pl));
        pl.d = p->items[i];
        pl.tiles_per_sky = (int32_t)tiles;
        std::copy(tile_start.begin(), tile_start.end(), pl.tile_start);
        p->plain_blocks[i] = tiles * it.n_sky;
        if (it.seg.n_seg == 0) continue;   // the map is zero-filled at run time
        for (int32_t s = 0; s < it.n_sky; ++s)
            for (int32_t ip = 0; ip < g.n_per; ++ip) {
                const int64_t nt = (groups[ip] + lanes - 1) / lanes;
                for (int64_t t = 0; t < nt; ++t) {
                    units.push_back(WorkUnit{i, s, ip, (int32_t)t});
                    unit_cost.push_back(it.seg.n_seg);
                }
            }
    }
    for (int32_t i = 0; i < n_items; ++i) p->band_off[items[i].band + 1] += o.k_item;
    for (int32_t b = 0; b < n_bands; ++b) {
        p->band_off[b + 1] += p->band_off[b];
        p->max_band_len = std::max(p->max_band_len, p->band_off[b + 1] - p->band_off[b]);
    }
    // longest-processing-time-first order (stable, so equal costs keep item order)
    if (o.lpt) {
        std::vector<int64_t> order(units.size());
        for (size_t u = 0; u < order.size(); ++u) order[u] = (int64_t)u;
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t a, int64_t b) { return unit_cost[a] > unit_cost[b]; });
        std::vector<WorkUnit> sorted(units.size());
        for (size_t u = 0; u < order.size(); ++u) sorted[u] = units[order[u]];
        units.swap(sorted);
    }
    p->n_units = (int64_t)units.size();

    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        set_error("bsh_plan_create: cannot query the current device");
        delete p;
        return BSH_EHIP;
    }
    p->blocks = std::max(1, n_cu) * batch_blocks_per_cu(lanes, chunk, p->mode);
    if (o.blocks > 0) p->blocks = o.blocks;

    rc = dev_alloc(&p->d_items, n_items);
    if (!rc) rc = dev_alloc(&p->d_units, units.size());
    if (!rc) rc = dev_alloc(&p->d_counter, 64);
    if (!rc) rc = dev_alloc(&p->d_item_off, n_items + 1);
    if (!rc) rc = dev_alloc(&p->d_band_off, n_bands + 1);
    if (!rc && p->k_item > 0) {
        // the batched run takes one list per item in one segmented call, the plain run one
        // single-segment call per item: room for either
        p->ws_item = std::max(topk_workspace_bytes(n_items, p->k_item), topk_workspace_bytes(1, p->k_item));
        if (!rc) rc = dev_alloc((char**)&p->d_ws_item, p->ws_item);
        if (!rc && p->k_band > 0) {
            p->ws_band = topk_workspace_bytes(n_bands, p->k_band);
            rc = dev_alloc((char**)&p->d_ws_band, p->ws_band);
        }
    }
    if (!rc && (hipMemcpy(p->d_items, p->items.data(), sizeof(ItemDesc) * n_items, hipMemcpyHostToDevice) != hipSuccess ||
                (!units.empty() && hipMemcpy(p->d_units, units.data(), sizeof(WorkUnit) * units.size(),
                                             hipMemcpyHostToDevice) != hipSuccess) ||
                hipMemcpy(p->d_item_off, p->item_off.data(), sizeof(int64_t) * (n_items + 1),
                          hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(p->d_band_off, p->band_off.data(), sizeof(int64_t) * (n_bands + 1),
                          hipMemcpyHostToDevice) != hipSuccess)) {
        rc = check_launch("bsh_plan_create copies");
        if (!rc) rc = BSH_EHIP;
    }
    if (!rc && p->use_graph) {
        if (hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess) {
            rc = check_launch("plan stream");
            if (!rc) rc = BSH_EHIP;
        } else if (hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = check_launch("begin capture");
            if (!rc) rc = BSH_EHIP;
        } else {
            int rc2 = enqueue_batched(p, p->capture_stream);
            hipError_t e = hipStreamEndCapture(p->capture_stream, &p->graph);
            if (rc2) rc = rc2;
            else if (e != hipSuccess) { set_error("end capture: %s", hipGetErrorString(e)); rc = BSH_EHIP; }
            else if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
                rc = check_launch("graph instantiate");
                if (!rc) rc = BSH_EHIP;
            }
        }
    }
    if (rc) {
        (void)release_plan(p);   // keeps the error text of the step that failed
        return rc;
    }
    *out = p;
    return BSH_OK;
}

extern "C" int bsh_plan_run(bsh_plan* p, bsh_stream stream)
{
    clear_error();
    if (!p) return fail_inval("plan is NULL");
    hipStream_t s = (hipStream_t)stream;
    for (int32_t i = 0; i < p->n_items; ++i)
        if (p->items[i].n_seg == 0) {
            int rc = zero_words(p->maps + p->item_off[i], p->item_off[i + 1] - p->item_off[i], s);
            if (rc) return rc;
        }
    if (p->use_graph && p->exec) {
        if (hipGraphLaunch(p->exec, s) != hipSuccess) {
            int rc = check_launch("graph launch");
            return rc ? rc : BSH_EHIP;
        }
        return BSH_OK;
    }
    return enqueue_batched(p, s);
}

extern "C" int bsh_plan_run_plain(bsh_plan* p, bsh_stream stream)
{
    clear_error();
    if (!p) return fail_inval("plan is NULL");
    hipStream_t s = (hipStream_t)stream;
    for (int32_t i = 0; i < p->n_items; ++i) {
        const int64_t len = p->item_off[i + 1] - p->item_off[i];
        int rc;
        if (p->items[i].n_seg == 0)
            rc = zero_words(p->maps + p->item_off[i], len, s);
        else
            rc = launch_plain(p->plain[i], p->plain_blocks[i], p->lanes, p->chunk, p->mode, s);
        if (rc) return rc;
        if (p->k_item > 0) {
            // one list per item, from that item's own launch
            rc = topk_segmented(p->maps, nullptr, p->d_item_off + i, 1, len, 0, p->k_item,
                                p->d_item_score + (size_t)i * p->k_item,
                                p->d_item_index + (size_t)i * p->k_item, p->d_ws_item, p->ws_item, s);
            if (rc) return rc;
        }
    }
    if (p->k_item > 0) {
        // the per-item lists carry positions; give them the item prefix, then merge per band
        const int64_t n = (int64_t)p->n_items * p->k_item;
        hipLaunchKernelGGL(tag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p->d_item_index, n,
                           p->k_item, kItemShift);
        int rc = check_launch("tag item lists");
        if (rc) return rc;
        if (p->k_band > 0)
            return topk_segmented(p->d_item_score, p->d_item_index, p->d_band_off, p->n_bands,
                                  p->max_band_len, 0, p->k_band, p->band_score, p->band_index,
                                  p->d_ws_band, p->ws_band, s);
    }
    return BSH_OK;
}

extern "C" int64_t bsh_plan_units(const bsh_plan* p) { return p ? p->n_units : -1; }

extern "C" int32_t bsh_plan_blocks(const bsh_plan* p) { return p ? p->blocks : -1; }

// Release everything a plan owns, even if one release fails; returns the first failure.
static hipError_t release_plan(bsh_plan* p)
{
    hipError_t first = hipSuccess;
    auto keep = [&](hipError_t e) {
        if (first == hipSuccess && e != hipSuccess) first = e;
    };
    if (p->exec) keep(hipGraphExecDestroy(p->exec));
    if (p->graph) keep(hipGraphDestroy(p->graph));
    if (p->capture_stream) keep(hipStreamDestroy(p->capture_stream));
    void* bufs[] = {p->d_items, p->d_units, p->d_counter, p->d_item_off, p->d_band_off, p->d_ws_item,
                    p->d_ws_band};
    for (void* b : bufs)
        if (b) keep(hipFree(b));
    delete p;
    return first;
}

extern "C" int bsh_plan_destroy(bsh_plan* p)
{
    clear_error();
    if (!p) return BSH_OK;
    const hipError_t e = release_plan(p);
    if (e != hipSuccess) {
        set_error("bsh_plan_destroy: %s", hipGetErrorString(e));
        return BSH_EHIP;
    }
    return BSH_OK;
}
