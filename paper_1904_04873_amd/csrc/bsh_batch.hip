// Batched stage 1 over many work items (sky patches x bands) with uneven sizes: one launch over
// a queue of (item, pixel, period, tile) units ordered longest-first (persistent blocks pulling
// units from a counter, or one block per unit), then per-item and per-band top-lists, all
// captured in one HIP graph.
//
// The paper splits a search into independent band x sky-patch x binary-block jobs (eq:cost)
// and notes that the GPU idles while the host prepares the next job; here the whole set of
// jobs is one device-side queue, so the tail of one item overlaps the start of the next.
//
// Bounded memory.  A search keeps only the top candidates of each band (Sec. IV.C), and the
// stage-1 maps of a whole band of sky patches do not fit in HBM (eq:RAM1 counts them per patch).
// When the caller's map buffer is smaller than all maps together, the items are split, in
// order, into passes whose maps fit in it; each pass is one count launch followed by the
// top-k of each of its items, after which the buffer is reused.  The per-band lists are then
// merged from the item lists, which is exact: the best k of a union are among the best k of
// each part.
#include <algorithm>
#include <cstring>
#include <vector>

#include "bsh_count.h"

struct bsh_plan {
    int32_t n_items = 0, n_bands = 0, k_item = 0, k_band = 0;
    int32_t lanes = bsh::kDefaultLanes, chunk = bsh::kDefaultChunk, blocks = 0;
    bool use_graph = false;
    bool persistent = false;
    int32_t mode = 2;
    int32_t n_words = 1;                          // widest staged row of any item (sizes the rows' LDS)
    int64_t n_units = 0, max_band_len = 0;
    std::vector<bsh::ItemDesc> items;            // host copies (plain mode)
    std::vector<bsh::PlainLaunch> plain;          // per-item plain launch parameters
    std::vector<int64_t> plain_blocks;
    std::vector<int64_t> band_off;                // host offsets of the band lists' inputs
    // passes: items [pass_item[q], pass_item[q+1]), units [pass_unit[q], pass_unit[q+1])
    std::vector<int32_t> pass_item;               // [n_passes + 1]
    std::vector<int64_t> pass_unit;               // [n_passes + 1]
    std::vector<int64_t> pass_off_at;             // [n_passes] first entry of the pass in d_pass_off
    std::vector<int64_t> pass_max_len;            // [n_passes] longest item map of the pass
    std::vector<int64_t> item_start;              // [n_items] map offset of each item in the buffer
    std::vector<int64_t> item_len;                // [n_items]
    bsh::ItemDesc* d_items = nullptr;
    bsh::WorkUnit* d_units = nullptr;
    uint32_t* d_counter = nullptr;                // one queue counter per pass
    int64_t* d_pass_off = nullptr;                // per pass: item offsets inside the buffer, then its end
    int64_t* d_single_off = nullptr;              // [n_items][2]: (start, end) of each item's map
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

    int32_t n_passes() const { return (int32_t)pass_item.size() - 1; }
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

// Items without segments have all-zero maps; their buffer regions are cleared by a fill
// kernel inside the pass that holds them (earlier passes may have used the same memory).
int zero_empty_items(bsh_plan* p, int32_t lo, int32_t hi, hipStream_t s)
{
    for (int32_t i = lo; i < hi; ++i)
        if (p->items[i].n_seg == 0) {
            const int rc = zero_words(p->maps + p->item_start[i], p->item_len[i], s);
            if (rc) return rc;
        }
    return BSH_OK;
}

// The count launches of every pass, each followed (when lists are asked for) by
// the top-k of each of its items; then the band lists.
int enqueue_batched(bsh_plan* p, hipStream_t s, bool count_only)
{
    int rc = zero_words(p->d_counter, p->n_passes(), s);
    if (rc) return rc;
    for (int32_t q = 0; q < p->n_passes(); ++q) {
        const int32_t lo = p->pass_item[q], hi = p->pass_item[q + 1];
        rc = zero_empty_items(p, lo, hi, s);
        if (rc) return rc;
        const int64_t u0 = p->pass_unit[q], nu = p->pass_unit[q + 1] - u0;
        if (nu > 0) {
            rc = launch_batch(p->d_items, p->d_units + u0, nu, p->d_counter + q, p->blocks, p->lanes, p->chunk,
                              p->mode, p->n_words, p->persistent, s);
            if (rc) return rc;
        }
        if (p->k_item > 0 && !count_only) {
            rc = topk_segmented(p->maps, nullptr, p->d_pass_off + p->pass_off_at[q], hi - lo, p->pass_max_len[q],
                                kItemShift, p->k_item, p->d_item_score + (size_t)lo * p->k_item,
                                p->d_item_index + (size_t)lo * p->k_item, p->d_ws_item, p->ws_item, s,
                                (int64_t)lo << kItemShift);
            if (rc) return rc;
        }
    }
    if (p->k_item > 0 && p->k_band > 0 && !count_only)
        rc = topk_segmented(p->d_item_score, p->d_item_index, p->d_band_off, p->n_bands, p->max_band_len, 0,
                            p->k_band, p->band_score, p->band_index, p->d_ws_band, p->ws_band, s);
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
    if (n_items > 65535) return fail_inval("more than 65535 items");
    const int64_t need = bsh_items_map_floats(items, n_items, grids, n_grids);
    int64_t largest = 0;
    for (int32_t i = 0; i < n_items; ++i)
        largest = std::max(largest, item_templates(items[i], grids[items[i].grid]));
    if (maps_floats < largest) {
        set_error("maps holds %lld floats, the largest item needs %lld", (long long)maps_floats,
                  (long long)largest);
        return BSH_ENOMEM;
    }
    if (maps_floats < need && o.k_item == 0)
        return fail_inval("a map buffer smaller than all maps together needs item lists (k_item > 0)");

    bsh_plan* p = new bsh_plan();
    p->n_items = n_items;
    p->n_bands = n_bands;
    p->k_item = o.k_item;
    p->k_band = o.k_band;
    p->lanes = lanes;
    p->chunk = chunk;
    // one kernel for the whole plan: the ELL1 form when any grid has an eccentricity pair (its
    // zero eccentric terms leave circular items' maps as the circular kernel gives them)
    int ecc = 0;
    for (int32_t q = 0; q < n_grids; ++q) ecc = std::max(ecc, ecc_mode(&grids[q]));
    p->mode = kernel_mode(o.variant, false) + ecc;
    p->use_graph = o.use_graph != 0;
    p->maps = maps;
    p->band_score = band_score;
    p->band_index = band_index;
    p->d_item_score = item_score;
    p->d_item_index = item_index;

    // passes: consecutive items whose maps fit in the buffer together
    p->item_start.assign(n_items, 0);
    p->item_len.assign(n_items, 0);
    p->pass_item.push_back(0);
    int64_t fill = 0;
    for (int32_t i = 0; i < n_items; ++i) {
        const int64_t n_t = item_templates(items[i], grids[items[i].grid]);
        if (fill + n_t > maps_floats) {
            p->pass_item.push_back(i);
            fill = 0;
        }
        p->item_start[i] = fill;
        p->item_len[i] = n_t;
        fill += n_t;
    }
    p->pass_item.push_back(n_items);
    const int32_t n_passes = p->n_passes();
    std::vector<int64_t> pass_off;          // per pass: (hi - lo + 1) offsets
    for (int32_t q = 0; q < n_passes; ++q) {
        p->pass_off_at.push_back((int64_t)pass_off.size());
        int64_t mx = 0;
        for (int32_t i = p->pass_item[q]; i < p->pass_item[q + 1]; ++i) {
            pass_off.push_back(p->item_start[i]);
            mx = std::max(mx, p->item_len[i]);
        }
        const int32_t last = p->pass_item[q + 1] - 1;
        pass_off.push_back(p->item_start[last] + p->item_len[last]);
        p->pass_max_len.push_back(mx);
    }
    std::vector<int64_t> single_off(2 * (size_t)n_items);
    for (int32_t i = 0; i < n_items; ++i) {
        single_off[2 * i] = p->item_start[i];
        single_off[2 * i + 1] = p->item_start[i] + p->item_len[i];
    }

    // item descriptors and the unit queue, longest-processing-time first inside each pass
    // (stable, so equal costs keep item order)
    std::vector<WorkUnit> units;
    p->items.resize(n_items);
    p->plain.resize(n_items);
    p->plain_blocks.resize(n_items);
    p->band_off.assign(n_bands + 1, 0);
    std::vector<int32_t> tile_start(BSH_MAX_PER + 1);
    p->pass_unit.push_back(0);
    // the proven form of the table kernel when every item with segments is proven (proven_window)
    bool all_proven = mode_table(p->mode);
    for (int32_t q = 0; q < n_passes; ++q) {
        std::vector<WorkUnit> pu;
        std::vector<int64_t> cost;
        for (int32_t i = p->pass_item[q]; i < p->pass_item[q + 1]; ++i) {
            const bsh_item& it = items[i];
            const bsh_grid& g = grids[it.grid];
            fill_desc(p->items[i], &it.seg, &g, it.sky_lo, it.n_sky, nullptr, maps + p->item_start[i], status);
            if (it.seg.n_seg > 0 && !prove_item(p->mode, p->items[i], &it.seg, &g)) all_proven = false;
            std::vector<int64_t> groups(g.n_per);
            const int tt = tile_templates(p->mode, lanes);
            const int64_t tiles = plan_tiles(&g, tt, tile_start.data(), groups.data());
            p->n_words = std::max(p->n_words, p->items[i].n_words);
            PlainLaunch& pl = p->plain[i];
            std::memset(&pl, 0, sizeof(pl));
            pl.d = p->items[i];
            pl.tiles_per_sky = (int32_t)tiles;
            std::copy(tile_start.begin(), tile_start.end(), pl.tile_start);
            p->plain_blocks[i] = tiles * it.n_sky;
            if (it.seg.n_seg == 0) continue;   // the map is zero-filled at run time
            for (int32_t sk = 0; sk < it.n_sky; ++sk)
                for (int32_t ip = 0; ip < g.n_per; ++ip) {
                    const int64_t nt = (groups[ip] + tt - 1) / tt;
                    for (int64_t t = 0; t < nt; ++t) {
                        pu.push_back(WorkUnit{i, sk, ip, (int32_t)t});
                        cost.push_back(it.seg.n_seg);
                    }
                }
        }
        if (o.lpt) {
            std::vector<int64_t> order(pu.size());
            for (size_t u = 0; u < order.size(); ++u) order[u] = (int64_t)u;
            std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cost[a] > cost[b]; });
            for (int64_t u : order) units.push_back(pu[u]);
        } else {
            units.insert(units.end(), pu.begin(), pu.end());
        }
        p->pass_unit.push_back((int64_t)units.size());
    }
    for (int32_t i = 0; i < n_items; ++i) p->band_off[items[i].band + 1] += o.k_item;
    for (int32_t b = 0; b < n_bands; ++b) {
        p->band_off[b + 1] += p->band_off[b];
        p->max_band_len = std::max(p->max_band_len, p->band_off[b + 1] - p->band_off[b]);
    }
    p->n_units = (int64_t)units.size();
    if (all_proven) p->mode += kProvenMode;   // (the descriptors hold the proofs' bounds)

    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        set_error("bsh_plan_create: cannot query the current device");
        delete p;
        return BSH_EHIP;
    }
    // Launch form: asked for, or (persistent < 0) the persistent blocks when as many of them fit
    // per CU as blocks of the one-block-per-unit form (both are bound by the tile's registers and
    // LDS; the persistent loop keeps more registers live, and with fewer resident blocks it is the
    // slower form).  Persistent form: CUs x resident blocks; else the largest pass's unit count.
    const int per_cu = batch_blocks_per_cu(lanes, chunk, p->mode, p->n_words, true);
    p->persistent = o.persistent > 0 ||
                    (o.persistent < 0 && per_cu >= batch_blocks_per_cu(lanes, chunk, p->mode, p->n_words, false));
    p->blocks = std::max(1, n_cu) * per_cu;
    if (o.blocks > 0) p->blocks = o.blocks;
    if (!p->persistent) {
        int64_t widest = 0;
        for (int32_t q = 0; q < n_passes; ++q) widest = std::max(widest, p->pass_unit[q + 1] - p->pass_unit[q]);
        if (widest > 0x7fffffff) {
            set_error("more than 2^31 - 1 units in one pass");
            delete p;
            return BSH_EINVAL;
        }
        p->blocks = (int32_t)widest;
    }

    rc = dev_alloc(&p->d_items, n_items);
    if (!rc) rc = dev_alloc(&p->d_units, units.size());
    if (!rc) rc = dev_alloc(&p->d_counter, (size_t)n_passes);
    if (!rc) rc = dev_alloc(&p->d_pass_off, pass_off.size());
    if (!rc) rc = dev_alloc(&p->d_single_off, single_off.size());
    if (!rc) rc = dev_alloc(&p->d_band_off, n_bands + 1);
    if (!rc && p->k_item > 0) {
        // the batched run takes one list per item of a pass in one segmented call, the plain run
        // one single-segment call per item: room for either
        int32_t widest = 1;
        for (int32_t q = 0; q < n_passes; ++q) widest = std::max(widest, p->pass_item[q + 1] - p->pass_item[q]);
        // with room for the segmented top-k's candidate pass when that costs at most 2 GiB more
        const size_t plain_ws = topk_workspace_bytes(widest, p->k_item);
        const size_t cand_ws = topk_candidate_workspace_bytes(widest, p->k_item);
        p->ws_item = std::max(cand_ws - plain_ws <= ((size_t)2 << 30) ? cand_ws : plain_ws,
                              topk_workspace_bytes(1, p->k_item));
        if (!rc) rc = dev_alloc((char**)&p->d_ws_item, p->ws_item);
        if (!rc && p->k_band > 0) {
            p->ws_band = topk_candidate_workspace_bytes(n_bands, p->k_band);
            rc = dev_alloc((char**)&p->d_ws_band, p->ws_band);
        }
    }
    if (!rc && (hipMemcpy(p->d_items, p->items.data(), sizeof(ItemDesc) * n_items, hipMemcpyHostToDevice) != hipSuccess ||
                (!units.empty() && hipMemcpy(p->d_units, units.data(), sizeof(WorkUnit) * units.size(),
                                             hipMemcpyHostToDevice) != hipSuccess) ||
                hipMemcpy(p->d_pass_off, pass_off.data(), sizeof(int64_t) * pass_off.size(),
                          hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(p->d_single_off, single_off.data(), sizeof(int64_t) * single_off.size(),
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
            int rc2 = enqueue_batched(p, p->capture_stream, false);
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
    if (p->use_graph && p->exec) {
        if (hipGraphLaunch(p->exec, s) != hipSuccess) {
            int rc = check_launch("graph launch");
            return rc ? rc : BSH_EHIP;
        }
        return BSH_OK;
    }
    return enqueue_batched(p, s, false);
}

extern "C" int bsh_plan_run_count(bsh_plan* p, bsh_stream stream)
{
    clear_error();
    if (!p) return fail_inval("plan is NULL");
    return enqueue_batched(p, (hipStream_t)stream, true);
}

extern "C" int bsh_plan_run_plain(bsh_plan* p, bsh_stream stream)
{
    clear_error();
    if (!p) return fail_inval("plan is NULL");
    hipStream_t s = (hipStream_t)stream;
    for (int32_t i = 0; i < p->n_items; ++i) {
        const int64_t len = p->item_len[i];
        int rc;
        if (p->items[i].n_seg == 0)
            rc = zero_words(p->maps + p->item_start[i], len, s);
        else
            rc = launch_plain(p->plain[i], p->plain_blocks[i], p->lanes, p->chunk, p->mode, p->items[i].n_words, s);
        if (rc) return rc;
        if (p->k_item > 0) {
            // one list per item, from that item's own launch, indices tagged with the item
            rc = topk_segmented(p->maps, nullptr, p->d_single_off + 2 * i, 1, len, 0, p->k_item,
                                p->d_item_score + (size_t)i * p->k_item,
                                p->d_item_index + (size_t)i * p->k_item, p->d_ws_item, p->ws_item, s,
                                (int64_t)i << kItemShift);
            if (rc) return rc;
        }
    }
    if (p->k_item > 0 && p->k_band > 0)
        return topk_segmented(p->d_item_score, p->d_item_index, p->d_band_off, p->n_bands, p->max_band_len, 0,
                              p->k_band, p->band_score, p->band_index, p->d_ws_band, p->ws_band, s);
    return BSH_OK;
}

extern "C" int64_t bsh_plan_units(const bsh_plan* p) { return p ? p->n_units : -1; }

extern "C" int32_t bsh_plan_blocks(const bsh_plan* p) { return p ? p->blocks : -1; }

extern "C" int32_t bsh_plan_persistent(const bsh_plan* p) { return p ? (p->persistent ? 1 : 0) : -1; }

extern "C" int32_t bsh_plan_proven(const bsh_plan* p) { return p ? (mode_proven(p->mode) ? 1 : 0) : -1; }

extern "C" int32_t bsh_plan_passes(const bsh_plan* p) { return p ? p->n_passes() : -1; }

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
    void* bufs[] = {p->d_items, p->d_units, p->d_counter, p->d_pass_off, p->d_single_off, p->d_band_off,
                    p->d_ws_item, p->d_ws_band};
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
