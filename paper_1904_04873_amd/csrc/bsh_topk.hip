// Exact top-k under the total order (score descending, index ascending): the per-band
// top-lists of Sec. IV.C (N_C candidates out of stage 1, N_CF out of stage 2), for one list
// or for many independent lists ("segments") in the same launches.
//
// Per segment:
// 1. Radix select on the 32-bit order-preserving key of the score: four 8-bit digit passes
//    (block histograms in LDS added into one histogram per pass and segment) find the key T of
//    the k-th best score, the number of scores strictly better, and how many ties at T are
//    still needed.  Every block of a pass derives the digits chosen so far from the previous
//    pass's histogram itself (a block scan), so no launch is spent on picking a digit.
// 2. One compaction pass writes every entry with key > T (and those equal to T when all of
//    them are needed) to the segment's output pool.
// 3. Otherwise ties at T are resolved by index with a second radix select over the index bits
//    of the entries whose key equals T (re-reading the scores instead of buffering the ties,
//    so the workspace stays O(k) per segment), then a pass appends the chosen ties.
// 4. The k chosen entries are ordered by rank counting (each entry counts the entries that
//    precede it), which is exact, deterministic and independent of the arrival order.
// Short segments run all of this in one block (small_topk_kernel).  Everything stays on the
// stream: no host synchronisation, counts live in the workspace.
//
// Candidate pass (several long segments, given the larger workspace): instead of the six or
// more passes over every entry above, one block per segment takes the key T_g of rank m in a
// sample of the segment (runs of consecutive entries spread over it, m chosen so that about a
// quarter of the buffer's room is expected at or above it), one pass copies the entries with
// key >= T_g to a buffer per segment (cand_cap(k) entries), and the selection runs on that
// buffer: one block per segment for k <= kSmallK, else the passes above on the buffers.  It is
// exact whenever at least k_eff entries were copied and none dropped: every entry of the
// segment's top-k then has a key >= T_g.  The segments where either bound fails (a sample that
// misrepresents its segment, mass ties at T_g) are marked and taken by the passes above over
// the whole segments afterwards, whose kernels skip the settled ones.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "bsh_internal.h"

namespace {

using namespace bsh;

constexpr int kThreads = 256;
constexpr int kBins = 256;
constexpr int kMaxBlocksPerSeg = 1024;

constexpr int kKeyPasses = 4;
constexpr int kMaxIdxPasses = 8;
constexpr int kHists = kKeyPasses + kMaxIdxPasses;

struct State {
    uint32_t k_eff;          // min(k, segment length)
    uint32_t n_sel;          // output-pool fill
    uint32_t kmax;           // largest chosen key (bucketed ordering)
    uint32_t prefix[kKeyPasses + 1];      // key digits fixed before pass p; prefix[4] = T
    uint32_t remaining[kKeyPasses + 1];   // entries still to take before pass p; remaining[4]
                                          // = ties at T still to take (0 when all are taken)
    uint32_t iremaining[kMaxIdxPasses + 1];   // ties still to take before index pass p
    unsigned long long iprefix[kMaxIdxPasses + 1];   // index digits fixed before index pass p
};

struct Seg {
    const float* score;
    const int64_t* index;    // NULL: implicit index (g << shift) | position
    const int64_t* off;      // [n_segs + 1] device offsets; NULL: one segment [0, n_single)
    int64_t n_single;
    int32_t n_segs;
    int32_t shift;           // implicit-index segment shift (0: position only)
    int32_t k;
    int64_t out_base;        // added to the implicit indices of the written lists (0 for explicit)
    int32_t idx_bits;        // index bits that can differ inside a segment
    int32_t copies;          // copies of each global histogram (blocks add to copy b % copies)
    State* st;               // [n_segs]
    uint32_t* hist;          // [n_segs][kHists][copies][kBins]: key passes, then index passes
    float* sel_score;        // [n_segs][k]
    int64_t* sel_index;      // [n_segs][k]
    uint32_t* rank;          // [n_segs][k]
    // bucketed ordering (k > kRankDirect), else NULL
    int32_t bucket_log2;     // log2 of the buckets per segment
    uint32_t* bcnt;          // [n_segs][buckets] entries per bucket
    uint32_t* bbase;         // [n_segs][buckets] entries in the buckets before
    uint32_t* bfill;         // [n_segs][buckets] scatter cursors
    uint32_t* tkey;          // [n_segs][k] chosen entries grouped by bucket
    float* tscore;           // [n_segs][k]
    int64_t* tindex;         // [n_segs][k]
    // candidate pass: a Seg over the candidate buffers takes segment g as entries
    // [g cand_cap, g cand_cap + min(cand_cnt[g], cand_cap)); the one-block selection records in
    // done_out[g] whether they settle it (cand_keff[g]: k_eff of the full segment).  Launches
    // skip the segments whose done[g] equals done_skip: over the buffers those not settled,
    // over the whole segments those settled.
    const uint32_t* cand_cnt;
    int64_t cand_cap;
    const uint32_t* cand_keff;
    uint32_t* done_out;
    const uint32_t* done;
    uint32_t done_skip;      // segments with done[g] == done_skip are skipped
};

__host__ __device__ inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// A single long segment has up to kMaxBlocksPerSeg blocks adding their histograms to bins
// that hold most entries (the scores share their leading bits), and same-address atomics
// serialize at the L2: each histogram is kept in kHistCopies copies that the blocks spread
// over, summed when a digit is picked.
constexpr int kHistCopies = 16;
__host__ __device__ inline int hist_copies(int32_t n_segs) { return n_segs == 1 ? kHistCopies : 1; }

// Ordering the k chosen entries: up to kRankDirect by counting, for each entry, the entries
// that precede it (k^2 comparisons spread over the device); beyond, the entries are first
// grouped into about k/4 buckets of equal key width between T and the largest chosen key, and
// an entry only counts within its bucket (the buckets before it precede it as a whole).
constexpr int32_t kRankDirect = 16384;

__host__ __device__ inline int bucket_log2(int32_t k)
{
    int b = 8;
    while (b < 16 && (1 << (b + 2)) < k) ++b;
    return b;
}

size_t bucket_bytes(int32_t n_segs, int32_t k)
{
    if (k <= kRankDirect) return 0;
    const size_t ns = (size_t)(n_segs > 0 ? n_segs : 1);
    const size_t nb = (size_t)1 << bucket_log2(k);
    return 3 * align_up(sizeof(uint32_t) * nb * ns) + align_up(sizeof(uint32_t) * (size_t)k * ns) +
           align_up(sizeof(float) * (size_t)k * ns) + align_up(sizeof(int64_t) * (size_t)k * ns);
}

size_t workspace_bytes(int32_t n_segs, int32_t k)
{
    const size_t ns = (size_t)(n_segs > 0 ? n_segs : 1);
    const size_t hb = sizeof(uint32_t) * kHists * kBins * (size_t)hist_copies(n_segs);
    return align_up(sizeof(State) * ns) + align_up(hb * ns) +
           align_up(sizeof(float) * (size_t)k * ns) + align_up(sizeof(int64_t) * (size_t)k * ns) +
           align_up(sizeof(uint32_t) * (size_t)k * ns) + bucket_bytes(n_segs, k);
}

void carve(void* ws, Seg& s)
{
    const size_t ns = (size_t)s.n_segs;
    char* p = (char*)ws;
    s.st = (State*)p;
    p += align_up(sizeof(State) * ns);
    s.copies = hist_copies(s.n_segs);
    s.hist = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * kHists * kBins * (size_t)s.copies * ns);
    s.sel_score = (float*)p;
    p += align_up(sizeof(float) * (size_t)s.k * ns);
    s.sel_index = (int64_t*)p;
    p += align_up(sizeof(int64_t) * (size_t)s.k * ns);
    s.rank = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * (size_t)s.k * ns);
    s.bucket_log2 = 0;
    s.bcnt = s.bbase = s.bfill = s.tkey = nullptr;
    s.tscore = nullptr;
    s.tindex = nullptr;
    if (s.k > kRankDirect) {
        s.bucket_log2 = bucket_log2(s.k);
        const size_t nb = (size_t)1 << s.bucket_log2;
        s.bcnt = (uint32_t*)p;
        p += align_up(sizeof(uint32_t) * nb * ns);
        s.bbase = (uint32_t*)p;
        p += align_up(sizeof(uint32_t) * nb * ns);
        s.bfill = (uint32_t*)p;
        p += align_up(sizeof(uint32_t) * nb * ns);
        s.tkey = (uint32_t*)p;
        p += align_up(sizeof(uint32_t) * (size_t)s.k * ns);
        s.tscore = (float*)p;
        p += align_up(sizeof(float) * (size_t)s.k * ns);
        s.tindex = (int64_t*)p;
    }
}

__device__ __forceinline__ void seg_range(const Seg& s, int g, int64_t& lo, int64_t& hi)
{
    if (s.cand_cnt) {
        lo = (int64_t)g * s.cand_cap;
        hi = lo + min((int64_t)s.cand_cnt[g], s.cand_cap);
    } else if (s.off) {
        lo = s.off[g];
        hi = s.off[g + 1];
    } else {
        lo = 0;
        hi = s.n_single;
    }
}

// Copy 0 of histogram h of segment g; copy c follows at c * kBins.
__device__ __forceinline__ uint32_t* seg_hist(const Seg& s, int g, int h)
{
    return s.hist + ((size_t)g * kHists + h) * (size_t)s.copies * kBins;
}

// Histogram h of segment g summed over its copies into LDS (every thread of the block calls this).
__device__ __forceinline__ void sum_hist(const Seg& s, int g, int h, uint32_t* out)
{
    const uint32_t* src = seg_hist(s, g, h);
    for (int b = threadIdx.x; b < kBins; b += blockDim.x) {
        uint32_t t = 0u;
        for (int c = 0; c < s.copies; ++c) t += src[c * kBins + b];
        out[b] = t;
    }
    __syncthreads();
}

// Order-preserving map float -> uint32 (larger float -> larger key); -0 is folded onto +0.
__device__ __forceinline__ uint32_t score_key(float f)
{
    uint32_t u = __float_as_uint(f);
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}


// Segment g is not this launch's to take (block-uniform): settled by the candidate pass, for the
// passes over the whole segments; not settled, for the passes over the candidate buffers.
__device__ __forceinline__ bool seg_done(const Seg& s, int g) { return s.done && s.done[g] == s.done_skip; }

__device__ __forceinline__ int64_t entry_index(const Seg& s, int g, int64_t e, int64_t lo)
{
    if (s.index) return s.index[e];
    const int64_t pos = e - lo;
    return s.shift > 0 ? (((int64_t)g << s.shift) | pos) : pos;
}

// Count `bin` for every active lane whose `take` is set: lanes sharing the first taker's bin
// are added with one atomic (scores concentrate in few digit values, so this takes most of
// the LDS atomic traffic off the hottest bins).
__device__ __forceinline__ void wave_hist_add(uint32_t* h, bool take, uint32_t bin)
{
    const unsigned long long any = __ballot(take);
    if (!any) return;
    const int leader = __ffsll((long long)any) - 1;
    const uint32_t lb = __shfl(bin, leader);
    const unsigned long long same = __ballot(take && bin == lb);
    if ((int)(threadIdx.x & 63) == leader) atomicAdd(&h[lb], (uint32_t)__popcll(same));
    if (take && bin != lb) atomicAdd(&h[bin], 1u);
}

// Slot in the segment's output pool for every active lane whose `take` is set: one atomic
// per wave.
__device__ __forceinline__ uint32_t wave_claim(uint32_t* n_sel, bool take)
{
    const unsigned long long m = __ballot(take);
    if (!m) return 0u;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0u;
    if (lane == leader) base = atomicAdd(n_sel, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// Grid-stride walk over scores [lo, hi) with four independent loads in flight per lane.
template <typename F>
__device__ __forceinline__ void for_each_score(const float* __restrict__ score, int64_t lo, int64_t hi, F f)
{
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int64_t e = lo + (int64_t)blockIdx.x * kThreads + threadIdx.x;
    for (; e + 3 * stride < hi; e += 4 * stride) {
        const float a = score[e], b = score[e + stride], c = score[e + 2 * stride], d = score[e + 3 * stride];
        f(e, a);
        f(e + stride, b);
        f(e + 2 * stride, c);
        f(e + 3 * stride, d);
    }
    for (; e < hi; e += stride) f(e, score[e]);
}

// The digit that holds the rem-th entry when the 256 bins of h are taken in order (from the top
// for scores, from the bottom for tie indices), and how many entries the bins before it hold.
// A block scan over the bins (every thread of the block calls this; at least 256 threads).
// When the bins hold fewer than rem entries the last bin in take order is returned.
__device__ void pick_digit(const uint32_t* h, uint32_t rem, bool from_top, uint32_t* scan, int* d_out,
                           uint32_t* before_out)
{
    const int t = threadIdx.x;
    const uint32_t v = t < kBins ? h[from_top ? kBins - 1 - t : t] : 0u;
    if (t < kBins) scan[t] = v;
    __syncthreads();
    for (int off = 1; off < kBins; off <<= 1) {
        const uint32_t add = (t < kBins && t >= off) ? scan[t - off] : 0u;
        __syncthreads();
        if (t < kBins) scan[t] += add;
        __syncthreads();
    }
    if (t < kBins) {
        const uint32_t incl = scan[t], excl = incl - v;
        if ((excl < rem && rem <= incl) || (t == kBins - 1 && incl < rem)) {
            *d_out = from_top ? kBins - 1 - t : t;
            *before_out = excl;
        }
    }
    __syncthreads();
}

// State, histograms and ranks of segment blockIdx.y start from zero; grid.x covers the k
// ranks, and its blocks share the histograms' zeroing.
__global__ void init_kernel(Seg s)
{
    const int g = blockIdx.y;
    if (seg_done(s, g)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t lo, hi;
        seg_range(s, g, lo, hi);
        const int64_t len = hi - lo;
        const uint32_t k_eff = (uint32_t)(len < (int64_t)s.k ? len : (int64_t)s.k);
        s.st[g].k_eff = k_eff;
        s.st[g].n_sel = 0u;
        s.st[g].kmax = 0u;
        s.st[g].prefix[0] = 0u;
        s.st[g].remaining[0] = k_eff;
        s.st[g].iprefix[0] = 0ull;
        s.st[g].iremaining[0] = 0u;
    }
    const size_t per = (size_t)kHists * s.copies * kBins;
    for (size_t b = (size_t)blockIdx.x * blockDim.x + threadIdx.x; b < per; b += (size_t)gridDim.x * blockDim.x)
        s.hist[(size_t)g * per + b] = 0u;
    if (s.bcnt) {
        const size_t nb = (size_t)1 << s.bucket_log2;
        for (size_t b = (size_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (size_t)gridDim.x * blockDim.x) {
            s.bcnt[(size_t)g * nb + b] = 0u;
            s.bfill[(size_t)g * nb + b] = 0u;
        }
    }
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (uint32_t)s.k) s.rank[(size_t)g * s.k + e] = 0u;
}

// The key digits fixed before pass p (prefix, entries still to take), derived in every block
// from pass p-1's histogram; block 0 records them.  After the last pass, count_at is the
// number of entries equal to the full key T.
struct KeyStep {
    uint32_t prefix, remaining, count_at;
};

__device__ KeyStep key_step(const Seg& s, int g, int p, uint32_t* scan)
{
    __shared__ int d;
    __shared__ uint32_t before;
    const uint32_t pre = s.st[g].prefix[p - 1];
    const uint32_t rem = s.st[g].remaining[p - 1];
    KeyStep k{pre << 8, 0u, 0u};
    if (rem == 0u) return k;      // block-uniform
    __shared__ uint32_t h[kBins];
    sum_hist(s, g, p - 1, h);
    pick_digit(h, rem, true, scan, &d, &before);
    k.prefix = (pre << 8) | (uint32_t)d;
    k.remaining = rem - before;
    k.count_at = h[d];
    return k;
}

// Histogram of key digit `pass` (0 = most significant byte) over entries matching the prefix.
__global__ __launch_bounds__(kThreads) void key_hist_kernel(Seg s, int pass)
{
    __shared__ uint32_t h[kBins], scan[kBins];
    const int g = blockIdx.y;
    if (seg_done(s, g)) return;
    uint32_t prefix = 0u, remaining = s.st[g].remaining[0];
    if (pass > 0) {
        const KeyStep k = key_step(s, g, pass, scan);
        prefix = k.prefix;
        remaining = k.remaining;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            s.st[g].prefix[pass] = prefix;
            s.st[g].remaining[pass] = remaining;
        }
    }
    if (remaining == 0u) return;
    for (int b = threadIdx.x; b < kBins; b += kThreads) h[b] = 0u;
    __syncthreads();
    int64_t lo, hi;
    seg_range(s, g, lo, hi);
    const int shift = 24 - 8 * pass;
    for_each_score(s.score, lo, hi, [&](int64_t, float sc) {
        const uint32_t key = score_key(sc);
        wave_hist_add(h, pass == 0 || (key >> (shift + 8)) == prefix, (key >> shift) & 0xffu);
    });
    __syncthreads();
    uint32_t* gh = seg_hist(s, g, pass) + (blockIdx.x % s.copies) * kBins;
    for (int b = threadIdx.x; b < kBins; b += kThreads)
        if (h[b]) atomicAdd(&gh[b], h[b]);
}

// Entries with key > T go to the output pool (and those equal to T when all of them are
// needed).  Each block gathers its entries in LDS and reserves pool slots with one atomic (a
// single pool counter hit once per entry serializes at the L2); entries beyond the LDS buffer
// reserve their slots directly.
__global__ __launch_bounds__(kThreads) void split_kernel(Seg s)
{
    constexpr uint32_t kCap = 1024;
    __shared__ float lsc[kCap];
    __shared__ int64_t lix[kCap];
    __shared__ uint32_t lcount, gbase, scan[kBins];
    const int g = blockIdx.y;
    if (seg_done(s, g)) return;
    const uint32_t k_eff = s.st[g].k_eff;
    if (k_eff == 0u) return;
    const KeyStep k = key_step(s, g, kKeyPasses, scan);
    const uint32_t T = k.prefix;
    // after the last digit count_at is the number of entries equal to T
    const bool tie_all = k.count_at == k.remaining;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.st[g].prefix[kKeyPasses] = T;
        s.st[g].remaining[kKeyPasses] = tie_all ? 0u : k.remaining;
        s.st[g].iprefix[0] = 0ull;
        s.st[g].iremaining[0] = tie_all ? 0u : k.remaining;
    }
    if (threadIdx.x == 0) lcount = 0u;
    __syncthreads();
    int64_t lo, hi;
    seg_range(s, g, lo, hi);
    for_each_score(s.score, lo, hi, [&](int64_t e, float sc) {
        const uint32_t key = score_key(sc);
        const bool take = key > T || (tie_all && key == T);
        const uint32_t pos = wave_claim(&lcount, take);
        if (take) {
            const int64_t ix = entry_index(s, g, e, lo);
            if (pos < kCap) {
                lsc[pos] = sc;
                lix[pos] = ix;
            } else {
                const uint32_t gp = atomicAdd(&s.st[g].n_sel, 1u);
                if (gp < k_eff) {
                    s.sel_score[(size_t)g * s.k + gp] = sc;
                    s.sel_index[(size_t)g * s.k + gp] = ix;
                }
            }
        }
    });
    __syncthreads();
    const uint32_t n_local = min(lcount, kCap);
    if (threadIdx.x == 0) gbase = n_local ? atomicAdd(&s.st[g].n_sel, n_local) : 0u;
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < n_local; q += kThreads) {
        const uint32_t pos = gbase + q;
        if (pos < k_eff) {
            s.sel_score[(size_t)g * s.k + pos] = lsc[q];
            s.sel_index[(size_t)g * s.k + pos] = lix[q];
        }
    }
}

// The index digits fixed before tie pass p (smallest indices win: digits are taken from the
// low end), derived in every block from pass p-1's histogram; block 0 records them.
struct TieStep {
    unsigned long long prefix;
    uint32_t remaining;
};

__device__ TieStep tie_step(const Seg& s, int g, int p, uint32_t* scan, bool record)
{
    __shared__ int d;
    __shared__ uint32_t below;
    const unsigned long long pre = s.st[g].iprefix[p - 1];
    const uint32_t rem = s.st[g].iremaining[p - 1];
    TieStep t{pre << 8, 0u};
    if (rem != 0u) {      // block-uniform
        __shared__ uint32_t h[kBins];
        sum_hist(s, g, kKeyPasses + p - 1, h);
        pick_digit(h, rem, false, scan, &d, &below);
        t.prefix = (pre << 8) | (unsigned long long)d;
        t.remaining = rem - below;
    }
    if (record && blockIdx.x == 0 && threadIdx.x == 0) {
        s.st[g].iprefix[p] = t.prefix;
        s.st[g].iremaining[p] = t.remaining;
    }
    return t;
}

// Histogram of index digit `pass` over entries whose key equals T.  The digits cover the
// low idx_bits of the index (rounded up to bytes); the bits above are equal in a segment.
__global__ __launch_bounds__(kThreads) void tie_hist_kernel(Seg s, int pass, int n_pass)
{
    __shared__ uint32_t h[kBins], scan[kBins];
    const int g = blockIdx.y;
    if (seg_done(s, g)) return;
    unsigned long long prefix = 0ull;
    uint32_t remaining = s.st[g].iremaining[0];
    if (pass > 0) {
        const TieStep t = tie_step(s, g, pass, scan, true);
        prefix = t.prefix;
        remaining = t.remaining;
    }
    if (remaining == 0u) return;
    for (int b = threadIdx.x; b < kBins; b += kThreads) h[b] = 0u;
    __syncthreads();
    int64_t lo, hi;
    seg_range(s, g, lo, hi);
    const uint32_t T = s.st[g].prefix[kKeyPasses];
    const int shift = 8 * (n_pass - 1 - pass);
    for_each_score(s.score, lo, hi, [&](int64_t e, float sc) {
        const bool tie = score_key(sc) == T;
        unsigned long long ix = tie ? (unsigned long long)entry_index(s, g, e, lo) : 0ull;
        if (n_pass < 8) ix &= (1ull << (8 * n_pass)) - 1ull;
        wave_hist_add(h, tie && (pass == 0 || (ix >> (shift + 8)) == prefix), (uint32_t)((ix >> shift) & 0xffull));
    });
    __syncthreads();
    uint32_t* gh = seg_hist(s, g, kKeyPasses + pass) + (blockIdx.x % s.copies) * kBins;
    for (int b = threadIdx.x; b < kBins; b += kThreads)
        if (h[b]) atomicAdd(&gh[b], h[b]);
}

__global__ __launch_bounds__(kThreads) void tie_take_kernel(Seg s, int n_pass)
{
    __shared__ uint32_t scan[kBins];
    const int g = blockIdx.y;
    if (seg_done(s, g)) return;
    const uint32_t k_eff = s.st[g].k_eff;
    if (k_eff == 0u || s.st[g].remaining[kKeyPasses] == 0u) return;
    // largest index (low bits) that makes the cut
    const unsigned long long cut = tie_step(s, g, n_pass, scan, false).prefix;
    int64_t lo, hi;
    seg_range(s, g, lo, hi);
    const uint32_t T = s.st[g].prefix[kKeyPasses];
    for_each_score(s.score, lo, hi, [&](int64_t e, float v) {
        const bool tie = score_key(v) == T;
        const int64_t ix = tie ? entry_index(s, g, e, lo) : 0;
        unsigned long long low = (unsigned long long)ix;
        if (n_pass < 8) low &= (1ull << (8 * n_pass)) - 1ull;
        const bool take = tie && low <= cut;
        const uint32_t pos = wave_claim(&s.st[g].n_sel, take);
        if (take && pos < k_eff) {
            s.sel_score[(size_t)g * s.k + pos] = v;
            s.sel_index[(size_t)g * s.k + pos] = ix;
        }
    });
}

// rank(e) = number of chosen entries of segment g preceding e, accumulated over slices of
// the chosen entries (grid.z) so that large k still fills the device (ranks start at zero).
__global__ __launch_bounds__(kThreads) void rank_kernel(Seg s, uint32_t slice)
{
    __shared__ uint32_t tk[kThreads];
    __shared__ int64_t ti[kThreads];
    const int g = blockIdx.y;
    if (seg_done(s, g)) return;
    const uint32_t k_eff = s.st[g].k_eff;
    if (blockIdx.x * kThreads >= k_eff) return;
    const uint32_t f_lo = blockIdx.z * slice;
    if (f_lo >= k_eff) return;
    const uint32_t f_hi = min(k_eff, f_lo + slice);
    const float* ss = s.sel_score + (size_t)g * s.k;
    const int64_t* si = s.sel_index + (size_t)g * s.k;
    const uint32_t e = blockIdx.x * kThreads + threadIdx.x;
    const bool mine = e < k_eff;
    const uint32_t key = mine ? score_key(ss[e]) : 0u;
    const int64_t ix = mine ? si[e] : 0;
    uint32_t rank = 0u;
    for (uint32_t base = f_lo; base < f_hi; base += kThreads) {
        __syncthreads();
        const uint32_t f = base + threadIdx.x;
        if (f < f_hi) { tk[threadIdx.x] = score_key(ss[f]); ti[threadIdx.x] = si[f]; }
        __syncthreads();
        const uint32_t m = min((uint32_t)kThreads, f_hi - base);
        // entry q precedes e: a larger key, or the same key and a smaller index
        if (mine)
            for (uint32_t q = 0; q < m; ++q) rank += (tk[q] > key) | ((tk[q] == key) & (ti[q] < ix)) ? 1u : 0u;
    }
    if (mine && rank) atomicAdd(&s.rank[(size_t)g * s.k + e], rank);
}

// out[g][rank(e)] = e; the slots past k_eff get (-inf, -1).
__global__ void scatter_kernel(Seg s, float* __restrict__ out_score, int64_t* __restrict__ out_index)
{
    const int g = blockIdx.y;
    if (seg_done(s, g)) return;
    const uint32_t k_eff = s.st[g].k_eff;
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (uint32_t)s.k) return;
    if (e >= k_eff) {
        out_score[(size_t)g * s.k + e] = -__builtin_huge_valf();
        out_index[(size_t)g * s.k + e] = -1;
        return;
    }
    const uint32_t r = s.rank[(size_t)g * s.k + e];
    if (r < k_eff) {
        out_score[(size_t)g * s.k + r] = s.sel_score[(size_t)g * s.k + e];
        out_index[(size_t)g * s.k + r] = s.sel_index[(size_t)g * s.k + e] + s.out_base;
    }
}

// ---------------------------------------------------------------- bucketed ordering (k > kRankDirect)

__global__ __launch_bounds__(kThreads) void winners_max_kernel(Seg s)
{
    const int g = blockIdx.y;
    if (seg_done(s, g)) return;
    const uint32_t k_eff = s.st[g].k_eff;
    const uint32_t e = blockIdx.x * kThreads + threadIdx.x;
    uint32_t key = e < k_eff ? score_key(s.sel_score[(size_t)g * s.k + e]) : 0u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(key, off, 64);
        key = o > key ? o : key;
    }
    if ((threadIdx.x & 63) == 0 && key) atomicMax(&s.st[g].kmax, key);
}

// Bucket of a chosen key: (kmax - key) scaled to the bucket count, so that a lower bucket holds
// larger keys only.
__device__ __forceinline__ uint32_t bucket_of(const Seg& s, int g, uint32_t key)
{
    const uint32_t kmax = s.st[g].kmax, range = kmax - s.st[g].prefix[kKeyPasses];
    const int bits = range ? 32 - __clz(range) : 0;
    const int shift = bits > s.bucket_log2 ? bits - s.bucket_log2 : 0;
    return (kmax - key) >> shift;
}

__global__ __launch_bounds__(kThreads) void bucket_count_kernel(Seg s)
{
    const int g = blockIdx.y;
    if (seg_done(s, g)) return;
    const uint32_t e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= s.st[g].k_eff) return;
    const uint32_t b = bucket_of(s, g, score_key(s.sel_score[(size_t)g * s.k + e]));
    atomicAdd(&s.bcnt[((size_t)g << s.bucket_log2) + b], 1u);
}

// Exclusive prefix of the bucket counts, one block per segment.
__global__ __launch_bounds__(1024) void bucket_scan_kernel(Seg s)
{
    __shared__ uint32_t part[1024];
    const int g = blockIdx.x;
    if (seg_done(s, g)) return;
    const int t = threadIdx.x;
    const uint32_t nb = 1u << s.bucket_log2;
    const uint32_t per = (nb + 1023) / 1024;
    const uint32_t* cnt = s.bcnt + ((size_t)g << s.bucket_log2);
    uint32_t* base = s.bbase + ((size_t)g << s.bucket_log2);
    uint32_t sum = 0u;
    for (uint32_t i = t * per; i < min(nb, (t + 1) * per); ++i) sum += cnt[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (uint32_t i = t * per; i < min(nb, (t + 1) * per); ++i) {
        base[i] = run;
        run += cnt[i];
    }
}

__global__ __launch_bounds__(kThreads) void bucket_scatter_kernel(Seg s)
{
    const int g = blockIdx.y;
    if (seg_done(s, g)) return;
    const uint32_t e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= s.st[g].k_eff) return;
    const float sc = s.sel_score[(size_t)g * s.k + e];
    const uint32_t key = score_key(sc);
    const size_t bb = ((size_t)g << s.bucket_log2) + bucket_of(s, g, key);
    const uint32_t pos = s.bbase[bb] + atomicAdd(&s.bfill[bb], 1u);
    s.tkey[(size_t)g * s.k + pos] = key;
    s.tscore[(size_t)g * s.k + pos] = sc;
    s.tindex[(size_t)g * s.k + pos] = s.sel_index[(size_t)g * s.k + e];
}

// out[g][rank] with rank = entries of the buckets before + entries of its own bucket that
// precede it; the slots past k_eff get (-inf, -1).
__global__ __launch_bounds__(kThreads) void bucket_rank_kernel(Seg s, float* __restrict__ out_score,
                                                               int64_t* __restrict__ out_index)
{
    const int g = blockIdx.y;
    if (seg_done(s, g)) return;
    const uint32_t k_eff = s.st[g].k_eff;
    const uint32_t p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= (uint32_t)s.k) return;
    if (p >= k_eff) {
        out_score[(size_t)g * s.k + p] = -__builtin_huge_valf();
        out_index[(size_t)g * s.k + p] = -1;
        return;
    }
    const uint32_t* tk = s.tkey + (size_t)g * s.k;
    const int64_t* ti = s.tindex + (size_t)g * s.k;
    const uint32_t key = tk[p];
    const int64_t ix = ti[p];
    const size_t bb = ((size_t)g << s.bucket_log2) + bucket_of(s, g, key);
    const uint32_t lo = s.bbase[bb], hi = lo + s.bcnt[bb];
    uint32_t r = lo;
    for (uint32_t q = lo; q < hi; ++q) r += (tk[q] > key) | ((tk[q] == key) & (ti[q] < ix)) ? 1u : 0u;
    if (r < k_eff) {
        out_score[(size_t)g * s.k + r] = s.tscore[(size_t)g * s.k + p];
        out_index[(size_t)g * s.k + r] = ix + s.out_base;
    }
}

// The whole selection for short segments (at most kSmallLen entries, k at most kSmallK) in
// one block per segment: the same radix select, compaction, tie resolution and rank ordering
// as the multi-block path, with the passes separated by block barriers instead of launches.
// Segments of at most kStageLen entries are first copied to LDS, so that the passes after the
// first read LDS instead of waiting on L2 for every few entries.
constexpr int kSmallThreads = 1024;
constexpr int64_t kSmallLen = 1 << 16;
constexpr int32_t kSmallK = 2048;
constexpr int kStageLen = 12288;

template <bool kStaged>
__global__ __launch_bounds__(kSmallThreads) void small_topk_kernel(Seg s, float* __restrict__ out_score,
                                                                   int64_t* __restrict__ out_index,
                                                                   int n_pass)
{
    __shared__ uint32_t sv[kStaged ? kStageLen : 1];
    __shared__ uint32_t h[kBins], scan[kBins];
    __shared__ uint32_t prefix, remaining, n_sel, passed, tie_all;
    __shared__ int digit;
    __shared__ unsigned long long iprefix;
    __shared__ float cs[kSmallK];
    __shared__ uint32_t ck[kSmallK];
    __shared__ int64_t ci[kSmallK];
    const int g = blockIdx.x;
    const int t = threadIdx.x;
    if (seg_done(s, g)) return;
    if (s.done_out) {
        // over a segment's candidates: they settle it when none was dropped for want of room
        // and at least k_eff of the full segment's entries were copied
        const uint32_t c = s.cand_cnt[g];
        const bool ok = (int64_t)c <= s.cand_cap && c >= s.cand_keff[g];
        if (t == 0) s.done_out[g] = ok ? 1u : 0u;
        if (!ok) return;
    }
    int64_t lo, hi;
    seg_range(s, g, lo, hi);
    const int64_t len = hi - lo;
    const uint32_t k_eff = (uint32_t)(len < (int64_t)s.k ? len : (int64_t)s.k);
    float* os = out_score + (size_t)g * s.k;
    int64_t* oi = out_index + (size_t)g * s.k;
    for (uint32_t e = k_eff + t; e < (uint32_t)s.k; e += kSmallThreads) {
        os[e] = -__builtin_huge_valf();
        oi[e] = -1;
    }
    if (k_eff == 0u) return;
    if (t == 0) {
        prefix = 0u;
        remaining = k_eff;
        n_sel = 0u;
        iprefix = 0ull;
        tie_all = 0u;
    }
    if constexpr (kStaged)
        for (int64_t e = t; e < len; e += kSmallThreads) sv[e] = score_key(s.score[lo + e]);
    // order-preserving key of entry e (absolute position); the staged copy when there is one
    auto key_at = [&](int64_t e) { return kStaged ? sv[e - lo] : score_key(s.score[e]); };
    // 1. key digits, most significant first
    for (int pass = 0; pass < 4; ++pass) {
        for (int b = t; b < kBins; b += kSmallThreads) h[b] = 0u;
        __syncthreads();
        const int shift = 24 - 8 * pass;
        const uint32_t pre = prefix;
        for (int64_t e = lo + t; e < hi; e += kSmallThreads) {
            const uint32_t key = key_at(e);
            wave_hist_add(h, pass == 0 || (key >> (shift + 8)) == pre, (key >> shift) & 0xffu);
        }
        __syncthreads();
        pick_digit(h, remaining, true, scan, &digit, &passed);
        if (t == 0) {
            remaining -= passed;
            prefix = (prefix << 8) | (uint32_t)digit;
            // h[digit] counts the entries equal to T after the last digit: when all of them
            // are needed, take them with the rest and skip the tie resolution
            if (pass == 3 && h[digit] == remaining) {
                tie_all = 1u;
                remaining = 0u;
            }
        }
        __syncthreads();
    }
    const uint32_t T = prefix;
    // 2. everything better than T (and T itself when all of its entries are taken)
    for (int64_t e = lo + t; e < hi; e += kSmallThreads) {
        const uint32_t key = key_at(e);
        const bool take = key > T || (tie_all != 0u && key == T);
        const uint32_t pos = wave_claim(&n_sel, take);
        if (take && pos < k_eff) {
            cs[pos] = s.score[e];
            ck[pos] = key;
            ci[pos] = entry_index(s, g, e, lo);
        }
    }
    // 3. the smallest indices among the entries equal to T
    for (int pass = 0; pass < n_pass && remaining > 0u; ++pass) {
        for (int b = t; b < kBins; b += kSmallThreads) h[b] = 0u;
        __syncthreads();
        const int shift = 8 * (n_pass - 1 - pass);
        const unsigned long long pre = iprefix;
        for (int64_t e = lo + t; e < hi; e += kSmallThreads) {
            const bool tie = key_at(e) == T;
            unsigned long long ix = tie ? (unsigned long long)entry_index(s, g, e, lo) : 0ull;
            if (n_pass < 8) ix &= (1ull << (8 * n_pass)) - 1ull;
            wave_hist_add(h, tie && (pass == 0 || (ix >> (shift + 8)) == pre),
                          (uint32_t)((ix >> shift) & 0xffull));
        }
        __syncthreads();
        pick_digit(h, remaining, false, scan, &digit, &passed);
        if (t == 0) {
            remaining -= passed;
            iprefix = (iprefix << 8) | (unsigned long long)digit;
        }
        __syncthreads();
    }
    if (remaining > 0u) {     // (remaining is block-uniform here)
        const unsigned long long cut = iprefix;
        for (int64_t e = lo + t; e < hi; e += kSmallThreads) {
            const bool tie = key_at(e) == T;
            const int64_t ix = tie ? entry_index(s, g, e, lo) : 0;
            unsigned long long low = (unsigned long long)ix;
            if (n_pass < 8) low &= (1ull << (8 * n_pass)) - 1ull;
            const bool take = tie && low <= cut;
            const uint32_t pos = wave_claim(&n_sel, take);
            if (take && pos < k_eff) {
                cs[pos] = s.score[e];
                ck[pos] = T;
                ci[pos] = ix;
            }
        }
    }
    __syncthreads();
    // 4. order by rank counting
    for (uint32_t e = t; e < k_eff; e += kSmallThreads) {
        const uint32_t key = ck[e];
        const int64_t ix = ci[e];
        uint32_t rank = 0u;
        for (uint32_t f = 0; f < k_eff; ++f) rank += (ck[f] > key) | ((ck[f] == key) & (ci[f] < ix)) ? 1u : 0u;
        if (rank < k_eff) {
            os[rank] = cs[e];
            oi[rank] = ix + s.out_base;
        }
    }
}

// ---------------------------------------------------------------- candidate pass

constexpr int64_t kCandCap = 32768;      // candidates kept per segment for k <= kSmallK (at least)
constexpr int kSampleRun = 64;           // consecutive entries per sampled run
constexpr int kSampleRuns = 512;         // runs per segment, first and last at its two ends
constexpr int kSample = kSampleRun * kSampleRuns;
constexpr int kGuessThreads = 512;
constexpr int kFallbackBlocks = 64;      // blocks per segment of the passes after the candidates

static_assert(kCandCap <= kSmallLen, "the one-block selection takes a segment's candidates");
static_assert(kSample % kGuessThreads == 0, "every thread takes the same number of samples");

// Room per segment: 32768 for the one-block selection, else 8 k (rounded up to 1024), so that
// the threshold aims at 2 k candidates.
int64_t cand_cap(int32_t k)
{
    const int64_t c = ((int64_t)8 * k + 1023) / 1024 * 1024;
    return k <= kSmallK || c < kCandCap ? kCandCap : c;
}

struct CandBufs {
    int64_t cap;        // cand_cap(k)
    uint32_t* T;        // [n_segs] threshold key
    uint32_t* cnt;      // [n_segs] entries with key >= T (also those beyond the buffer)
    uint32_t* keff;     // [n_segs] k_eff of the full segment
    uint32_t* done;     // [n_segs] settled by the candidates
    float* score;       // [n_segs][cap]
    int64_t* index;     // [n_segs][cap]
};

size_t cand_bytes(int32_t n_segs, int32_t k)
{
    const size_t ns = (size_t)(n_segs > 0 ? n_segs : 1);
    const size_t cap = (size_t)cand_cap(k);
    return 4 * align_up(sizeof(uint32_t) * ns) + align_up(sizeof(float) * cap * ns) +
           align_up(sizeof(int64_t) * cap * ns);
}

CandBufs carve_cand(void* base, int32_t n_segs, int32_t k)
{
    const size_t ns = (size_t)n_segs;
    char* p = (char*)base;
    CandBufs c;
    c.cap = cand_cap(k);
    c.T = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * ns);
    c.cnt = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * ns);
    c.keff = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * ns);
    c.done = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * ns);
    c.score = (float*)p;
    p += align_up(sizeof(float) * (size_t)c.cap * ns);
    c.index = (int64_t*)p;
    return c;
}

// One block per segment: T_g = the key of rank m (from the top) among kSample entries of the
// segment, in kSampleRuns runs of kSampleRun consecutive entries spread evenly from its first
// entry to its last; m is chosen so that about cap / 4 of the segment's entries are expected at
// or above T_g.  A segment of at most cap entries takes T_g = 0 (all of it).  Also clears the
// segment's candidate count and records its k_eff.
__global__ __launch_bounds__(kGuessThreads) void cand_guess_kernel(Seg s, int64_t cap, uint32_t* cand_T,
                                                                   uint32_t* cand_cnt, uint32_t* cand_keff)
{
    __shared__ uint32_t h[kBins], scan[kBins];
    __shared__ uint32_t prefix, remaining, passed;
    __shared__ int digit;
    const int g = blockIdx.x;
    const int t = threadIdx.x;
    int64_t lo, hi;
    seg_range(s, g, lo, hi);
    const int64_t len = hi - lo;
    if (t == 0) {
        cand_cnt[g] = 0u;
        cand_keff[g] = (uint32_t)(len < (int64_t)s.k ? len : (int64_t)s.k);
    }
    if (len <= cap) {
        if (t == 0) cand_T[g] = 0u;
        return;
    }
    // (len > cap, so m < kSample / 4)
    const uint32_t m = (uint32_t)max((int64_t)1, (int64_t)kSample * (cap / 4) / len);
    // run r starts at lo + r (len - kSampleRun) / (kSampleRuns - 1): inside the segment
    const int64_t gap = len - kSampleRun;
    if (t == 0) {
        prefix = 0u;
        remaining = m;
    }
    for (int pass = 0; pass < kKeyPasses; ++pass) {
        for (int b = t; b < kBins; b += kGuessThreads) h[b] = 0u;
        __syncthreads();
        const int shift = 24 - 8 * pass;
        const uint32_t pre = prefix;
        for (int e = t; e < kSample; e += kGuessThreads) {
            const int r = e / kSampleRun;
            const int64_t at = lo + (int64_t)r * gap / (kSampleRuns - 1) + (e - r * kSampleRun);
            const uint32_t key = score_key(s.score[at]);
            wave_hist_add(h, pass == 0 || (key >> (shift + 8)) == pre, (key >> shift) & 0xffu);
        }
        __syncthreads();
        pick_digit(h, remaining, true, scan, &digit, &passed);
        if (t == 0) {
            remaining -= passed;
            prefix = (prefix << 8) | (uint32_t)digit;
        }
        __syncthreads();
    }
    if (t == 0) cand_T[g] = prefix;
}

// Copies the entries with key >= T_g (score and index) to the segment's candidate buffer; the
// count goes on past the buffer's room (cap), so that an overfull buffer is seen.  As in split_kernel, each block
// gathers its entries in LDS and reserves their slots with one atomic (all blocks of a segment
// run at once, and an atomic per entry on the segment's one counter serializes at the L2).
__global__ __launch_bounds__(kThreads) void cand_compact_kernel(Seg s, int64_t cap, const uint32_t* __restrict__ cand_T,
                                                                uint32_t* cand_cnt, float* __restrict__ cs,
                                                                int64_t* __restrict__ ci)
{
    constexpr uint32_t kLCap = 1024;
    __shared__ float lsc[kLCap];
    __shared__ int64_t lix[kLCap];
    __shared__ uint32_t lcount, gbase;
    const int g = blockIdx.y;
    int64_t lo, hi;
    seg_range(s, g, lo, hi);
    const uint32_t T = cand_T[g];
    float* os = cs + (size_t)g * cap;
    int64_t* oi = ci + (size_t)g * cap;
    if (threadIdx.x == 0) lcount = 0u;
    __syncthreads();
    for_each_score(s.score, lo, hi, [&](int64_t e, float sc) {
        const bool take = score_key(sc) >= T;
        const uint32_t pos = wave_claim(&lcount, take);
        if (take) {
            const int64_t ix = entry_index(s, g, e, lo);
            if (pos < kLCap) {
                lsc[pos] = sc;
                lix[pos] = ix;
            } else {
                const uint32_t gp = atomicAdd(&cand_cnt[g], 1u);
                if ((int64_t)gp < cap) {
                    os[gp] = sc;
                    oi[gp] = ix;
                }
            }
        }
    });
    __syncthreads();
    const uint32_t n_local = min(lcount, kLCap);
    if (threadIdx.x == 0) gbase = n_local ? atomicAdd(&cand_cnt[g], n_local) : 0u;
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < n_local; q += kThreads) {
        const uint32_t pos = gbase + q;
        if ((int64_t)pos < cap) {
            os[pos] = lsc[q];
            oi[pos] = lix[q];
        }
    }
}

// Whether each segment's candidates settle it: none dropped for want of room, and at least
// k_eff of the full segment's entries copied.
__global__ void cand_done_kernel(const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ keff, int64_t cap,
                                 uint32_t* __restrict__ done, int n_segs)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n_segs) done[g] = ((int64_t)cnt[g] <= cap && cnt[g] >= keff[g]) ? 1u : 0u;
}

// The selection over s's segments (at most max_len entries each): one block per segment for
// short ones and small k, else the radix passes on `blocks` blocks per segment.
void run_passes(const Seg& s, int64_t max_len, int blocks, int n_pass, float* out_score, int64_t* out_index,
                hipStream_t st)
{
    if (max_len <= kSmallLen && s.k <= kSmallK) {
        if (max_len <= kStageLen)
            hipLaunchKernelGGL(small_topk_kernel<true>, dim3(s.n_segs), dim3(kSmallThreads), 0, st, s,
                               out_score, out_index, n_pass);
        else
            hipLaunchKernelGGL(small_topk_kernel<false>, dim3(s.n_segs), dim3(kSmallThreads), 0, st, s,
                               out_score, out_index, n_pass);
        return;
    }
    const dim3 grid(blocks, s.n_segs);
    // 8 + n_pass launches: the digit picks run at the head of the next pass's kernel
    const uint32_t kb = (uint32_t)((s.k + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(init_kernel, dim3(kb, s.n_segs), dim3(kThreads), 0, st, s);
    for (int pass = 0; pass < kKeyPasses; ++pass)
        hipLaunchKernelGGL(key_hist_kernel, grid, dim3(kThreads), 0, st, s, pass);
    hipLaunchKernelGGL(split_kernel, grid, dim3(kThreads), 0, st, s);
    // The tie passes keep the full grid: the stage-1 maps hold exact ties (templates whose tracks
    // pick the same bins), so some lists resolve ties, and a list's tie pass on few blocks is the
    // launch's tail (cut to about 4096 blocks in all, the batched step's lists took 10 ms more).
    for (int pass = 0; pass < n_pass; ++pass)
        hipLaunchKernelGGL(tie_hist_kernel, grid, dim3(kThreads), 0, st, s, pass, n_pass);
    hipLaunchKernelGGL(tie_take_kernel, grid, dim3(kThreads), 0, st, s, n_pass);
    if (s.bcnt) {
        // grouped by key bucket, then ranks within the buckets
        hipLaunchKernelGGL(winners_max_kernel, dim3(kb, s.n_segs), dim3(kThreads), 0, st, s);
        hipLaunchKernelGGL(bucket_count_kernel, dim3(kb, s.n_segs), dim3(kThreads), 0, st, s);
        hipLaunchKernelGGL(bucket_scan_kernel, dim3(s.n_segs), dim3(1024), 0, st, s);
        hipLaunchKernelGGL(bucket_scatter_kernel, dim3(kb, s.n_segs), dim3(kThreads), 0, st, s);
        hipLaunchKernelGGL(bucket_rank_kernel, dim3(kb, s.n_segs), dim3(kThreads), 0, st, s, out_score,
                           out_index);
        return;
    }
    // rank counting: k x k comparisons spread over (k/256) x slices blocks
    const uint32_t n_slices = kb < 64 ? kb : 64;
    const uint32_t slice = (uint32_t)((s.k + n_slices - 1) / n_slices);
    hipLaunchKernelGGL(rank_kernel, dim3(kb, s.n_segs, n_slices), dim3(kThreads), 0, st, s, slice);
    hipLaunchKernelGGL(scatter_kernel, dim3(kb, s.n_segs), dim3(kThreads), 0, st, s, out_score, out_index);
}

int blocks_for(int64_t len)
{
    const int64_t b = (len + kThreads - 1) / kThreads;
    return (int)(b > kMaxBlocksPerSeg ? kMaxBlocksPerSeg : (b < 1 ? 1 : b));
}

int topk_launch(Seg s, int64_t max_len, float* out_score, int64_t* out_index, hipStream_t st,
                const CandBufs* cb = nullptr)
{
    const int bps = blocks_for(max_len);
    if (s.n_segs > 65535) return fail_inval("more than 65535 segments");
    // index digits to resolve: 64 bits for explicit indices, the position bits otherwise
    int bits = 64;
    if (!s.index) {
        bits = 1;
        while (bits < 63 && ((int64_t)1 << bits) < max_len) ++bits;
    }
    const int n_pass = (bits + 7) / 8;
    s.idx_bits = bits;
    if (!cb) {
        run_passes(s, max_len, bps, n_pass, out_score, out_index, st);
        return check_launch("bsh_topk");
    }
    hipLaunchKernelGGL(cand_guess_kernel, dim3(s.n_segs), dim3(kGuessThreads), 0, st, s, cb->cap, cb->T, cb->cnt,
                       cb->keff);
    hipLaunchKernelGGL(cand_compact_kernel, dim3(bps, s.n_segs), dim3(kThreads), 0, st, s, cb->cap, cb->T, cb->cnt,
                       cb->score, cb->index);
    // the selection over each segment's candidates (explicit indices: those of the full segment,
    // whose implicit ones were formed in the copy)
    Seg f = s;
    f.score = cb->score;
    f.index = cb->index;
    f.off = nullptr;
    f.cand_cnt = cb->cnt;
    f.cand_cap = cb->cap;
    f.cand_keff = cb->keff;
    if (s.k <= kSmallK) {
        // one block per segment, which also records which segments its candidates settle
        f.done_out = cb->done;
        hipLaunchKernelGGL(small_topk_kernel<false>, dim3(s.n_segs), dim3(kSmallThreads), 0, st, f, out_score,
                           out_index, n_pass);
    } else {
        hipLaunchKernelGGL(cand_done_kernel, dim3((s.n_segs + 255) / 256), dim3(256), 0, st, cb->cnt, cb->keff,
                           cb->cap, cb->done, s.n_segs);
        f.done = cb->done;
        f.done_skip = 0u;
        run_passes(f, cb->cap, blocks_for(cb->cap), n_pass, out_score, out_index, st);
    }
    // the segments the candidates did not settle: the passes over the whole segments, which
    // return at once for the others, on fewer blocks per segment
    s.done = cb->done;
    s.done_skip = 1u;
    run_passes(s, max_len, bps < kFallbackBlocks ? bps : kFallbackBlocks, n_pass, out_score, out_index, st);
    return check_launch("bsh_topk");
}

}  // namespace

namespace bsh {

size_t topk_workspace_bytes(int32_t n_segs, int32_t k) { return workspace_bytes(n_segs, k); }

size_t topk_candidate_workspace_bytes(int32_t n_segs, int32_t k)
{
    return workspace_bytes(n_segs, k) + (n_segs >= 2 ? cand_bytes(n_segs, k) : 0);
}

// Segmented top-k for library-internal callers (the batched plan); offsets on the device,
// the longest segment given by the host.  NULL offsets: one segment [0, max_len).
int topk_segmented(const float* score, const int64_t* index, const int64_t* offsets, int32_t n_segs,
                   int64_t max_len, int32_t shift, int32_t k, float* out_score, int64_t* out_index,
                   void* ws, size_t ws_bytes, hipStream_t stream, int64_t index_base)
{
    if (n_segs < 1 || k < 1) return fail_inval("n_segs and k must be >= 1");
    if (ws_bytes < workspace_bytes(n_segs, k)) {
        set_error("workspace %zu < %zu bytes", ws_bytes, workspace_bytes(n_segs, k));
        return BSH_ENOMEM;
    }
    if (max_len >= (int64_t)0xffffffff) return fail_inval("segments must be shorter than 2^32 - 1");
    if (!offsets && n_segs != 1) return fail_inval("NULL offsets need exactly one segment");
    Seg s;
    std::memset(&s, 0, sizeof(s));
    s.score = score;
    s.index = index;
    s.off = offsets;
    s.n_single = max_len;
    s.n_segs = n_segs;
    s.shift = shift;
    s.k = k;
    s.out_base = index ? 0 : index_base;
    carve(ws, s);
    // the candidate pass when there are several segments longer than its buffers and the
    // workspace has room for them
    const size_t base = workspace_bytes(n_segs, k);
    if (n_segs >= 2 && max_len > cand_cap(k) && ws_bytes >= base + cand_bytes(n_segs, k)) {
        const CandBufs cb = carve_cand((char*)ws + base, n_segs, k);
        return topk_launch(s, max_len, out_score, out_index, stream, &cb);
    }
    return topk_launch(s, max_len, out_score, out_index, stream);
}

}  // namespace bsh

extern "C" size_t bsh_topk_workspace(int64_t n, int32_t k)
{
    if (n < 0 || k < 0) return 0;
    return workspace_bytes(1, k > 0 ? k : 1);
}

extern "C" int bsh_topk(const float* score, const int64_t* index, int64_t n, int32_t k,
                        float* out_score, int64_t* out_index, void* ws, size_t ws_bytes,
                        bsh_stream stream)
{
    clear_error();
    if (n < 0 || k < 0) return fail_inval("n or k negative");
    if (n >= (int64_t)0xffffffff) return fail_inval("n must be below 2^32 - 1");
    if (k == 0) return BSH_OK;
    if (!out_score || !out_index) return fail_inval("NULL output");
    if (n > 0 && !score) return fail_inval("score is NULL");
    if (!ws) return fail_inval("workspace is NULL");
    const size_t need = bsh_topk_workspace(n, k);
    if (ws_bytes < need) {
        set_error("workspace %zu < %zu bytes", ws_bytes, need);
        return BSH_ENOMEM;
    }
    return bsh::topk_segmented(score, index, nullptr, 1, n, 0, k, out_score, out_index, ws, ws_bytes,
                               (hipStream_t)stream);
}

extern "C" size_t bsh_topk_segmented_workspace(int32_t n_segs, int32_t k)
{
    if (n_segs < 1 || k < 1) return 0;
    return workspace_bytes(n_segs, k);
}

extern "C" size_t bsh_topk_segmented_candidate_workspace(int32_t n_segs, int32_t k)
{
    if (n_segs < 1 || k < 1) return 0;
    return bsh::topk_candidate_workspace_bytes(n_segs, k);
}

extern "C" int bsh_topk_segmented(const float* score, const int64_t* index, const int64_t* offsets,
                                  const int64_t* offsets_host, int32_t n_segs, int32_t k,
                                  int32_t index_shift, float* out_score, int64_t* out_index,
                                  void* ws, size_t ws_bytes, bsh_stream stream)
{
    clear_error();
    if (n_segs < 1 || k < 1) return fail_inval("n_segs and k must be >= 1");
    if (!score || !offsets || !offsets_host || !out_score || !out_index || !ws)
        return fail_inval("NULL pointer");
    if (index_shift < 0 || index_shift > 62) return fail_inval("index_shift out of 0..62");
    int64_t max_len = 0;
    if (offsets_host[0] < 0) return fail_inval("offsets[0] < 0");
    for (int32_t g = 0; g < n_segs; ++g) {
        const int64_t len = offsets_host[g + 1] - offsets_host[g];
        if (len < 0) return fail_inval("offsets not monotone");
        if (len > max_len) max_len = len;
    }
    return bsh::topk_segmented(score, index, offsets, n_segs, max_len, index_shift, k, out_score,
                               out_index, ws, ws_bytes, (hipStream_t)stream);
}

// ---------------------------------------------------------------- top-k without allocation
//
// For callers that cannot allocate (code under graph capture, serving loops): the workspace is
// a file-scope device array of fixed size, one copy per GPU.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol); it passes the
// device address that hipGetSymbolAddress gives, taken once per device with that device current.
namespace {

constexpr size_t kScratchBytes = (size_t)8 << 20;
constexpr int kScratchDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// The scratch array's device address on the current device (NULL and an error on failure).
void* scratch_on_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) {
        set_error("no usable current device for the scratch workspace");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" size_t bsh_topk_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" int bsh_topk_noalloc(const float* score, const int64_t* index, int64_t n, int32_t k,
                                float* out_score, int64_t* out_index, bsh_stream stream)
{
    clear_error();
    if (n < 0 || k < 0) return fail_inval("n or k negative");
    if (n >= (int64_t)0xffffffff) return fail_inval("n must be below 2^32 - 1");
    if (k == 0) return BSH_OK;
    if (!out_score || !out_index) return fail_inval("NULL output");
    if (n > 0 && !score) return fail_inval("score is NULL");
    const size_t need = workspace_bytes(1, k);
    if (need > kScratchBytes) {
        set_error("k = %d needs a %zu-byte workspace, above the %zu-byte static scratch of bsh_topk_noalloc",
                  (int)k, need, kScratchBytes);
        return BSH_ENOMEM;
    }
    void* ws = scratch_on_current_device();
    if (!ws) return BSH_EHIP;
    return bsh::topk_segmented(score, index, nullptr, 1, n, 0, k, out_score, out_index, ws, kScratchBytes,
                               (hipStream_t)stream);
}
