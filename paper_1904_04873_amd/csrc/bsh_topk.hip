// Exact top-k under the total order (score descending, index ascending): the per-band
// top-lists of Sec. IV.C (N_C candidates out of stage 1, N_CF out of stage 2).
//
// 1. Radix select on the 32-bit order-preserving key of the score: four 8-bit digit passes
//    (block histograms in LDS, one global histogram, a one-block digit pick) find the key T
//    of the k-th best score, the number of scores strictly better, and how many ties at T
//    are still needed.
// 2. One compaction pass writes every entry with key > T to the output pool and the
//    indices of entries with key == T to a tie buffer.
// 3. Ties are resolved by index: a radix select over the 64-bit indices of the tie buffer
//    finds the largest index that still makes the cut, and a second compaction appends the
//    chosen ties.
// 4. The k chosen entries are ordered by rank counting (each entry counts the entries that
//    precede it), which is exact, deterministic and independent of the arrival order.
// Everything stays on the stream: no host synchronisation, counts live in the workspace.
#include "bsh_internal.h"

namespace {

using namespace bsh;

constexpr int kThreads = 256;
constexpr int kBins = 256;

struct State {
    uint32_t prefix;         // key digits fixed so far
    uint32_t remaining;      // entries still to take at the current prefix
    uint32_t n_gt;           // entries with key > T (after the key passes)
    uint32_t n_tie;          // tie-buffer fill
    uint32_t n_sel;          // output-pool fill
    uint32_t pad;
    unsigned long long iprefix;    // index digits fixed so far (tie resolution)
    uint32_t iremaining;
    uint32_t n_lt;
};

struct Work {
    State* st;
    uint32_t* hist;          // [kBins]
    int64_t* tie;            // [n]
    float* sel_score;        // [k]
    int64_t* sel_index;      // [k]
};

__host__ __device__ inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

Work carve(void* ws, int64_t n, int32_t k)
{
    char* p = (char*)ws;
    Work w;
    w.st = (State*)p;
    p += align_up(sizeof(State));
    w.hist = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * kBins);
    w.tie = (int64_t*)p;
    p += align_up(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    w.sel_score = (float*)p;
    p += align_up(sizeof(float) * (size_t)k);
    w.sel_index = (int64_t*)p;
    return w;
}

size_t workspace_bytes(int64_t n, int32_t k)
{
    return align_up(sizeof(State)) + align_up(sizeof(uint32_t) * kBins) +
           align_up(sizeof(int64_t) * (size_t)(n > 0 ? n : 1)) + align_up(sizeof(float) * (size_t)k) +
           align_up(sizeof(int64_t) * (size_t)k);
}

// Order-preserving map float -> uint32 (larger float -> larger key); -0 is folded onto +0.
__device__ __forceinline__ uint32_t score_key(float f)
{
    uint32_t u = __float_as_uint(f);
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_score(uint32_t k)
{
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

__device__ __forceinline__ int64_t entry_index(const int64_t* index, int64_t e)
{
    return index ? index[e] : e;
}

__global__ void init_kernel(Work w, uint32_t k_eff)
{
    const int t = threadIdx.x;
    if (t == 0) {
        w.st->prefix = 0u;
        w.st->remaining = k_eff;
        w.st->n_gt = 0u;
        w.st->n_tie = 0u;
        w.st->n_sel = 0u;
        w.st->iprefix = 0ull;
        w.st->iremaining = 0u;
        w.st->n_lt = 0u;
    }
    for (int b = t; b < kBins; b += blockDim.x) w.hist[b] = 0u;
}

// Histogram of key digit `pass` (0 = most significant byte) over entries matching the prefix.
__global__ __launch_bounds__(kThreads) void key_hist_kernel(const float* __restrict__ score,
                                                            int64_t n, Work w, int pass)
{
    __shared__ uint32_t h[kBins];
    for (int b = threadIdx.x; b < kBins; b += kThreads) h[b] = 0u;
    __syncthreads();
    const uint32_t prefix = w.st->prefix;
    const int shift = 24 - 8 * pass;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kThreads) {
        const uint32_t key = score_key(score[e]);
        if (pass == 0 || (key >> (shift + 8)) == prefix) atomicAdd(&h[(key >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += kThreads)
        if (h[b]) atomicAdd(&w.hist[b], h[b]);
}

// Pick the digit holding the remaining-th best entry; entries with larger digits are taken.
__global__ void key_pick_kernel(Work w)
{
    __shared__ uint32_t h[kBins];
    const int t = threadIdx.x;   // kBins threads
    h[t] = w.hist[t];
    __syncthreads();
    if (t == 0) {
        uint32_t rem = w.st->remaining;
        uint32_t above = 0u;
        int d = kBins - 1;
        for (; d > 0; --d) {
            if (above + h[d] >= rem) break;
            above += h[d];
        }
        w.st->n_gt += above;
        w.st->remaining = rem - above;
        w.st->prefix = (w.st->prefix << 8) | (uint32_t)d;
    }
    __syncthreads();
    w.hist[t] = 0u;
}

__global__ __launch_bounds__(kThreads) void split_kernel(const float* __restrict__ score,
                                                         const int64_t* __restrict__ index,
                                                         int64_t n, Work w, uint32_t k_cap)
{
    const uint32_t T = w.st->prefix;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kThreads) {
        const float sc = score[e];
        const uint32_t key = score_key(sc);
        if (key > T) {
            const uint32_t pos = atomicAdd(&w.st->n_sel, 1u);
            if (pos < k_cap) {
                w.sel_score[pos] = sc;
                w.sel_index[pos] = entry_index(index, e);
            }
        } else if (key == T) {
            const uint32_t pos = atomicAdd(&w.st->n_tie, 1u);
            w.tie[pos] = entry_index(index, e);
        }
    }
}

__global__ void tie_init_kernel(Work w)
{
    if (threadIdx.x == 0) {
        w.st->iprefix = 0ull;
        w.st->iremaining = w.st->remaining;
        w.st->n_lt = 0u;
    }
    for (int b = threadIdx.x; b < kBins; b += blockDim.x) w.hist[b] = 0u;
}

// Histogram of index digit `pass` (0 = most significant byte of the 64-bit index).
__global__ __launch_bounds__(kThreads) void tie_hist_kernel(Work w, int pass)
{
    __shared__ uint32_t h[kBins];
    for (int b = threadIdx.x; b < kBins; b += kThreads) h[b] = 0u;
    __syncthreads();
    const uint32_t nt = w.st->n_tie;
    const unsigned long long prefix = w.st->iprefix;
    const int shift = 56 - 8 * pass;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < (int64_t)nt;
         e += (int64_t)gridDim.x * kThreads) {
        const unsigned long long ix = (unsigned long long)w.tie[e];
        if (pass == 0 || (ix >> (shift + 8)) == prefix) atomicAdd(&h[(ix >> shift) & 0xffull], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += kThreads)
        if (h[b]) atomicAdd(&w.hist[b], h[b]);
}

// Smallest indices win: take digits from the low end.
__global__ void tie_pick_kernel(Work w)
{
    __shared__ uint32_t h[kBins];
    const int t = threadIdx.x;
    h[t] = w.hist[t];
    __syncthreads();
    if (t == 0) {
        uint32_t rem = w.st->iremaining;
        uint32_t below = 0u;
        int d = 0;
        for (; d < kBins - 1; ++d) {
            if (below + h[d] >= rem) break;
            below += h[d];
        }
        w.st->n_lt += below;
        w.st->iremaining = rem - below;
        w.st->iprefix = (w.st->iprefix << 8) | (unsigned long long)d;
    }
    __syncthreads();
    w.hist[t] = 0u;
}

__global__ __launch_bounds__(kThreads) void tie_take_kernel(Work w, uint32_t k_cap)
{
    const uint32_t nt = w.st->n_tie;
    const uint32_t need = w.st->remaining;
    if (need == 0u) return;
    const unsigned long long cut = w.st->iprefix;    // last index that makes the cut
    const float sc = key_score(w.st->prefix);
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < (int64_t)nt;
         e += (int64_t)gridDim.x * kThreads) {
        const int64_t ix = w.tie[e];
        if ((unsigned long long)ix <= cut) {
            const uint32_t pos = atomicAdd(&w.st->n_sel, 1u);
            if (pos < k_cap) {
                w.sel_score[pos] = sc;
                w.sel_index[pos] = ix;
            }
        }
    }
}

__device__ __forceinline__ bool precedes(float sa, int64_t ia, float sb, int64_t ib)
{
    const uint32_t ka = score_key(sa), kb = score_key(sb);
    return ka > kb || (ka == kb && ia < ib);
}

// out[rank(e)] = e, rank(e) = number of chosen entries preceding e.
__global__ __launch_bounds__(kThreads) void rank_kernel(Work w, uint32_t k_eff,
                                                        float* __restrict__ out_score,
                                                        int64_t* __restrict__ out_index)
{
    __shared__ float ts[kThreads];
    __shared__ int64_t ti[kThreads];
    const uint32_t e = blockIdx.x * kThreads + threadIdx.x;
    const bool mine = e < k_eff;
    const float s = mine ? w.sel_score[e] : 0.f;
    const int64_t ix = mine ? w.sel_index[e] : 0;
    uint32_t rank = 0u;
    for (uint32_t base = 0; base < k_eff; base += kThreads) {
        __syncthreads();
        const uint32_t f = base + threadIdx.x;
        if (f < k_eff) { ts[threadIdx.x] = w.sel_score[f]; ti[threadIdx.x] = w.sel_index[f]; }
        __syncthreads();
        const uint32_t m = min((uint32_t)kThreads, k_eff - base);
        if (mine)
            for (uint32_t q = 0; q < m; ++q) rank += precedes(ts[q], ti[q], s, ix) ? 1u : 0u;
    }
    if (mine && rank < k_eff) {
        out_score[rank] = s;
        out_index[rank] = ix;
    }
}

__global__ void fill_tail_kernel(uint32_t k_eff, int32_t k, float* out_score, int64_t* out_index)
{
    const uint32_t e = k_eff + blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (uint32_t)k) {
        out_score[e] = -__builtin_huge_valf();
        out_index[e] = -1;
    }
}

}  // namespace

extern "C" size_t bsh_topk_workspace(int64_t n, int32_t k)
{
    if (n < 0 || k < 0) return 0;
    return workspace_bytes(n, k);
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
    if (ws_bytes < workspace_bytes(n, k)) {
        set_error("workspace %zu < %zu bytes", ws_bytes, workspace_bytes(n, k));
        return BSH_ENOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    const uint32_t k_eff = (uint32_t)(n < (int64_t)k ? n : (int64_t)k);
    Work w = carve(ws, n, k);
    int blocks = (int)((n + kThreads - 1) / kThreads);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;

    if (k_eff > 0) {
        hipLaunchKernelGGL(init_kernel, dim3(1), dim3(kBins), 0, s, w, k_eff);
        for (int pass = 0; pass < 4; ++pass) {
            hipLaunchKernelGGL(key_hist_kernel, dim3(blocks), dim3(kThreads), 0, s, score, n, w, pass);
            hipLaunchKernelGGL(key_pick_kernel, dim3(1), dim3(kBins), 0, s, w);
        }
        hipLaunchKernelGGL(split_kernel, dim3(blocks), dim3(kThreads), 0, s, score, index, n, w, k_eff);
        hipLaunchKernelGGL(tie_init_kernel, dim3(1), dim3(kBins), 0, s, w);
        for (int pass = 0; pass < 8; ++pass) {
            hipLaunchKernelGGL(tie_hist_kernel, dim3(blocks), dim3(kThreads), 0, s, w, pass);
            hipLaunchKernelGGL(tie_pick_kernel, dim3(1), dim3(kBins), 0, s, w);
        }
        hipLaunchKernelGGL(tie_take_kernel, dim3(blocks), dim3(kThreads), 0, s, w, k_eff);
        hipLaunchKernelGGL(rank_kernel, dim3((k_eff + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                           w, k_eff, out_score, out_index);
    }
    if ((uint32_t)k > k_eff)
        hipLaunchKernelGGL(fill_tail_kernel, dim3((k - k_eff + 255) / 256), dim3(256), 0, s, k_eff, k,
                           out_score, out_index);
    return check_launch("bsh_topk");
}
