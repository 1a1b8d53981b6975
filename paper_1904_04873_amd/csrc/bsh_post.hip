// Post-processing of top-lists (Sec. V.E): template rows, significances, coincidences between
// two lists, clustering and significance-weighted centroids, on the device.
//
// Distances follow eq:postdist with the sky resolution of Sec. IV.C and the binary resolutions
// of eq:binaryres, each point-dependent resolution averaged over the two templates.  The window
// and cut decisions compare d^2 with the squared window in FP64 under one fixed evaluation order
// (the library is built without contraction):
//
//   k      = (pi Tc) f                          q_f = (f_b - f_a) Tc
//   dTheta = 1 / (((v Tc) f) P_F)               q_z = (z_b - z_a) / ((dz_a + dz_b) 0.5)
//   da_p   = sqrt(6 m_a) / (k W)                d^2 = ((((q_f^2 + q_x^2) + q_y^2) + q_a^2)
//   dW     = sqrt(72 m_W) / (((k a_p) W) T_obs)        + q_W^2) + q_t^2
//   dt_asc = sqrt(6 m_t) / (((k a_p) W) W)
//
// Clusters are the connected components of the "d < window" graph (templates closer than the
// window share a cluster, and clusters sharing a template merge).  They are found with a
// lock-free union-find over all pairs: a root is only ever hooked under a smaller root, so every
// tree's root is its smallest member and the labels do not depend on the order of the hooks.
#include "bsh_internal.h"

namespace bsh {
namespace {

constexpr double kPi = 3.141592653589793;
constexpr int kPostThreads = 256;

struct PostConst {
    double t_coh, pi_tc, v_tc, pf, t_obs, ca, cw, ct;
};

PostConst post_const(const bsh_post_params* pp)
{
    PostConst c;
    c.t_coh = pp->t_coh;
    c.pi_tc = kPi * pp->t_coh;
    c.v_tc = pp->v_over_c * pp->t_coh;
    c.pf = pp->pixel_factor;
    c.t_obs = pp->t_obs;
    c.ca = std::sqrt(6.0 * pp->m_a);
    c.cw = std::sqrt(72.0 * pp->m_omega);
    c.ct = std::sqrt(6.0 * pp->m_t);
    return c;
}

int check_post(const bsh_post_params* pp)
{
    if (!pp) return fail_inval("post-processing parameters are NULL");
    const double v[7] = {pp->t_coh, pp->t_obs, pp->m_a, pp->m_omega, pp->m_t, pp->pixel_factor,
                         pp->v_over_c};
    for (double x : v)
        if (!(std::isfinite(x) && x > 0.0))
            return fail_inval("post-processing parameters must be finite and positive");
    return BSH_OK;
}

// A template row with its four point-dependent resolutions.
struct PRow {
    double f, x, y, a, w, t;
    double rth, ra, rw, rt;
};

__device__ __forceinline__ PRow load_row(const double* r, const PostConst& c)
{
    PRow p;
    p.f = r[0];
    p.x = r[1];
    p.y = r[2];
    p.a = r[3];
    p.w = r[4];
    p.t = r[5];
    const double k = c.pi_tc * p.f;
    p.rth = 1.0 / ((c.v_tc * p.f) * c.pf);
    p.ra = c.ca / (k * p.w);
    const double kaw = (k * p.a) * p.w;
    p.rw = c.cw / (kaw * c.t_obs);
    p.rt = c.ct / (kaw * p.w);
    return p;
}

__device__ __forceinline__ double dist2(const PRow& a, const PRow& b, const PostConst& c)
{
    const double qf = (b.f - a.f) * c.t_coh;
    const double qx = (b.x - a.x) / ((a.rth + b.rth) * 0.5);
    const double qy = (b.y - a.y) / ((a.rth + b.rth) * 0.5);
    const double qa = (b.a - a.a) / ((a.ra + b.ra) * 0.5);
    const double qw = (b.w - a.w) / ((a.rw + b.rw) * 0.5);
    const double qt = (b.t - a.t) / ((a.rt + b.rt) * 0.5);
    double s = qf * qf + qx * qx;
    s = s + qy * qy;
    s = s + qa * qa;
    s = s + qw * qw;
    return s + qt * qt;
}

// ---------------------------------------------------------------- rows and significances

__global__ void rows_kernel(const double* sky, const int32_t* cand_sky, const double* cand, int64_t n,
                            double t_coh, double* rows)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* c = cand + 4 * i;
    const double* s = sky + 3 * (int64_t)cand_sky[i];
    double* r = rows + 6 * i;
    r[0] = c[0] / t_coh;
    r[1] = s[0];
    r[2] = s[1];
    r[3] = c[1];
    r[4] = kTwoPi / c[2];
    r[5] = c[3];
}

// W1 = sum w, W2 = sum w^2 over the segments (every block recomputes them: n_seg is small).
__global__ void significance_kernel(const float* score, int64_t n, const float* w, int64_t n_seg,
                                    int32_t kind, double p0, double* sig)
{
    __shared__ double s1[kPostThreads], s2[kPostThreads];
    double a = 0.0, b = 0.0;
    for (int64_t j = threadIdx.x; j < n_seg; j += blockDim.x) {
        const double x = (double)w[j];
        a += x;
        b += x * x;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s1[threadIdx.x] += s1[threadIdx.x + h];
            s2[threadIdx.x] += s2[threadIdx.x + h];
        }
        __syncthreads();
    }
    const double W1 = s1[0], W2 = s2[0];
    const double mean = kind == 0 ? p0 * W1 : W1;
    const double sd = kind == 0 ? sqrt(p0 * (1.0 - p0) * W2) : sqrt(W2);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        sig[i] = ((double)score[i] - mean) / sd;
}

// ---------------------------------------------------------------- coincidences

__global__ void zero_i64_kernel(int64_t* p) { *p = 0; }

// Matches of list-a row i among the list-b rows, in j order: one block per row.
template <bool kWrite>
__global__ void coinc_kernel(PostConst c, const double* ra, const double* sa, const double* rb,
                             const double* sb, int64_t nb, double w2, int64_t* count,
                             const int64_t* offset, int64_t cap, int64_t* pairs, double* rows_out,
                             double* sig_out)
{
    __shared__ int32_t wave_n[kPostThreads / 64];
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const PRow a = load_row(ra + 6 * i, c);
    int64_t running = kWrite ? offset[i] : 0;
    for (int64_t j0 = 0; j0 < nb; j0 += blockDim.x) {
        const int64_t j = j0 + threadIdx.x;
        bool hit = false;
        PRow b;
        if (j < nb) {
            b = load_row(rb + 6 * j, c);
            hit = dist2(a, b, c) < w2;
        }
        const uint64_t m = __ballot(hit);
        if (lane == 0) wave_n[wave] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            before += q < wave ? wave_n[q] : 0;
            total += wave_n[q];
        }
        if (kWrite && hit) {
            const int64_t pos = running + before + __popcll(m & ((1ull << lane) - 1ull));
            if (pos < cap) {
                const double wa = sa[i], wb = sb[j];
                const double ws = wa + wb;
                pairs[2 * pos] = i;
                pairs[2 * pos + 1] = j;
                const double* xa = ra + 6 * i;
                const double* xb = rb + 6 * j;
                for (int k = 0; k < 6; ++k) rows_out[6 * pos + k] = (wa * xa[k] + wb * xb[k]) / ws;
                sig_out[pos] = ws;
            }
        }
        running += total;
        __syncthreads();
    }
    if (!kWrite && threadIdx.x == 0) count[i] = running;
}

// Exclusive scan of n counts (one block), total into offset[n] and *n_total.
__global__ void scan_kernel(const int64_t* count, int64_t n, int64_t* offset, int64_t* n_total)
{
    __shared__ int64_t part[kPostThreads];
    const int t = threadIdx.x;
    const int64_t per = (n + blockDim.x - 1) / blockDim.x;
    const int64_t lo = min(n, t * per), hi = min(n, lo + per);
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += count[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int q = 0; q < (int)blockDim.x; ++q) {
            const int64_t v = part[q];
            part[q] = run;
            run += v;
        }
        offset[n] = run;
        *n_total = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int64_t i = lo; i < hi; ++i) {
        offset[i] = run;
        run += count[i];
    }
}

// ---------------------------------------------------------------- clustering

__device__ __forceinline__ int32_t ld(const int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st(int32_t* p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving.  Parents only ever point to smaller indices, so the walk ends.
__device__ int32_t find_root(int32_t* parent, int32_t x)
{
    int32_t p = ld(parent + x);
    while (p != x) {
        const int32_t g = ld(parent + p);
        if (g != p) st(parent + x, g);
        x = p;
        p = g;
    }
    return x;
}

// Join the trees of a and b by hooking the larger root under the smaller one.  A failed
// compare-and-swap means another thread hooked that root first; at most n - 1 hooks ever succeed,
// so the loop ends.
__device__ void unite(int32_t* parent, int32_t a, int32_t b)
{
    while (true) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b) return;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(parent + b, b, a) == b) return;
    }
}

__global__ void iota_kernel(int32_t* parent, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) parent[i] = (int32_t)i;
}

// Union-find on a tile's nodes in LDS (same hooking rule as the global one: the larger root
// under the smaller, so every walk ends).
__device__ __forceinline__ int32_t lds_ld(int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x with path halving (a stored grandparent is always an ancestor of x).
__device__ int32_t lds_find(int32_t* lp, int32_t x)
{
    int32_t p = lds_ld(lp + x);
    while (p != x) {
        const int32_t g = lds_ld(lp + p);
        if (g != p) __hip_atomic_store(lp + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = p;
        p = g;
    }
    return x;
}

__device__ void lds_unite(int32_t* lp, int32_t a, int32_t b)
{
    while (true) {
        a = lds_find(lp, a);
        b = lds_find(lp, b);
        if (a == b) return;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(lp + b, b, a) == b) return;
    }
}

// One block per (row tile, column tile) with column tile >= row tile; pairs i < j only.  The
// tile's close pairs are first joined in an LDS union-find over its nodes (row members
// 0..kPostThreads-1, column members after them; a diagonal tile has only the row members); then
// every node that is not its local root is joined to that root in the global structure, at most
// one global hook per node and tile instead of one per close pair.
//
// A pair can only be close when its frequency term alone is below the window (the six terms
// are non-negative and rounding is monotone), i.e. when |f_b - f_a| < window / Tc up to
// rounding.  The column tile is therefore ranked by frequency in LDS, and each row tests only
// the columns inside [f_a - df, f_a + df], df = window / Tc with a relative margin of 1e-9
// (far above the rounding of the test): the same close pairs as testing every column, with the
// distance evaluated as before.
// Ascending order of frequencies as unsigned keys, NaN last (a NaN row is never close to any).
__device__ __forceinline__ uint64_t freq_key(double x)
{
    if (x != x) return ~0ull;
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ void __launch_bounds__(kPostThreads) hook_kernel(PostConst c, const double* rows, int64_t n,
                                                            double w2, double df, int32_t* parent)
{
    __shared__ PRow tile[kPostThreads];
    __shared__ int32_t lp[2 * kPostThreads];
    __shared__ double sf[kPostThreads];      // the column tile's frequencies in ascending order
    __shared__ int16_t ord[kPostThreads];    // their positions in the tile
    const int64_t bidx = blockIdx.x;
    int64_t tj = (int64_t)((sqrt(8.0 * (double)bidx + 1.0) - 1.0) * 0.5);
    while (tj * (tj + 1) / 2 > bidx) --tj;
    while ((tj + 1) * (tj + 2) / 2 <= bidx) ++tj;
    const int64_t ti = bidx - tj * (tj + 1) / 2;
    const bool diag = ti == tj;
    const int t = threadIdx.x;
    const int64_t i0 = ti * kPostThreads, j0 = tj * kPostThreads;
    const int64_t i = i0 + t;
    const int jn = (int)min((int64_t)kPostThreads, n - j0);
    // the column tile with its resolutions, computed once per block
    if (t < jn) tile[t] = load_row(rows + 6 * (j0 + t), c);
    lp[t] = t;
    lp[kPostThreads + t] = kPostThreads + t;
    __syncthreads();
    if (t < jn) {
        // rank by (frequency key, position): a permutation of 0 .. jn-1 whatever the values
        const double f = tile[t].f;
        const uint64_t kf = freq_key(f);
        int r = 0;
        for (int u = 0; u < jn; ++u) {
            const uint64_t ku = freq_key(tile[u].f);
            r += (ku < kf || (ku == kf && u < t)) ? 1 : 0;
        }
        sf[r] = f;
        ord[r] = (int16_t)t;
    }
    __syncthreads();
    if (i < n) {
        const PRow a = load_row(rows + 6 * i, c);
        // first rank with f >= f_a - df, first rank with f > f_a + df
        const double lo_f = a.f - df, hi_f = a.f + df;
        int lo = 0, hi = jn;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sf[mid] < lo_f) lo = mid + 1; else hi = mid;
        }
        int end = lo, top = jn;
        while (end < top) {
            const int mid = (end + top) >> 1;
            if (sf[mid] <= hi_f) end = mid + 1; else top = mid;
        }
        for (int k = lo; k < end; ++k) {
            const int jj = ord[k];
            if (j0 + jj <= i) continue;
            const int node = diag ? jj : kPostThreads + jj;
            // a pair already in one component cannot change the components (they only merge)
            if (lds_find(lp, t) == lds_find(lp, node)) continue;
            if (dist2(a, tile[jj], c) < w2) lds_unite(lp, t, node);
        }
    }
    __syncthreads();
    for (int x = t; x < 2 * kPostThreads; x += kPostThreads) {
        if (diag && x >= kPostThreads) break;
        const int64_t gx = x < kPostThreads ? i0 + x : j0 + (x - kPostThreads);
        if (gx >= n) continue;
        const int32_t r = lds_find(lp, x);
        if (r == x) continue;
        const int64_t gr = r < kPostThreads ? i0 + r : j0 + (r - kPostThreads);
        unite(parent, (int32_t)gx, (int32_t)gr);
    }
}

// Final labels: every row walks to its root with loads only and stores that root in its own
// slot.  (Path splitting here could overwrite a slot that its owner has already set to the
// root with a stale, non-root ancestor.)
__global__ void flatten_kernel(int32_t* parent, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t x = (int32_t)i;
    int32_t p = ld(parent + x);
    while (p != x) {
        x = p;
        p = ld(parent + x);
    }
    st(parent + i, x);
}

// ---------------------------------------------------------------- centroids

// Order-preserving 64-bit key of a double (larger double -> larger unsigned key).
__device__ __forceinline__ uint64_t dkey(double x)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ void cen_init_kernel(int64_t n, uint64_t* key, int32_t* top, double* weight, double* cen,
                                uint64_t* best_key, int32_t* best)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *best_key = 0;
        *best = INT32_MAX;
    }
    if (i >= n) return;
    key[i] = 0;
    top[i] = INT32_MAX;
    weight[i] = 0.0;
    for (int k = 0; k < 6; ++k) cen[6 * i + k] = 0.0;
}

// The members of a top-list fall into few, large clusters, so per-member atomics on the same
// few addresses would serialize: lanes of a wave that hold the same label first combine their
// values with shuffles, and one lane per (wave, label) performs the atomic.  Returns false when
// no lane is pending; otherwise the label lr of the wave's first pending lane and that lane.
__device__ __forceinline__ bool wave_next_label(bool pending, int32_t r, int32_t& lr, int& leader)
{
    const unsigned long long m = __ballot(pending);
    if (!m) return false;
    leader = __ffsll((long long)m) - 1;
    lr = __shfl(r, leader);
    return true;
}

__global__ void cen_max_kernel(const double* sig, const int32_t* label, int64_t n, uint64_t* key,
                               int32_t* status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool pending = false;
    int32_t r = -1;
    uint64_t k = 0;
    if (i < n) {
        const double s = sig[i];
        if (!(s > 0.0) || !isfinite(s)) raise_status(status, BSH_STATUS_INPUT);
        r = label[i];
        if (r < 0 || r >= n || label[r] != r)      // a label must name a member labelled by itself
            raise_status(status, BSH_STATUS_INPUT);
        else {
            pending = true;
            k = dkey(s);
        }
    }
    int32_t lr;
    int leader;
    while (wave_next_label(pending, r, lr, leader)) {
        const bool mine = pending && r == lr;
        unsigned long long v = mine ? k : 0ull;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(v, off, 64);
            v = o > v ? o : v;
        }
        if (lane == leader) atomicMax((unsigned long long*)(key + lr), v);
        pending = pending && !mine;
    }
}

__global__ void cen_top_kernel(const double* sig, const int32_t* label, int64_t n, const uint64_t* key,
                               int32_t* top)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = label[i];
    if (r < 0 || r >= n || label[r] != r) return;
    if (dkey(sig[i]) == key[r]) atomicMin(top + r, (int32_t)i);
}

__global__ void cen_sum_kernel(PostConst c, const double* rows, const double* sig, const int32_t* label,
                               int64_t n, double cut2, const int32_t* top, double* weight, double* cen)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool pending = false;
    int32_t r = -1;
    double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < n) {
        r = label[i];
        const int32_t t = (r >= 0 && r < n && label[r] == r) ? top[r] : -1;
        if (t >= 0 && t < n) {
            bool keep = true;
            if (cut2 > 0.0 && t != (int32_t)i) {
                const PRow a = load_row(rows + 6 * (int64_t)t, c);
                const PRow b = load_row(rows + 6 * i, c);
                keep = dist2(a, b, c) < cut2;
            }
            if (keep) {
                pending = true;
                const double s = sig[i];
                v[0] = s;
                for (int k = 0; k < 6; ++k) v[1 + k] = s * rows[6 * i + k];
            }
        }
    }
    int32_t lr;
    int leader;
    while (wave_next_label(pending, r, lr, leader)) {
        const bool mine = pending && r == lr;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const double x = wave_sum(mine ? v[k] : 0.0);
            if (lane == leader) atomicAdd(k == 0 ? weight + lr : cen + 6 * (int64_t)lr + (k - 1), x);
        }
        pending = pending && !mine;
    }
}

__global__ void cen_final_kernel(const int32_t* label, int64_t n, double* weight, double* cen,
                                 int32_t* top, uint64_t* best_key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (label[i] != (int32_t)i) {
        top[i] = -1;
        return;
    }
    const double w = weight[i];
    for (int k = 0; k < 6; ++k) cen[6 * i + k] = cen[6 * i + k] / w;
    atomicMax((unsigned long long*)best_key, (unsigned long long)dkey(w));
}

__global__ void cen_best_kernel(const int32_t* label, int64_t n, const double* weight,
                                const uint64_t* best_key, int32_t* best)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (label[i] == (int32_t)i && dkey(weight[i]) == *best_key) atomicMin(best, (int32_t)i);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kPostThreads - 1) / kPostThreads); }

}  // namespace
}  // namespace bsh

using namespace bsh;

extern "C" int bsh_post_rows(const double* sky, const int32_t* cand_sky, const double* cand_params,
                             int64_t n, double t_coh, double* rows_out, bsh_stream stream_)
{
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    clear_error();
    if (n < 0) return fail_inval("n < 0");
    if (n == 0) return BSH_OK;
    if (!sky || !cand_sky || !cand_params || !rows_out) return fail_inval("NULL pointer");
    if (!(std::isfinite(t_coh) && t_coh > 0.0)) return fail_inval("t_coh must be finite and positive");
    rows_kernel<<<blocks_for(n), kPostThreads, 0, stream>>>(sky, cand_sky, cand_params, n, t_coh, rows_out);
    return check_launch("bsh_post_rows");
}

extern "C" int bsh_significance(const float* score, int64_t n, const float* weight, int64_t n_seg,
                                int32_t kind, double rho_th, double* sig_out, bsh_stream stream_)
{
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    clear_error();
    if (n < 0 || n_seg < 0) return fail_inval("negative size");
    if (kind != 0 && kind != 1) return fail_inval("kind must be 0 (s_H) or 1 (s_P)");
    if (n == 0) return BSH_OK;
    if (n_seg == 0) return fail_inval("no segments");
    if (!score || !weight || !sig_out) return fail_inval("NULL pointer");
    if (kind == 0 && !(std::isfinite(rho_th) && rho_th > 0.0)) return fail_inval("rho_th must be positive");
    const double p0 = std::exp(-rho_th);
    const unsigned blocks = (unsigned)std::min<int64_t>(blocks_for(n), 1024);
    significance_kernel<<<blocks, kPostThreads, 0, stream>>>(score, n, weight, n_seg, kind, p0, sig_out);
    return check_launch("bsh_significance");
}

extern "C" size_t bsh_coincidences_workspace(int64_t na)
{
    return na < 0 ? 0 : (size_t)(2 * na + 1) * sizeof(int64_t);
}

extern "C" int bsh_coincidences(const bsh_post_params* pp, const double* rows_a, const double* sig_a,
                                int64_t na, const double* rows_b, const double* sig_b, int64_t nb,
                                double window, int64_t cap, int64_t* pairs_out, double* rows_out,
                                double* sig_out, int64_t* n_pairs_out, void* ws, size_t ws_bytes,
                                bsh_stream stream_)
{
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    clear_error();
    int rc = check_post(pp);
    if (rc) return rc;
    if (na < 0 || nb < 0 || cap < 0) return fail_inval("negative size");
    if (!(std::isfinite(window) && window > 0.0)) return fail_inval("window must be finite and positive");
    if (!n_pairs_out) return fail_inval("n_pairs_out is NULL");
    if (cap > 0 && (!pairs_out || !rows_out || !sig_out)) return fail_inval("NULL output with cap > 0");
    if (na > 0 && nb > 0 && (!rows_a || !sig_a || !rows_b || !sig_b)) return fail_inval("NULL list");
    if (ws_bytes < bsh_coincidences_workspace(na) || (na > 0 && !ws)) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, bsh_coincidences_workspace(na));
        return BSH_ENOMEM;
    }
    if (na == 0 || nb == 0) {
        zero_i64_kernel<<<1, 1, 0, stream>>>(n_pairs_out);
        return check_launch("bsh_coincidences");
    }
    if (na > INT32_MAX) return fail_inval("list a longer than 2^31 - 1");
    const PostConst c = post_const(pp);
    const double w2 = window * window;
    int64_t* count = static_cast<int64_t*>(ws);
    int64_t* offset = count + na;
    coinc_kernel<false><<<(unsigned)na, kPostThreads, 0, stream>>>(c, rows_a, sig_a, rows_b, sig_b, nb, w2,
                                                                  count, nullptr, 0, nullptr, nullptr,
                                                                  nullptr);
    scan_kernel<<<1, kPostThreads, 0, stream>>>(count, na, offset, n_pairs_out);
    coinc_kernel<true><<<(unsigned)na, kPostThreads, 0, stream>>>(c, rows_a, sig_a, rows_b, sig_b, nb, w2,
                                                                 nullptr, offset, cap, pairs_out, rows_out,
                                                                 sig_out);
    return check_launch("bsh_coincidences");
}

extern "C" int bsh_cluster(const bsh_post_params* pp, const double* rows, int64_t n, double window,
                           int32_t* label_out, bsh_stream stream_)
{
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    clear_error();
    int rc = check_post(pp);
    if (rc) return rc;
    if (n < 0) return fail_inval("n < 0");
    if (n > INT32_MAX) return fail_inval("more than 2^31 - 1 templates");
    if (!(std::isfinite(window) && window > 0.0)) return fail_inval("window must be finite and positive");
    if (n == 0) return BSH_OK;
    if (!rows || !label_out) return fail_inval("NULL pointer");
    const PostConst c = post_const(pp);
    const int64_t nt = (n + kPostThreads - 1) / kPostThreads;
    const int64_t tiles = nt * (nt + 1) / 2;
    if (tiles > INT32_MAX) return fail_inval("too many templates for one launch");
    iota_kernel<<<blocks_for(n), kPostThreads, 0, stream>>>(label_out, n);
    // frequency half-width of the window, with a relative margin far above the rounding of the
    // distance's frequency term
    const double df = window / c.t_coh * (1.0 + 1e-9);
    hook_kernel<<<(unsigned)tiles, kPostThreads, 0, stream>>>(c, rows, n, window * window, df, label_out);
    flatten_kernel<<<blocks_for(n), kPostThreads, 0, stream>>>(label_out, n);
    return check_launch("bsh_cluster");
}

extern "C" size_t bsh_cluster_centroids_workspace(int64_t n)
{
    return n < 0 ? 0 : (size_t)(n + 1) * sizeof(uint64_t);
}

extern "C" int bsh_cluster_centroids(const bsh_post_params* pp, const double* rows, const double* sig,
                                     const int32_t* label, int64_t n, double cut, double* centroid_out,
                                     double* weight_out, int32_t* top_out, int32_t* best_out,
                                     int32_t* status, void* ws, size_t ws_bytes, bsh_stream stream_)
{
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    clear_error();
    int rc = check_post(pp);
    if (rc) return rc;
    if (n < 0) return fail_inval("n < 0");
    if (n > INT32_MAX) return fail_inval("more than 2^31 - 1 templates");
    if (std::isnan(cut)) return fail_inval("cut is NaN");
    if (n == 0) return BSH_OK;
    if (!rows || !sig || !label || !centroid_out || !weight_out || !top_out || !best_out)
        return fail_inval("NULL pointer");
    if (ws_bytes < bsh_cluster_centroids_workspace(n) || !ws) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, bsh_cluster_centroids_workspace(n));
        return BSH_ENOMEM;
    }
    const PostConst c = post_const(pp);
    uint64_t* key = static_cast<uint64_t*>(ws);
    uint64_t* best_key = key + n;
    const double cut2 = cut > 0.0 ? cut * cut : 0.0;
    const unsigned b = blocks_for(n);
    cen_init_kernel<<<b, kPostThreads, 0, stream>>>(n, key, top_out, weight_out, centroid_out, best_key,
                                                    best_out);
    cen_max_kernel<<<b, kPostThreads, 0, stream>>>(sig, label, n, key, status);
    cen_top_kernel<<<b, kPostThreads, 0, stream>>>(sig, label, n, key, top_out);
    cen_sum_kernel<<<b, kPostThreads, 0, stream>>>(c, rows, sig, label, n, cut2, top_out, weight_out,
                                                   centroid_out);
    cen_final_kernel<<<b, kPostThreads, 0, stream>>>(label, n, weight_out, centroid_out, top_out, best_key);
    cen_best_kernel<<<b, kPostThreads, 0, stream>>>(label, n, weight_out, best_key, best_out);
    return check_launch("bsh_cluster_centroids");
}
