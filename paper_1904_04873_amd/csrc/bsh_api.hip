// libbsh host entry points that are not the two statistics: error state, argument checks,
// template-bank enumeration (Sec. IV.C), the peakgram (Sec. IV.A), stage-1 index decoding
// and per-candidate track bins.
#include <cstdarg>
#include <cstring>

#include "bsh_internal.h"

namespace bsh {

static thread_local char g_err[512] = {0};

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

int check_segments(const bsh_segments* seg, bool need_bits, bool need_power)
{
    if (!seg) return fail_inval("segments is NULL");
    if (seg->n_seg < 0) return fail_inval("n_seg < 0");
    if (!(seg->t_coh > 0.0) || !std::isfinite(seg->t_coh)) return fail_inval("t_coh must be > 0");
    if (seg->n_bins < 1 || seg->n_bins > 32 * BSH_MAX_WORDS) return fail_inval("n_bins out of 1..512");
    if (seg->n_seg > 0) {
        if (!seg->t_mid || !seg->v_over_c || !seg->weight) return fail_inval("NULL segment table");
        if (need_bits && !seg->peak_bits) return fail_inval("peak_bits is NULL");
        if (need_power && !seg->power) return fail_inval("power is NULL");
    }
    if (!std::isfinite(seg->v_max_host) || seg->v_max_host < 0.0) return fail_inval("v_max_host");
    return BSH_OK;
}

int check_grid(const bsh_grid* g)
{
    if (!g) return fail_inval("grid is NULL");
    if (g->n_sky < 1 || !g->sky) return fail_inval("sky");
    if (g->n_f0 < 1 || g->n_f0 > BSH_MAX_F0) return fail_inval("n_f0 out of 1..90");
    if (g->n_ap < 1 || g->n_per < 1 || g->n_per > BSH_MAX_PER) return fail_inval("n_ap / n_per");
    if (!g->a_p || !g->period || !g->tasc_off || !g->t_asc) return fail_inval("NULL grid table");
    if (!g->a_p_host || !g->period_host || !g->tasc_off_host) return fail_inval("NULL host grid table");
    if (g->k0 < 1) return fail_inval("k0 < 1");
    const int64_t n_cells = (int64_t)g->n_ap * g->n_per;
    if (g->tasc_off_host[0] != 0) return fail_inval("tasc_off[0] != 0");
    for (int64_t c = 0; c < n_cells; ++c)
        if (g->tasc_off_host[c + 1] < g->tasc_off_host[c]) return fail_inval("tasc_off not monotone");
    for (int32_t i = 0; i < g->n_ap; ++i)
        if (!std::isfinite(g->a_p_host[i])) return fail_inval("a_p not finite");
    for (int32_t i = 0; i < g->n_per; ++i)
        if (!(g->period_host[i] > 0.0) || !std::isfinite(g->period_host[i]))
            return fail_inval("period must be finite and > 0");
    if (!std::isfinite(g->ecc_c) || !std::isfinite(g->ecc_s) || g->ecc_c * g->ecc_c + g->ecc_s * g->ecc_s >= 0.25)
        return fail_inval("eccentricity pair must be finite with e < 0.5");
    return BSH_OK;
}

// The bound on |G - 1| that the window checks use: |v/c| <= v, a_p W (1 + e) <= apw, so
// |D B - 1| <= v + apw + v apw; m is that bound in bins at the band's top, rounded up.
static void track_bound(const bsh_segments* seg, const bsh_grid* g, double& v, double& apw, double& m)
{
    apw = 0.0;
    for (int32_t ia = 0; ia < g->n_ap; ++ia)
        for (int32_t ip = 0; ip < g->n_per; ++ip)
            apw = std::fmax(apw, std::fabs(g->a_p_host[ia]) * (kTwoPi / g->period_host[ip]));
    // the ELL1 bracket is at most 1 + e in size
    apw *= 1.0 + std::sqrt(g->ecc_c * g->ecc_c + g->ecc_s * g->ecc_s);
    v = seg->v_max_host;
    const double f_hi = (double)(g->k0 + g->n_f0);
    m = std::ceil(f_hi * (v + apw + v * apw));
}

static bool window_covers(const bsh_segments* seg, const bsh_grid* g, double m, double& lo, double& hi)
{
    lo = (double)g->k0 - m - 1.0;
    hi = (double)(g->k0 + g->n_f0 - 1) + m + 1.0;
    return lo >= (double)seg->k_lo && hi <= (double)(seg->k_lo + seg->n_bins - 1);
}

int check_window(const bsh_segments* seg, const bsh_grid* g)
{
    if (seg->v_max_host <= 0.0) return BSH_OK;   // unknown: the device status flag decides
    double v, apw, m, lo, hi;
    track_bound(seg, g, v, apw, m);
    if (!window_covers(seg, g, m, lo, hi)) {
        set_error("staged row [%lld, %lld) does not cover the tracks' bound [%.0f, %.0f]",
                  (long long)seg->k_lo, (long long)(seg->k_lo + seg->n_bins), lo, hi);
        return BSH_ERANGE;
    }
    return BSH_OK;
}

bool proven_window(const bsh_segments* seg, const bsh_grid* g, double* v_out, double* apw_out)
{
    if (!(seg->v_max_host > 0.0)) return false;
    double v, apw, m, lo, hi;
    track_bound(seg, g, v, apw, m);
    // the band's offsets k_i - (k0 + i) drift by at most (n_f0 - 1) |G - 1| bins: below one half
    // they step at most once, so every track's span is last - 1, last or last + 1
    const double drift = (double)(g->n_f0 - 1) * (v + apw + v * apw);
    if (!window_covers(seg, g, m, lo, hi) || !(drift < 0.5)) return false;
    *v_out = v;
    *apw_out = apw;
    return true;
}

}  // namespace bsh

using namespace bsh;

extern "C" int bsh_version(void) { return 10000; }

extern "C" const char* bsh_last_error(void) { return bsh::g_err; }

// ---------------------------------------------------------------- template bank (host)

static double uniform_value(double lo, double hi, int32_t n, int32_t i)
{
    if (n == 1) return lo;
    if (i == n - 1) return hi;
    const double step = (hi - lo) / (double)(n - 1);
    return lo + (double)i * step;
}

extern "C" int bsh_grid_build(const bsh_grid_spec* spec, double t_mid, double* a_p, double* period,
                              int64_t* tasc_off, double* t_asc, int64_t t_asc_cap,
                              int64_t* n_bin_out)
{
    clear_error();
    if (!spec || !a_p || !period || !tasc_off || !n_bin_out) return fail_inval("NULL pointer");
    if (spec->n_ap < 1 || spec->n_per < 1 || spec->n_f0 < 1) return fail_inval("empty grid");
    if (!(spec->t_coh > 0.0)) return fail_inval("t_coh");
    if (!std::isfinite(t_mid)) return fail_inval("t_mid");
    if (spec->tasc_fixed <= 0 && (spec->tasc_min < 1 || spec->tasc_max < spec->tasc_min))
        return fail_inval("t_asc clamp");
    for (int32_t i = 0; i < spec->n_ap; ++i) a_p[i] = uniform_value(spec->ap_lo, spec->ap_hi, spec->n_ap, i);
    for (int32_t i = 0; i < spec->n_per; ++i) {
        period[i] = uniform_value(spec->per_lo, spec->per_hi, spec->n_per, i);
        if (!(period[i] > 0.0)) return fail_inval("period must be > 0");
    }
    const double f_hi = (double)(spec->k0 + spec->n_f0) / spec->t_coh;
    int64_t total = 0;
    tasc_off[0] = 0;
    for (int32_t ia = 0; ia < spec->n_ap; ++ia) {
        for (int32_t ip = 0; ip < spec->n_per; ++ip) {
            int64_t n;
            if (spec->tasc_fixed > 0) {
                n = spec->tasc_fixed;
            } else {
                const double w = kTwoPi / period[ip];
                const double x = spec->tasc_rule_m * spec->t_coh * f_hi * a_p[ia] * w;
                n = (int64_t)std::ceil(x);
                if (n < spec->tasc_min) n = spec->tasc_min;
                if (n > spec->tasc_max) n = spec->tasc_max;
            }
            const int64_t cell = (int64_t)ia * spec->n_per + ip;
            if (t_asc) {
                if (total + n > t_asc_cap) {
                    set_error("t_asc capacity %lld too small", (long long)t_asc_cap);
                    return BSH_ENOMEM;
                }
                const double P = period[ip];
                const double base = t_mid - 0.5 * P;
                const double step = P / (double)n;
                for (int64_t j = 0; j < n; ++j) t_asc[total + j] = base + (double)j * step;
            }
            total += n;
            tasc_off[cell + 1] = total;
        }
    }
    *n_bin_out = total;
    return BSH_OK;
}

// ---------------------------------------------------------------- normalized power

// eq:HoughPower: rho_k = P_k / <n_k>^2, the noise level <n_k>^2 estimated from the running median
// of the window [k - m, k + m] divided by the expected median of 2m+1 unit exponentials.
// One block per segment; the raw row sits in LDS.  The median of a window is the value v with
// #{< v} <= m < #{<= v}; instead of counting that for every candidate of every window, each
// raw position c counts it once for the first window that holds c and then slides the window
// across the 2m + 1 windows that hold c, updating both counts by the entry that leaves and the
// one that enters.  A window's median is the first position in window order that meets the
// condition (an LDS atomic minimum over the positions that do; they all hold the same value).
// A window that holds a NaN has no median: its output is NaN (as the median of such a window is
// taken to be), found by a scan of the window in the rows that hold a NaN at all.
constexpr int kMaxRaw = 4096;

__global__ __launch_bounds__(256) void normalize_kernel(const float* __restrict__ raw, int32_t n_raw,
                                                        int32_t m, double beta, float* __restrict__ rho)
{
    __shared__ float row[kMaxRaw];
    __shared__ int first[kMaxRaw];
    __shared__ int any_nan;
    const int64_t J = blockIdx.x;
    const float* src = raw + J * n_raw;
    const int n_out = n_raw - 2 * m;
    if (threadIdx.x == 0) any_nan = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n_raw; i += blockDim.x) {
        const float v = src[i];
        row[i] = v;
        if (v != v) any_nan = 1;
    }
    for (int i = threadIdx.x; i < n_out; i += blockDim.x) first[i] = n_raw;
    __syncthreads();
    for (int c = threadIdx.x; c < n_raw; c += blockDim.x) {
        const float v = row[c];
        const int w_lo = max(0, c - 2 * m), w_hi = min(c, n_out - 1);   // windows [w, w + 2m] holding c
        int lt = 0, le = 0;
        for (int i = w_lo; i <= w_lo + 2 * m; ++i) {
            lt += row[i] < v ? 1 : 0;
            le += row[i] <= v ? 1 : 0;
        }
        for (int w = w_lo;; ++w) {
            if (lt <= m && le > m) atomicMin(&first[w], c);
            if (w == w_hi) break;
            const float out = row[w], in = row[w + 2 * m + 1];
            lt += (in < v ? 1 : 0) - (out < v ? 1 : 0);
            le += (in <= v ? 1 : 0) - (out <= v ? 1 : 0);
        }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < n_out; w += blockDim.x) {
        const float centre = row[w + m];
        bool nan_in_window = false;
        if (any_nan)
            for (int i = w; i <= w + 2 * m; ++i) nan_in_window |= row[i] != row[i];
        const double med = nan_in_window || first[w] >= n_raw ? (double)NAN : (double)row[first[w]];
        rho[J * n_out + w] = (float)(((double)centre * beta) / med);
    }
}

extern "C" int bsh_normalize(const float* raw, int64_t n_seg, int32_t n_raw, int32_t window,
                             float* rho_out, bsh_stream stream)
{
    clear_error();
    if (n_seg < 0) return fail_inval("n_seg < 0");
    if (window < 1 || (window & 1) == 0) return fail_inval("window must be odd and >= 1");
    if (n_raw < window || n_raw > kMaxRaw) return fail_inval("n_raw must be in window .. 4096");
    if (n_seg == 0) return BSH_OK;
    if (n_seg > 0x7fffffff) return fail_inval("too many segments");
    if (!raw || !rho_out) return fail_inval("NULL pointer");
    const int32_t m = (window - 1) / 2;
    double beta = 0.0;                       // expected median of `window` unit exponentials
    for (int32_t i = 2 * m + 1; i >= m + 1; --i) beta += 1.0 / (double)i;
    hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)n_seg), dim3(256), 0, (hipStream_t)stream, raw,
                       n_raw, m, beta, rho_out);
    return check_launch("bsh_normalize");
}

// ---------------------------------------------------------------- peakgram

__global__ void peakgram_kernel(const float* __restrict__ power, int64_t n_seg, int32_t n_bins,
                                int32_t n_words, double rho_th, uint32_t* __restrict__ bits)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_seg * n_words) return;
    const int64_t J = e / n_words;
    const int32_t w = (int32_t)(e - J * n_words);
    const float* row = power + J * n_bins;
    uint32_t word = 0u;
    const int32_t c0 = 32 * w;
    const int32_t nb = min(32, n_bins - c0);
    for (int32_t b = 0; b < nb; ++b)
        word |= ((double)row[c0 + b] > rho_th ? 1u : 0u) << b;
    bits[e] = word;
}

extern "C" int bsh_peakgram(const float* power, int64_t n_seg, int32_t n_bins, double rho_th,
                            uint32_t* bits, bsh_stream stream)
{
    clear_error();
    if (n_seg < 0 || n_bins < 1) return fail_inval("shape");
    if (n_seg == 0) return BSH_OK;
    if (!power || !bits) return fail_inval("NULL pointer");
    if (!std::isfinite(rho_th)) return fail_inval("rho_th");
    const int32_t nw = words_for(n_bins);
    const int64_t n = n_seg * nw;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(peakgram_kernel, dim3((unsigned)blocks), dim3(threads), 0,
                       (hipStream_t)stream, power, n_seg, n_bins, nw, rho_th, bits);
    return check_launch("bsh_peakgram");
}

// ---------------------------------------------------------------- index decoding

__global__ void decode_kernel(const double* __restrict__ a_p, const double* __restrict__ period,
                              const int64_t* __restrict__ tasc_off, const double* __restrict__ t_asc,
                              int64_t n_cells, int32_t n_per, int32_t n_f0, int64_t k0,
                              int64_t n_bin, int32_t n_sky, const int64_t* __restrict__ index,
                              int64_t n, int32_t* __restrict__ cand_sky,
                              double* __restrict__ cand)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int64_t idx = index[c];
    const int64_t total = (int64_t)n_sky * n_bin * n_f0;
    if (idx < 0 || idx >= total) {
        cand_sky[c] = -1;
        cand[4 * c + 0] = 0.0; cand[4 * c + 1] = 0.0; cand[4 * c + 2] = 0.0; cand[4 * c + 3] = 0.0;
        return;
    }
    const int64_t i = idx % n_f0;
    const int64_t sb = idx / n_f0;
    const int64_t b = sb % n_bin;
    const int64_t s = sb / n_bin;
    int64_t lo = 0, hi = n_cells;            // tasc_off[lo] <= b < tasc_off[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (tasc_off[mid] <= b) lo = mid; else hi = mid;
    }
    cand_sky[c] = (int32_t)s;
    cand[4 * c + 0] = (double)(k0 + i);
    cand[4 * c + 1] = a_p[lo / n_per];
    cand[4 * c + 2] = period[lo % n_per];
    cand[4 * c + 3] = t_asc[b];
}

extern "C" int bsh_decode_templates(const bsh_grid* grid, const int64_t* index, int64_t n,
                                    int32_t* cand_sky, double* cand_params, bsh_stream stream)
{
    clear_error();
    int rc = check_grid(grid);
    if (rc) return rc;
    if (n < 0) return fail_inval("n < 0");
    if (n == 0) return BSH_OK;
    if (!index || !cand_sky || !cand_params) return fail_inval("NULL pointer");
    const int64_t n_cells = (int64_t)grid->n_ap * grid->n_per;
    const int64_t n_bin = grid->tasc_off_host[n_cells];
    const int threads = 256;
    hipLaunchKernelGGL(decode_kernel, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0,
                       (hipStream_t)stream, grid->a_p, grid->period, grid->tasc_off, grid->t_asc,
                       n_cells, grid->n_per, grid->n_f0, grid->k0, n_bin, grid->n_sky, index, n,
                       cand_sky, cand_params);
    return check_launch("bsh_decode_templates");
}

// ---------------------------------------------------------------- track bins

__global__ void track_bins_kernel(const double* __restrict__ t_mid, const double* __restrict__ v,
                                  const double* __restrict__ sky, int32_t n_sky,
                                  const int32_t* __restrict__ cand_sky,
                                  const double* __restrict__ cand, int64_t n, int64_t n_seg,
                                  int32_t* __restrict__ bins, int32_t* status)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n_seg) return;
    const int64_t c = e / n_seg;
    const int64_t J = e - c * n_seg;
    const int32_t s = cand_sky[c];
    if (s < 0 || s >= n_sky) {
        bins[e] = -1;
        if (J == 0) raise_status(status, BSH_STATUS_INPUT);
        return;
    }
    const Cand cd = load_cand(cand + 4 * c);
    double st, ct;
    track_sincos(cd.W * t_mid[J], st, ct);
    const double D = doppler_factor(v + 3 * J, sky[3 * s], sky[3 * s + 1], sky[3 * s + 2]);
    bins[e] = (int32_t)track_bin(cd.F, track_G(D, D * ct, D * st, cd.Ac, cd.As));
}

extern "C" int bsh_track_bins(const bsh_segments* seg, const double* sky, int32_t n_sky,
                              const int32_t* cand_sky, const double* cand_params, int64_t n,
                              int32_t* bins_out, int32_t* status, bsh_stream stream)
{
    clear_error();
    int rc = check_segments(seg, false, false);
    if (rc) return rc;
    if (n < 0) return fail_inval("n < 0");
    if (n_sky < 1) return fail_inval("n_sky < 1");
    if (n == 0 || seg->n_seg == 0) return BSH_OK;
    if (!sky || !cand_sky || !cand_params || !bins_out) return fail_inval("NULL pointer");
    const int64_t tot = n * seg->n_seg;
    const int threads = 256;
    hipLaunchKernelGGL(track_bins_kernel, dim3((unsigned)((tot + threads - 1) / threads)),
                       dim3(threads), 0, (hipStream_t)stream, seg->t_mid, seg->v_over_c, sky, n_sky,
                       cand_sky, cand_params, n, seg->n_seg, bins_out, status);
    return check_launch("bsh_track_bins");
}
