// Stage-1 weighted number count (Sec. IV.C eq:hough2; the GPU loop K1 of Sec. IV.B).
//
// Work decomposition.  A block owns one sky pixel, one orbital period P and a tile of
// kBlock binary templates (a_p, t_asc) of that period; each lane owns one binary template
// and all n_f0 (<= 90) frequency bins of the band.  Segments stream through LDS in chunks:
// per segment the block stages cos(W t_J), sin(W t_J) (shared by every lane, since W is the
// block's), the Doppler factor D_J of the pixel, the weight and the bit-packed peakgram row.
//
// Per (lane, segment) the orbit factor is B = 1 - a_p W (cos(W t_J) cos(W t_asc) +
// sin(W t_J) sin(W t_asc)) and G = D B, in the operation order of track_x.  Bins of the band follow from G alone:
//   k_i = floor(fl((k0 + i) G) + 1/2),  i = 0 .. n_f0-1.
// For |G - 1| < 1/(2 n_f0) the offsets r_i = k_i - (k0 + i) form a monotone step with at
// most one step (the canonical rounding is monotone in i and the exact offsets drift by
// (n_f0-1)|G-1| < 1 bin).  So two evaluations (i = 0 and the last) give r_0 and r_last;
// when they differ a binary search over canonical evaluations finds the first i with
// r_i = r_last.  The band's n_f0 peak bits are then one funnel-shifted 96-bit window of the
// row, with the part above the step taken one bit further (or nearer).  This is the exact
// counterpart of the look-up-table reuse of one Doppler modulation over neighbouring
// frequencies (Sec. IV.B): every template still reads the bin of its own exact track.
//
// Accumulation: per lane, 90 FP32 partial sums of w_J p_J that are folded into 90 running
// totals every kFlush segments (bounded error for long observations), plus optional uint32
// counts.  Each bit costs a sign-extending bit-field extract, an AND with the weight's bit
// pattern and an add.
#include <cstring>

#include "bsh_internal.h"

namespace {

using namespace bsh;

constexpr int kBlock = 256;    // binary templates per block (lanes)
constexpr int kChunk = 256;    // segments staged per LDS pass
constexpr int kFlush = 64;     // segments per FP32 partial sum
constexpr int kRowPad = 3;     // zero words staged after each row
constexpr int kNF = BSH_MAX_F0;

struct CountParams {
    const double* t_mid;
    const double* v;
    const float* w;
    const uint32_t* bits;
    const double* sky;
    const double* a_p;
    const double* period;
    const int64_t* tasc_off;
    const double* t_asc;
    uint32_t* count_out;
    float* wsum_out;
    int32_t* status;
    int64_t n_seg;
    int64_t n_bin;
    int64_t k_lo;
    int64_t k0;
    int32_t w_per_sky;
    int32_t n_words;
    int32_t n_bins;
    int32_t n_f0;
    int32_t n_ap;
    int32_t n_per;
    int32_t tiles_per_sky;
    int32_t tile_start[BSH_MAX_PER + 1];   // first tile of each period group
};

__device__ __forceinline__ uint32_t upper_mask(int t)
{
    // bits b with b >= t set
    return t <= 0 ? 0xffffffffu : (t >= 32 ? 0u : (0xffffffffu << t));
}

template <bool kCount>
__global__ __launch_bounds__(kBlock) void hough_count_kernel(const CountParams p)
{
    __shared__ double sC[kChunk];
    __shared__ double sS[kChunk];
    __shared__ double sD[kChunk];
    __shared__ float sW[kChunk];
    __shared__ uint32_t sRow[kChunk * (BSH_MAX_WORDS + kRowPad)];

    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    const int s = blk / p.tiles_per_sky;
    const int t = blk - s * p.tiles_per_sky;
    int ip = 0;
    {
        int lo = 0, hi = p.n_per;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (p.tile_start[mid] <= t) lo = mid; else hi = mid;
        }
        ip = lo;
    }
    const int64_t q = (int64_t)(t - p.tile_start[ip]) * kBlock + tid;

    // position q of the period group -> (a_p index, t_asc point)
    int ia = -1;
    int64_t j = 0, cum = 0;
    for (int a = 0; a < p.n_ap; ++a) {
        const int64_t c0 = p.tasc_off[(int64_t)a * p.n_per + ip];
        const int64_t n = p.tasc_off[(int64_t)a * p.n_per + ip + 1] - c0;
        if (ia < 0 && q < cum + n) { ia = a; j = q - cum; }
        cum += n;
    }
    const bool active = ia >= 0;
    const int64_t b = active ? p.tasc_off[(int64_t)ia * p.n_per + ip] + j : 0;
    const double W = kTwoPi / p.period[ip];
    const double apW = active ? p.a_p[ia] * W : 0.0;
    double sb = 0.0, cb = 1.0;
    if (active) sincos(W * p.t_asc[b], &sb, &cb);

    const double nx = p.sky[3 * s], ny = p.sky[3 * s + 1], nz = p.sky[3 * s + 2];
    const float* wrow = p.w + (p.w_per_sky ? (int64_t)s * p.n_seg : 0);
    const double F0 = (double)p.k0;
    const int last = p.n_f0 - 1;
    const double FL = (double)(p.k0 + last);
    const double klo = (double)p.k_lo;
    const int nwp = p.n_words + kRowPad;

    float acc[kNF], tot[kNF];
    uint32_t cnt[kCount ? kNF : 1];
#pragma unroll
    for (int i = 0; i < kNF; ++i) { acc[i] = 0.f; tot[i] = 0.f; }
#pragma unroll
    for (int i = 0; i < (kCount ? kNF : 1); ++i) cnt[i] = 0u;
    int since_flush = 0;
    bool bad_range = false, bad_model = false;

    for (int64_t j0 = 0; j0 < p.n_seg; j0 += kChunk) {
        const int nj = (int)min((int64_t)kChunk, p.n_seg - j0);
        __syncthreads();
        for (int jj = tid; jj < nj; jj += kBlock) {
            const int64_t J = j0 + jj;
            double sp, cp;
            sincos(W * p.t_mid[J], &sp, &cp);
            sC[jj] = cp;
            sS[jj] = sp;
            sD[jj] = doppler_factor(p.v + 3 * J, nx, ny, nz);
            sW[jj] = wrow[J];
        }
        for (int e = tid; e < nj * nwp; e += kBlock) {
            const int jj = e / nwp;
            const int wd = e - jj * nwp;
            sRow[e] = wd < p.n_words ? p.bits[(j0 + jj) * p.n_words + wd] : 0u;
        }
        __syncthreads();
        if (!active) continue;

        for (int jj = 0; jj < nj; ++jj) {
            // same operation order as orbit_phase / track_x: G = D (1 - a_p W cos phi)
            const double cphi = fma(sC[jj], cb, sS[jj] * sb);
            const double G = sD[jj] * (1.0 - apW * cphi);
            const double kf = floor(F0 * G + 0.5);
            const double kl = floor(FL * G + 0.5);
            const int r0 = (int)(kf - F0);
            const int delta = (int)(kl - FL) - r0;
            const int base = (int)(kf - klo);
            const int top = (int)(kl - klo);
            if (base < 0 || top >= p.n_bins) { bad_range = true; continue; }
            if (delta < -1 || delta > 1) { bad_model = true; continue; }

            const uint32_t* row = sRow + jj * nwp;
            const int qw = base >> 5;
            const int sh = base & 31;
            const uint32_t w0 = row[qw], w1 = row[qw + 1], w2 = row[qw + 2], w3 = row[qw + 3];
            uint32_t m0 = __builtin_amdgcn_alignbit(w1, w0, sh);
            uint32_t m1 = __builtin_amdgcn_alignbit(w2, w1, sh);
            uint32_t m2 = __builtin_amdgcn_alignbit(w3, w2, sh);
            if (delta != 0) {
                int lo = 0, hi = last;   // r_lo = r0, r_hi = r0 + delta
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    const double Fm = F0 + (double)mid;
                    const int rm = (int)(floor(Fm * G + 0.5) - Fm);
                    if (rm == r0) lo = mid; else hi = mid;
                }
                uint32_t n0, n1, n2;
                if (delta > 0) {
                    n0 = __builtin_amdgcn_alignbit(m1, m0, 1);
                    n1 = __builtin_amdgcn_alignbit(m2, m1, 1);
                    n2 = m2 >> 1;
                } else {
                    n0 = m0 << 1;
                    n1 = __builtin_amdgcn_alignbit(m1, m0, 31);
                    n2 = __builtin_amdgcn_alignbit(m2, m1, 31);
                }
                const uint32_t s0 = upper_mask(hi), s1 = upper_mask(hi - 32), s2 = upper_mask(hi - 64);
                m0 = (n0 & s0) | (m0 & ~s0);
                m1 = (n1 & s1) | (m1 & ~s1);
                m2 = (n2 & s2) | (m2 & ~s2);
            }

            const uint32_t wb = __float_as_uint(sW[jj]);
#pragma unroll
            for (int i = 0; i < kNF; ++i) {
                const uint32_t m = i < 32 ? m0 : (i < 64 ? m1 : m2);
                const int bit = ((int)(m << (31 - (i & 31)))) >> 31;   // 0 or -1
                acc[i] += __uint_as_float((uint32_t)bit & wb);
                if (kCount) cnt[i] -= (uint32_t)bit;
            }
            if (++since_flush == kFlush) {
                since_flush = 0;
#pragma unroll
                for (int i = 0; i < kNF; ++i) { tot[i] += acc[i]; acc[i] = 0.f; }
            }
        }
    }
    if (bad_range) raise_status(p.status, BSH_STATUS_RANGE);
    if (bad_model) raise_status(p.status, BSH_STATUS_MODEL);
    if (!active) return;

    const int64_t base_idx = ((int64_t)s * p.n_bin + b) * p.n_f0;
#pragma unroll
    for (int i = 0; i < kNF; ++i) {
        if (i < p.n_f0) {
            if (p.wsum_out) p.wsum_out[base_idx + i] = tot[i] + acc[i];
            if (kCount && p.count_out) p.count_out[base_idx + i] = cnt[kCount ? i : 0];
        }
    }
}

}  // namespace

extern "C" int bsh_hough_count(const bsh_segments* seg, const bsh_grid* grid, uint32_t* count_out,
                               float* wsum_out, int32_t* status, bsh_stream stream)
{
    clear_error();
    int rc = check_segments(seg, true, false);
    if (rc) return rc;
    rc = check_grid(grid);
    if (rc) return rc;
    if (!count_out && !wsum_out) return fail_inval("both outputs are NULL");
    rc = check_window(seg, grid);
    if (rc) return rc;

    CountParams p;
    std::memset(&p, 0, sizeof(p));
    p.t_mid = seg->t_mid;
    p.v = seg->v_over_c;
    p.w = seg->weight;
    p.bits = seg->peak_bits;
    p.sky = grid->sky;
    p.a_p = grid->a_p;
    p.period = grid->period;
    p.tasc_off = grid->tasc_off;
    p.t_asc = grid->t_asc;
    p.count_out = count_out;
    p.wsum_out = wsum_out;
    p.status = status;
    p.n_seg = seg->n_seg;
    p.k_lo = seg->k_lo;
    p.k0 = grid->k0;
    p.w_per_sky = seg->weight_per_sky;
    p.n_words = words_for(seg->n_bins);
    p.n_bins = seg->n_bins;
    p.n_f0 = grid->n_f0;
    p.n_ap = grid->n_ap;
    p.n_per = grid->n_per;
    const int64_t n_cells = (int64_t)grid->n_ap * grid->n_per;
    p.n_bin = grid->tasc_off_host[n_cells];

    // tiles of each period group
    int64_t tiles = 0;
    for (int32_t ip = 0; ip < grid->n_per; ++ip) {
        int64_t group = 0;
        for (int32_t ia = 0; ia < grid->n_ap; ++ia) {
            const int64_t c = (int64_t)ia * grid->n_per + ip;
            group += grid->tasc_off_host[c + 1] - grid->tasc_off_host[c];
        }
        p.tile_start[ip] = (int32_t)tiles;
        tiles += (group + kBlock - 1) / kBlock;
    }
    p.tile_start[grid->n_per] = (int32_t)tiles;
    for (int32_t ip = grid->n_per + 1; ip <= BSH_MAX_PER; ++ip) p.tile_start[ip] = (int32_t)tiles;
    p.tiles_per_sky = (int32_t)tiles;
    const int64_t blocks = tiles * grid->n_sky;
    if (tiles == 0 || p.n_bin == 0) return BSH_OK;
    if (blocks > 0x7fffffff) return fail_inval("grid too large for one launch");
    if (seg->n_seg == 0) {
        // no segments: every count is zero
        const int64_t n_t = (int64_t)grid->n_sky * p.n_bin * grid->n_f0;
        if (wsum_out && hipMemsetAsync(wsum_out, 0, n_t * sizeof(float), (hipStream_t)stream) != hipSuccess)
            return check_launch("bsh_hough_count memset");
        if (count_out && hipMemsetAsync(count_out, 0, n_t * sizeof(uint32_t), (hipStream_t)stream) != hipSuccess)
            return check_launch("bsh_hough_count memset");
        return BSH_OK;
    }

    if (count_out)
        hipLaunchKernelGGL(hough_count_kernel<true>, dim3((unsigned)blocks), dim3(kBlock), 0,
                           (hipStream_t)stream, p);
    else
        hipLaunchKernelGGL(hough_count_kernel<false>, dim3((unsigned)blocks), dim3(kBlock), 0,
                           (hipStream_t)stream, p);
    return check_launch("bsh_hough_count");
}
