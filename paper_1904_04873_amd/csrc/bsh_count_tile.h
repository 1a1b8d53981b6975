// Tile body of the stage-1 weighted number count (Sec. IV.C eq:hough2; the GPU loop K1 of
// Sec. IV.B), shared by the plain kernel (bsh_count.hip) and the persistent kernel of the
// batched plan (bsh_count_batch.hip).  Internal to libbsh.
//
// Work decomposition.  A tile is one sky pixel, one orbital period P and `lanes` binary
// templates (a_p, t_asc) of that period; each lane owns one binary template and all n_f0
// (<= 90) frequency bins of the band.  Segments stream through LDS in chunks: per segment the
// block stages D cos(W t_J), D sin(W t_J) and D (W is the tile's, D_J the pixel's Doppler
// factor), the weight (or the group subset sums) and the bit-packed peakgram row.
//
// Per (lane, segment) G = D (1 - a_p W cos(W (t_J - t_asc))) is evaluated as track_G does in
// every kernel, from the staged D C, D S and the lane's a_p W cos / sin(W t_asc).  The band's
// bins follow from G alone:  k_i = floor(fl((k0 + i) G + 1/2)),  i = 0 .. n_f0-1.
// For |G - 1| < 1/(2 n_f0) the offsets r_i = k_i - (k0 + i) form a monotone step with at
// most one step (the canonical rounding is monotone in i and the exact offsets drift by
// (n_f0-1)|G-1| < 1 bin).  So two evaluations (i = 0 and the last) give r_0 and r_last;
// when they differ, a single-precision guess of the step's position (taken as it is when its
// error bound cannot move it across an integer, else checked by exact evaluations and a
// bisection) gives the first i with r_i = r_last.  The band's n_f0
// peak bits are then one funnel-shifted 96-bit window of the row, with the part above the
// step taken one bit further (or nearer).  This is the exact counterpart of the
// look-up-table reuse of one Doppler modulation over neighbouring frequencies (Sec. IV.B):
// every template still reads the bin of its own exact track.
//
// Accumulation: either select-and-add (each bit selects its weight; optional uint32 counts)
// or subset-sum tables over groups of segments (see count_tile_pair).
#pragma once

#include "bsh_count.h"

namespace bsh {

// One (binary template, segment) track across the band: G = D (1 - a_p W cos phi) and the
// canonical bins kf, kf + span of the band's lowest and highest f0 (span = last + the residual's
// step, -1, 0 or +1, when the track is valid).
struct BandTrack {
    double G, y0;
    int kf, span;
    bool ok;
};

// G of one (binary template, segment): the circular track_G, or track_G_ecc on a grid with an
// eccentricity pair (Ac2 = As2 = 0 there gives the circular value bit for bit anyway).
template <bool kEcc>
__device__ __forceinline__ double tile_G(double DC, double DS, double D, double DC2, double DS2, double Ac,
                                         double As, double Ac2, double As2)
{
    if constexpr (kEcc) return track_G_ecc(D, DC, DS, Ac, As, DC2, DS2, Ac2, As2);
    else return track_G(D, DC, DS, Ac, As);
}

// The canonical evaluations (no branches).  ok is false, and a flag is raised, when the track
// leaves the staged row [klo, khi) or drifts more than one bin across the band.
__device__ __forceinline__ BandTrack band_track(double G, double F0, double FL, int klo, int khi, int last,
                                                bool& bad_range, bool& bad_model)
{
    BandTrack t;
    t.G = G;
    // the nearest bin floor(F G + 1/2) of a positive track value is its truncation
    t.y0 = fma(F0, t.G, 0.5);
    t.kf = (int)t.y0;
    const int kl = (int)fma(FL, t.G, 0.5);
    t.span = kl - t.kf;
    const bool in_range = (t.kf >= klo) & (kl < khi);
    t.ok = in_range & (t.span >= last - 1) & (t.span <= last + 1);
    bad_range |= !in_range;
    bad_model |= in_range & !t.ok;
    return t;
}

// Bit i of the 96-bit (m0, m1, m2) is the peakgram bit of f0 bin i as if the band had no f0-shift
// step: one funnel-shifted window of the LDS row.  A failed track reads the row's zero padding
// (pad_at = 32 n_words), so its masks are zero without a select.
__device__ __forceinline__ void band_window(const uint32_t* row, const BandTrack& t, int klo, int pad_at,
                                            uint32_t& m0, uint32_t& m1, uint32_t& m2)
{
    const int at = t.ok ? t.kf - klo : pad_at;
    const int qw = at >> 5;
    const int sh = at & 31;
    const uint32_t w0 = row[qw], w1 = row[qw + 1], w2 = row[qw + 2], w3 = row[qw + 3];
    m0 = __builtin_amdgcn_alignbit(w1, w0, sh);
    m1 = __builtin_amdgcn_alignbit(w2, w1, sh);
    m2 = __builtin_amdgcn_alignbit(w3, w2, sh);
}

// The first f0 index whose residual differs from r0, by canonical evaluations: the guess
// g = floor(q) + 1 (clamped to 1 .. last) is checked at g and g - 1, and a bisection runs when
// it is off.
__device__ __forceinline__ int step_exact(double G, int kf, double F0, int last, float q)
{
    const int r0 = kf - (int)F0;
    auto resid = [&](int i) { return (int)fma(F0 + (double)i, G, 0.5) - ((int)F0 + i); };
    const float qc = fminf(fmaxf(q, 0.f), (float)last);
    const int g = min(max((int)qc + 1, 1), last);
    int lo, hi;              // r_lo = r0, r_hi != r0
    if (g < last && resid(g) == r0) {
        lo = g;
        hi = last;
    } else if (g == 1 || resid(g - 1) == r0) {
        lo = g - 1;
        hi = g;
    } else {
        lo = 0;
        hi = g - 1;
    }
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (resid(mid) == r0) lo = mid; else hi = mid;
    }
    return hi;
}

// Where the band has an f0-shift step (t.ok and t.span != last), take the bins above it one bit
// further (span = last + 1) or nearer (span = last - 1).
__device__ __forceinline__ void band_step(const BandTrack& t, double F0, int last, uint32_t& m0, uint32_t& m1,
                                          uint32_t& m2)
{
    // The residual r_i = k_i - (k0 + i) steps once, at the first index past the crossing
    // i* = (u - frac(y0)) / (G - 1) of y0 + i (G - 1) with the next integer above (a step up,
    // u = 1) or below (a step down, u = 0); the numerator is exact (y0 > 0, so frac(y0) =
    // y0 - kf).  The single-precision q carries a relative error below 4e-7 (two conversions,
    // the reciprocal, the product), i.e. below 4e-5 for i* < 96, and the canonical evaluations
    // place the step within 3e-11 / |G - 1| < 3e-5 of i* when |G - 1| >= 1e-6.  A q further
    // than 1e-3 from an integer, in (0, last), is therefore floor(i*) and the step sits at
    // floor(q) + 1; the rest (a few in a thousand, or a G - 1 whose sign contradicts the
    // step's direction, which makes q <= 0) is decided by canonical evaluations.
    const bool up = t.span > last;
    const double f = __builtin_amdgcn_fract(t.y0);
    const float num = (float)((up ? 1.0 : 0.0) - f);
    const float gm1 = (float)(t.G - 1.0);
    const float q = num * __builtin_amdgcn_rcpf(gm1);
    // 0 <= q < last as one unsigned comparison of the bit patterns (negative q and NaN have the
    // sign or all exponent bits set); q = 0 fails the distance test
    const bool in_band = __float_as_uint(q) < __float_as_uint((float)last);
    const bool sure = (fabsf(__builtin_amdgcn_fractf(q) - 0.5f) < 0.499f) & in_band & (fabsf(gm1) >= 1e-6f);
    int hi = sure ? (int)q + 1 : 0;
    if (!sure) hi = step_exact(t.G, t.kf, F0, last, q);
    // the 96-bit mask moved by one bin: down a bit (a step up: bin i takes bin i + 1's bit) or
    // up a bit, as funnel shifts by 1 or 31 of the words (m2, m1, m0) framed by zeros
    const uint32_t b0 = up ? m0 : 0u, b1 = up ? m1 : m0, b2 = up ? m2 : m1, b3 = up ? 0u : m2;
    const uint32_t by = up ? 1u : 31u;
    const uint32_t n0 = __builtin_amdgcn_alignbit(b1, b0, by);
    const uint32_t n1 = __builtin_amdgcn_alignbit(b2, b1, by);
    const uint32_t n2 = __builtin_amdgcn_alignbit(b3, b2, by);
    // bits hi.. of the 96-bit mask (1 <= hi < 96): one shift, placed by word
    const uint32_t sh = 0xffffffffu << (hi & 31);
    const uint32_t s0 = hi < 32 ? sh : 0u;
    const uint32_t s1 = hi < 32 ? 0xffffffffu : (hi < 64 ? sh : 0u);
    const uint32_t s2 = hi < 64 ? 0xffffffffu : sh;
    m0 = (n0 & s0) | (m0 & ~s0);
    m1 = (n1 & s1) | (m1 & ~s1);
    m2 = (n2 & s2) | (m2 & ~s2);
}

// The peak bits of the band's n_f0 templates of one (binary template, segment): bit i of the
// 96-bit (m0, m1, m2) is the peakgram bit of f0 bin i's track.  Returns false, with zero masks,
// when the track failed.
__device__ __forceinline__ bool band_mask(const uint32_t* row, double G, double F0, double FL, int klo, int khi,
                                          int last, int pad_at, uint32_t& m0, uint32_t& m1, uint32_t& m2,
                                          bool& bad_range, bool& bad_model)
{
    const BandTrack t = band_track(G, F0, FL, klo, khi, last, bad_range, bad_model);
    band_window(row, t, klo, pad_at, m0, m1, m2);
    if (t.ok && t.span != last) band_step(t, F0, last, m0, m1, m2);
    return t.ok;
}

template <bool kCount, int kChunk, bool kEcc>
__device__ __forceinline__ void count_tile(const ItemDesc& d, int s, int ip, int64_t tile,
                                           TileSmem<kChunk, kEcc>& sm, uint32_t* row)
{
    const int tid = threadIdx.x;
    const int lanes = blockDim.x;
    const int64_t q = tile * lanes + tid;

    // position q of the period group -> (a_p index, t_asc point)
    int ia = -1;
    int64_t j = 0, cum = 0;
    for (int a = 0; a < d.n_ap; ++a) {
        const int64_t c0 = d.tasc_off[(int64_t)a * d.n_per + ip];
        const int64_t n = d.tasc_off[(int64_t)a * d.n_per + ip + 1] - c0;
        if (ia < 0 && q < cum + n) { ia = a; j = q - cum; }
        cum += n;
    }
    const bool active = ia >= 0;
    const int64_t b = active ? d.tasc_off[(int64_t)ia * d.n_per + ip] + j : 0;
    const double W = kTwoPi / d.period[ip];
    const double apW = active ? d.a_p[ia] * W : 0.0;
    double sb = 0.0, cb = 1.0;
    if (active) track_sincos(W * d.t_asc[b], sb, cb);
    const double Ac = apW * cb, As = apW * sb;
    double Ac2 = 0.0, As2 = 0.0;
    if constexpr (kEcc) ecc_coeffs(apW, cb, sb, d.ec, d.es, Ac2, As2);

    const int sg = d.sky_lo + s;
    const double nx = d.sky[3 * sg], ny = d.sky[3 * sg + 1], nz = d.sky[3 * sg + 2];
    const float* wrow = d.w + (d.w_per_sky ? (int64_t)s * d.n_seg : 0);
    const double F0 = (double)d.k0;
    const int last = d.n_f0 - 1;
    const double FL = (double)(d.k0 + last);
    const int klo = (int)d.k_lo;
    const int nwp = d.n_words + kRowPad;

    float acc[kNF], tot[kNF];
    uint32_t cnt[kCount ? kNF : 1];
#pragma unroll
    for (int i = 0; i < kNF; ++i) { acc[i] = 0.f; tot[i] = 0.f; }
#pragma unroll
    for (int i = 0; i < (kCount ? kNF : 1); ++i) cnt[i] = 0u;
    int since_flush = 0;
    bool bad_range = false, bad_model = false;

    for (int64_t j0 = 0; j0 < d.n_seg; j0 += kChunk) {
        const int nj = (int)min((int64_t)kChunk, d.n_seg - j0);
        __syncthreads();
        for (int jj = tid; jj < nj; jj += lanes) {
            const int64_t J = j0 + jj;
            double sp, cp;
            track_sincos(W * d.t_mid[J], sp, cp);
            const double D = doppler_factor(d.v + 3 * J, nx, ny, nz);
            sm.DC[jj] = D * cp;
            sm.DS[jj] = D * sp;
            sm.D[jj] = D;
            if constexpr (kEcc) {
                double c2, s2;
                double_angle(cp, sp, c2, s2);
                sm.DC2[jj] = D * c2;
                sm.DS2[jj] = D * s2;
            }
            sm.W[jj] = wrow[J];
        }
        for (int e = tid; e < nj * nwp; e += lanes) {
            const int jj = e / nwp;
            const int wd = e - jj * nwp;
            row[e] = wd < d.n_words ? d.bits[(j0 + jj) * d.n_words + wd] : 0u;
        }
        __syncthreads();
        if (!active) continue;

        for (int jj = 0; jj < nj; ++jj) {
            uint32_t m0, m1, m2;
            const double G = tile_G<kEcc>(sm.DC[jj], sm.DS[jj], sm.D[jj], kEcc ? sm.DC2[jj] : 0.0,
                                          kEcc ? sm.DS2[jj] : 0.0, Ac, As, Ac2, As2);
            if (!band_mask(row + jj * nwp, G, F0, FL, klo, klo + d.n_bins, last, 32 * d.n_words, m0, m1, m2,
                           bad_range, bad_model))
                continue;

            const uint32_t wb = __float_as_uint(sm.W[jj]);
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
    if (bad_range) raise_status(d.status, BSH_STATUS_RANGE);
    if (bad_model) raise_status(d.status, BSH_STATUS_MODEL);
    if (!active) return;

    const int64_t base_idx = ((int64_t)s * d.n_bin + b) * d.n_f0;
#pragma unroll
    for (int i = 0; i < kNF; ++i) {
        if (i < d.n_f0) {
            if (d.wsum_out) d.wsum_out[base_idx + i] = tot[i] + acc[i];
            if (kCount && d.count_out) d.count_out[base_idx + i] = cnt[kCount ? i : 0];
        }
    }
}


// Table variant of the weighted count.  Segments are taken in groups of eight; a 256-entry
// table per group holds every subset sum of the group's eight weights, so that for each f0 bin
// the eight peak bits of the group form a byte index and one table read and one add replace
// eight select-and-add steps.  The table is built from the 16-entry subset-sum tables of the
// group's two halves, T8[b] = T_first[b & 15] + T_second[b >> 4].
//
// Two adjacent lanes share one binary template.  With bin i = 32 w + 4 n + r (w = 0..2,
// n = 0..7, r = 0..3), lane h = lane & 1 owns the bins with r = 2h, 2h + 1 (46 and 44 of the
// band's 90), so it keeps 46 register partial sums instead of 90, which leaves room for three
// waves per SIMD.  Per group lane h evaluates the tracks of the group's segments 4h .. 4h + 3,
// transposes their four 96-bit masks (a 4 x 4 bit transpose per nibble column: word A[w][r] holds
// in nibble n the four segments' bits of bin 32 w + 4 n + r), and the pair swaps the two words
// A[w][r] of the partner's r values (a cross-lane move inside each pair of lanes).  Each lane then
// merges the first four segments' nibbles (from lane 0) and the last four's (from lane 1) into
// bytes, and every one of its bins costs one byte extraction, one table address and one FP32 add
// per eight segments.  The register partial sums (at most kFlushGroups groups each) are folded
// into the lane's own slots of the output map, bounding the FP32 error by
// (kFlushGroups + 4 + n_seg / (8 kFlushGroups)) ulps of the total.  Per bin the table entries and
// the order of the additions do not depend on the tile shape or on how lanes share templates.
constexpr int kPairSlots = 46;   // (w, k, n) with k = r - 2h, minus w = 2, n = 7

// (w, k, n) -> 0 .. 45: sixteen slots per word for w = 0, 1, fourteen (n < 7) for w = 2
__device__ __forceinline__ constexpr int pair_slot(int w, int k, int n) { return w < 2 ? (w * 2 + k) * 8 + n : 32 + k * 7 + n; }

__device__ __forceinline__ uint32_t pair_swap(uint32_t x)
{
    // quad_perm [1, 0, 3, 2]: every lane takes its pair partner's value
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);
}

template <int kChunk, bool kEcc>
__device__ __forceinline__ void count_tile_pair(const ItemDesc& d, int s, int ip, int64_t tile,
                                                TileSmemLut<kChunk, kEcc>& sm, uint32_t* row)
{
    static_assert(kChunk % kGroup8 == 0, "chunks hold whole groups");
    const int tid = threadIdx.x;
    const int lanes = blockDim.x;
    const int h = tid & 1;
    const int64_t q = tile * (lanes >> 1) + (tid >> 1);

    int ia = -1;
    int64_t j = 0, cum = 0;
    for (int a = 0; a < d.n_ap; ++a) {
        const int64_t c0 = d.tasc_off[(int64_t)a * d.n_per + ip];
        const int64_t n = d.tasc_off[(int64_t)a * d.n_per + ip + 1] - c0;
        if (ia < 0 && q < cum + n) { ia = a; j = q - cum; }
        cum += n;
    }
    const bool active = ia >= 0;
    const int64_t b = active ? d.tasc_off[(int64_t)ia * d.n_per + ip] + j : 0;
    const double W = kTwoPi / d.period[ip];
    const double apW = active ? d.a_p[ia] * W : 0.0;
    double sb = 0.0, cb = 1.0;
    if (active) track_sincos(W * d.t_asc[b], sb, cb);
    const double Ac = apW * cb, As = apW * sb;
    double Ac2 = 0.0, As2 = 0.0;
    if constexpr (kEcc) ecc_coeffs(apW, cb, sb, d.ec, d.es, Ac2, As2);

    const int sg = d.sky_lo + s;
    const double nx = d.sky[3 * sg], ny = d.sky[3 * sg + 1], nz = d.sky[3 * sg + 2];
    const float* wrow = d.w + (d.w_per_sky ? (int64_t)s * d.n_seg : 0);
    const double F0 = (double)d.k0;
    const int last = d.n_f0 - 1;
    const double FL = (double)(d.k0 + last);
    const int klo = (int)d.k_lo;
    const int nwp = d.n_words + kRowPad;

    float acc[kPairSlots];
#pragma unroll
    for (int i = 0; i < kPairSlots; ++i) acc[i] = 0.f;
    int since_flush = 0;
    bool flushed = false;
    float* out = d.wsum_out + ((int64_t)s * d.n_bin + b) * d.n_f0;
    const int nf = d.n_f0;
    auto flush = [&]() {
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int n = 0; n < 8; ++n) {
                    if (w == 2 && n == 7) continue;
                    const int sl = pair_slot(w, k, n);
                    const int i = 32 * w + 4 * n + 2 * h + k;
                    if (i < nf) out[i] = flushed ? out[i] + acc[sl] : acc[sl];
                    acc[sl] = 0.f;
                }
        flushed = true;
    };
    bool bad_range = false, bad_model = false;

    for (int64_t j0 = 0; j0 < d.n_seg; j0 += kChunk) {
        const int nj = (int)min((int64_t)kChunk, d.n_seg - j0);
        const int ng8 = (nj + kGroup8 - 1) / kGroup8;
        const int ng = 2 * ng8;
        __syncthreads();
        for (int jj = tid; jj < ng * kGroup; jj += lanes) {
            const int64_t J = j0 + min(jj, nj - 1);
            double sp, cp;
            track_sincos(W * d.t_mid[J], sp, cp);
            const double D = doppler_factor(d.v + 3 * J, nx, ny, nz);
            sm.DC[jj] = D * cp;
            sm.DS[jj] = D * sp;
            sm.D[jj] = D;
            if constexpr (kEcc) {
                double c2, s2;
                double_angle(cp, sp, c2, s2);
                sm.DC2[jj] = D * c2;
                sm.DS2[jj] = D * s2;
            }
        }
        for (int e = tid; e < ng * kGroup * nwp; e += lanes) {
            const int jj = e / nwp;
            const int wd = e - jj * nwp;
            row[e] = (jj < nj && wd < d.n_words) ? d.bits[(j0 + jj) * d.n_words + wd] : 0u;
        }
        for (int g = tid; g < ng; g += lanes) {
            float w4[kGroup];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const int jj = g * kGroup + u;
                w4[u] = jj < nj ? wrow[j0 + jj] : 0.f;
            }
            float* T = sm.T + g * 16;
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                float t = 0.f;
#pragma unroll
                for (int u = 0; u < kGroup; ++u)
                    if (m & (1 << u)) t += w4[u];
                T[m] = t;
            }
        }
        __syncthreads();
        for (int e = tid; e < ng8 * 256; e += lanes) {
            const int g = e >> 8, m = e & 255;
            sm.T8[e] = sm.T[(2 * g) * 16 + (m & 15)] + sm.T[(2 * g + 1) * 16 + (m >> 4)];
        }
        __syncthreads();
        if (!active) continue;

        for (int g8 = 0; g8 < ng8; ++g8) {
            // this lane's half of the group: segments 4h .. 4h + 3
            const int hg = 2 * g8 + h;
            uint32_t mk[kGroup][3];
            BandTrack tr[kGroup];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const int jj = hg * kGroup + u;
                const double G = tile_G<kEcc>(sm.DC[jj], sm.DS[jj], sm.D[jj], kEcc ? sm.DC2[jj] : 0.0,
                                              kEcc ? sm.DS2[jj] : 0.0, Ac, As, Ac2, As2);
                tr[u] = band_track(G, F0, FL, klo, klo + d.n_bins, last, bad_range, bad_model);
            }
#pragma unroll
            for (int u = 0; u < kGroup; ++u)
                band_window(row + (hg * kGroup + u) * nwp, tr[u], klo, 32 * d.n_words, mk[u][0], mk[u][1],
                            mk[u][2]);
#pragma unroll
            for (int u = 0; u < kGroup; ++u)
                if (tr[u].ok && tr[u].span != last) band_step(tr[u], F0, last, mk[u][0], mk[u][1], mk[u][2]);
            const float* T8 = sm.T8 + g8 * 256;
#pragma unroll
            for (int w = 0; w < 3; ++w) {
                uint32_t x0 = mk[0][w], x1 = mk[1][w], x2 = mk[2][w], x3 = mk[3][w];
                uint32_t t;
                t = ((x0 >> 2) ^ x2) & 0x33333333u; x2 ^= t; x0 ^= t << 2;
                t = ((x1 >> 2) ^ x3) & 0x33333333u; x3 ^= t; x1 ^= t << 2;
                t = ((x0 >> 1) ^ x1) & 0x55555555u; x1 ^= t; x0 ^= t << 1;
                t = ((x2 >> 1) ^ x3) & 0x55555555u; x3 ^= t; x2 ^= t << 1;
                // A[w][r] = x_r: this lane's four segments, every bin
                const uint32_t A[4] = {x0, x1, x2, x3};
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    // the first four segments' nibbles (L) come from lane 0, the last four's (H)
                    // from lane 1: lane 0 takes its own word of r = k and lane 1's, lane 1 takes
                    // lane 0's word of r = 2 + k and its own
                    const uint32_t from_partner_hi = pair_swap(A[2 + k]);   // every lane swaps,
                    const uint32_t from_partner_lo = pair_swap(A[k]);       // then each selects
                    const uint32_t L = h == 0 ? A[k] : from_partner_hi;
                    const uint32_t H = h == 1 ? A[2 + k] : from_partner_lo;
                    const uint32_t b0 = (L & 0x0f0f0f0fu) | ((H << 4) & 0xf0f0f0f0u);
                    const uint32_t b1 = ((L >> 4) & 0x0f0f0f0fu) | (H & 0xf0f0f0f0u);
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb) {
                        acc[pair_slot(w, k, 2 * jb)] += T8[(b0 >> (8 * jb)) & 255u];
                        if (!(w == 2 && jb == 3)) acc[pair_slot(w, k, 2 * jb + 1)] += T8[(b1 >> (8 * jb)) & 255u];
                    }
                }
            }
            if (++since_flush == kFlushGroups) {
                since_flush = 0;
                flush();
            }
        }
    }
    if (bad_range) raise_status(d.status, BSH_STATUS_RANGE);
    if (bad_model) raise_status(d.status, BSH_STATUS_MODEL);
    if (active && (since_flush > 0 || !flushed)) flush();
}

// kMode % kEccMode: 0 = select-and-add, weighted sums only; 1 = select-and-add with counts;
// 2 = table.  kMode >= kEccMode: the same on the ELL1 track of the item's eccentricity pair.
template <int kMode, int kChunk>
constexpr size_t fixed_smem_bytes()
{
    constexpr bool kEcc = kMode >= kEccMode;
    constexpr size_t b = kMode % kEccMode == 2 ? sizeof(TileSmemLut<kChunk, kEcc>) : sizeof(TileSmem<kChunk, kEcc>);
    return (b + 15) & ~(size_t)15;
}

// The tile's LDS: the fixed structure, then the rows.
template <int kMode, int kChunk>
__device__ __forceinline__ void run_tile(const ItemDesc& d, int s, int ip, int64_t tile, unsigned char* smem)
{
    constexpr int kM = kMode % kEccMode;
    constexpr bool kEcc = kMode >= kEccMode;
    uint32_t* row = reinterpret_cast<uint32_t*>(smem + fixed_smem_bytes<kMode, kChunk>());
    if constexpr (kM == 2)
        count_tile_pair<kChunk, kEcc>(d, s, ip, tile, *reinterpret_cast<TileSmemLut<kChunk, kEcc>*>(smem), row);
    else
        count_tile<kM == 1, kChunk, kEcc>(d, s, ip, tile, *reinterpret_cast<TileSmem<kChunk, kEcc>*>(smem), row);
}

// Launch-bounds hint of the blocks per CU: two for the table variant, one for the select
// variants (whose 90 partial sums, and 90 counts, fill the registers).  The table variant's
// register allocation comes out at about 155 registers, so three waves per SIMD fit.
template <int kMode>
constexpr int min_blocks() { return kMode % kEccMode == 2 ? 2 : 1; }

// Instantiate a kernel template for every (mode, chunk) and call f with the chosen one.
#define BSH_DISPATCH(MODE, CHUNK, F)                                                          \
    switch ((MODE) * 1000 + (CHUNK)) {                                                        \
    case 128: F(0, 128); break;                                                               \
    case 256: F(0, 256); break;                                                               \
    case 512: F(0, 512); break;                                                               \
    case 1128: F(1, 128); break;                                                              \
    case 1256: F(1, 256); break;                                                              \
    case 1512: F(1, 512); break;                                                              \
    case 2128: F(2, 128); break;                                                              \
    case 2256: F(2, 256); break;                                                              \
    case 2512: F(2, 512); break;                                                              \
    case 3128: F(3, 128); break;                                                              \
    case 3256: F(3, 256); break;                                                              \
    case 3512: F(3, 512); break;                                                              \
    case 4128: F(4, 128); break;                                                              \
    case 4256: F(4, 256); break;                                                              \
    case 4512: F(4, 512); break;                                                              \
    case 5128: F(5, 128); break;                                                              \
    case 5256: F(5, 256); break;                                                              \
    case 5512: F(5, 512); break;                                                              \
    default: return fail_inval("kernel mode / chunk");                                        \
    }

// LDS bytes of one block: the fixed structure and the rows of n_words words (0 for an unknown
// mode or chunk).
#define BSH_FIXED_SMEM(M, C) fixed = fixed_smem_bytes<M, C>()
inline size_t smem_bytes_of(int mode, int chunk, int n_words)
{
    size_t fixed = 0;
    switch (mode * 1000 + chunk) {
    case 128: BSH_FIXED_SMEM(0, 128); break;
    case 256: BSH_FIXED_SMEM(0, 256); break;
    case 512: BSH_FIXED_SMEM(0, 512); break;
    case 1128: BSH_FIXED_SMEM(1, 128); break;
    case 1256: BSH_FIXED_SMEM(1, 256); break;
    case 1512: BSH_FIXED_SMEM(1, 512); break;
    case 2128: BSH_FIXED_SMEM(2, 128); break;
    case 2256: BSH_FIXED_SMEM(2, 256); break;
    case 2512: BSH_FIXED_SMEM(2, 512); break;
    case 3128: BSH_FIXED_SMEM(3, 128); break;
    case 3256: BSH_FIXED_SMEM(3, 256); break;
    case 3512: BSH_FIXED_SMEM(3, 512); break;
    case 4128: BSH_FIXED_SMEM(4, 128); break;
    case 4256: BSH_FIXED_SMEM(4, 256); break;
    case 4512: BSH_FIXED_SMEM(4, 512); break;
    case 5128: BSH_FIXED_SMEM(5, 128); break;
    case 5256: BSH_FIXED_SMEM(5, 256); break;
    case 5512: BSH_FIXED_SMEM(5, 512); break;
    default: return 0;
    }
    return fixed + row_bytes(chunk, n_words);
}
#undef BSH_FIXED_SMEM

}  // namespace bsh
