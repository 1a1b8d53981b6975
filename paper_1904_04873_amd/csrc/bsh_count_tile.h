// Tile body of the stage-1 weighted number count (Sec. IV.C eq:hough2; the GPU loop K1 of
// Sec. IV.B), shared by the kernels of every launch form (bsh_count_kernels.h).  Internal to
// libbsh.
//
// Work decomposition.  A tile is one sky pixel, one orbital period P and binary templates
// (a_p, t_asc) of that period: in the select variant each of the `lanes` lanes owns one binary
// template and all n_f0 (<= 90) frequency bins of the band; in the table variant two lanes share
// one (count_tile_pair).  Segments stream through LDS in chunks: per segment the block stages
// D cos(W t_J), D sin(W t_J) and D (W is the tile's, D_J the pixel's Doppler factor), the weight
// (or the groups' subset-sum tables) and the bit-packed peakgram row.
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

#include <cstddef>

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
// leaves the staged row [klo, khi) or drifts more than one bin across the band.  kProven: the
// launch's bounds exclude both (proven_window), so neither is tested.
template <bool kProven = false>
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
    if constexpr (kProven) {
        t.ok = true;
    } else {
        const bool in_range = (t.kf >= klo) & (kl < khi);
        t.ok = in_range & (t.span >= last - 1) & (t.span <= last + 1);
        bad_range |= !in_range;
        bad_model |= in_range & !t.ok;
    }
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
// off: the mask bit of f0 bin 0 (bit i + off holds bin i).
__device__ __forceinline__ void band_step(const BandTrack& t, double F0, int last, uint32_t& m0, uint32_t& m1,
                                          uint32_t& m2, int off = 0)
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
    // bits hb = hi + off .. of the 96-bit mask (1 <= hb < 96): one shift, placed by word
    const int hb = hi + off;
    const uint32_t sh = 0xffffffffu << (hb & 31);
    const uint32_t s0 = hb < 32 ? sh : 0u;
    const uint32_t s1 = hb < 32 ? 0xffffffffu : (hb < 64 ? sh : 0u);
    const uint32_t s2 = hb < 64 ? 0xffffffffu : sh;
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
// Two adjacent lanes share one binary template; lane h = lane & 1 evaluates the tracks of the
// group's segments 4h .. 4h + 3 and owns the bins i = 32 w + 8 j + 4 h + t (w = 0..2, j = 0..3,
// t = 0..3; 46 and 44 of the band's 90), so it keeps 46 register partial sums instead of 90,
// which leaves room for three waves per SIMD.  Lane 1 reads its 96-bit windows four bins lower
// than lane 0 (its mask bit i + 4 holds bin i).  Per group each lane transposes its four masks (a
// 4 x 4 bit transpose per nibble column: word A[w][t] holds in nibble n the four segments' bits
// of the lane's bin 32 w + 4 n + t, minus 4 on lane 1), and both lanes of the pair swap the same
// word A[w][t].  Each lane merges its own low nibbles with its partner's high nibbles: on lane 0
// the merged word's bytes are the indices (first four segments low, last four high) of bins
// 32 w + 8 j + t, and on lane 1 the merged word moved down by one nibble (with the next word's
// first nibble on top) holds those of bins 32 w + 8 j + 4 + t, so the exchange needs no select.  The indices are split into 16-bit halves, each turned into its table
// address by one multiply-add, and every bin of the lane costs that address (and half a split)
// and one FP32 add per eight segments.  The register partial sums (at most kFlushGroups groups
// each) are folded into the lane's own slots of the output map, bounding the FP32 error by
// (kFlushGroups + 4 + n_seg / (8 kFlushGroups)) ulps of the total.  Per bin the table entries and
// the order of the additions do not depend on the tile shape or on how lanes share templates.
constexpr int kPairSlots = 46;   // (w, t, j), minus w = 2, j = 3 for t = 2, 3

// (w, t, j) -> 0 .. 45: sixteen slots per word for w = 0, 1; for w = 2 twelve with j < 3 and two
// (t = 0, 1) with j = 3
__device__ __forceinline__ constexpr int pair_slot(int w, int t, int j)
{
    return w < 2 ? (w * 4 + t) * 4 + j : (j < 3 ? 32 + t * 3 + j : 44 + t);
}

__device__ __forceinline__ uint32_t pair_swap(uint32_t x)
{
    // quad_perm [1, 0, 3, 2]: every lane takes its pair partner's value
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);
}

// LDS byte address base + 4 x (low or high 16-bit half of y); each half of y holds a table
// index below 256 in its low byte and zeros above.  lds_at reads the float at such an address.
__device__ __forceinline__ uint32_t lut_addr_lo(uint32_t y, uint32_t base)
{
    uint32_t a;
    asm("v_mad_u32_u16 %0, %1, 4, %2" : "=v"(a) : "v"(y), "s"(base));
    return a;
}

__device__ __forceinline__ uint32_t lut_addr_hi(uint32_t y, uint32_t base)
{
    uint32_t a;
    asm("v_mad_u32_u16 %0, %1, 4, %2 op_sel:[1,0,0,0]" : "=v"(a) : "v"(y), "s"(base));
    return a;
}

__device__ __forceinline__ float lds_at(uint32_t a)
{
    return *(const __attribute__((address_space(3))) float*)(size_t)a;
}

// Row words per lane whose loads a chunk of the form for proven windows issues ahead of their
// stores (four of the five of a typical row at one lane per segment; one more and the batched
// kernel's registers no longer allow three waves per SIMD).
constexpr int kPreWords = 4;

// smem: the block's LDS (rows first, then the structure at byte offset sm_off).
// kProven: the launch's tracks are proven to stay inside the rows with at most one f0-shift step
// (proven_window).  Instead of testing every track, the inputs of the proof are tested as they
// are staged: each segment's |D - 1| against the proof's |v/c| and its phase for finiteness, each
// lane's a_p W (1 + e) against the proof's bound and its t_asc phase for finiteness.  A failed
// test raises the range flag (the outputs are then undefined, as for any track outside the rows);
// the segment is staged as one with G = 1, and the lane skips its groups, so that every window
// the kernel reads is one of a track inside the rows.
template <int kChunk, bool kEcc, bool kProven = false>
__device__ __forceinline__ void count_tile_pair(const ItemDesc& d, int s, int ip, int64_t tile,
                                                TileSmemLut<kChunk, kEcc>& sm, uint32_t* row,
                                                const unsigned char* smem, uint32_t sm_off)
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
    // the lane's a_p W (1 + e) within the proof's bound (a relative 1e-12 for rounding), and its
    // phase finite (fails on NaN)
    const bool claim_bad = kProven && active &&
                           !((fabs(apW) * (1.0 + sqrt(d.ec * d.ec + d.es * d.es)) <= d.apw_claim * (1.0 + 1e-12)) &
                             (fabs(sb) <= 1.0) & (fabs(cb) <= 1.0));

    const int sg = d.sky_lo + s;
    const double nx = d.sky[3 * sg], ny = d.sky[3 * sg + 1], nz = d.sky[3 * sg + 2];
    // NULL weights: every weight is one (the sums are then the unweighted counts)
    const float* wrow = d.w ? d.w + (d.w_per_sky ? (int64_t)s * d.n_seg : 0) : nullptr;
    const double F0 = (double)d.k0;
    const int last = d.n_f0 - 1;
    const double FL = (double)(d.k0 + last);
    const int klo = (int)d.k_lo;
    const int nwp = d.n_words + kRowPad;
    // The window of f0 bin 0 starts at row bit kf - klo on lane 0 and four bits lower on lane 1,
    // i.e. up to four bits before the row, in the previous row's zero padding (the rows of lane
    // 1's segments 4 .. 7 of a group are never the chunk's first); a failed track reads the row's
    // padding, from four bits before it on lane 1.  The bits below f0 bin 0 are never used.
    const int off = 4 * h;
    const int klo_h = klo + off;
    const int pad_h = 32 * d.n_words - off;
    const uint32_t nib = (uint32_t)off;
    // LDS address of the structure (its tables first)
    const uint32_t lds_base =
        (uint32_t)(size_t)(const __attribute__((address_space(3))) unsigned char*)smem + sm_off;

    float acc[kPairSlots];
#pragma unroll
    for (int i = 0; i < kPairSlots; ++i) acc[i] = 0.f;
    // groups of eight segments staged so far (uniform over the block): the partial sums are folded
    // after every kFlushGroups of them, which always ends a chunk (a chunk holds kChunk / 8 groups)
    static_assert(kFlushGroups % (kChunk / kGroup8) == 0, "folds fall at chunk ends");
    int64_t groups_done = 0;
    bool flushed = false;
    float* out = d.wsum_out + ((int64_t)s * d.n_bin + b) * d.n_f0;
    const int nf = d.n_f0;
    auto flush = [&]() {
        // the lane's offset taken opaque here, so that the 46 per-lane store addresses and bounds
        // are formed in the (rare) fold and not held in registers across the group loop
        int o = off;
        asm volatile("" : "+v"(o));
        float* po = out + o;
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) {
                    if (w == 2 && jb == 3 && t >= 2) continue;
                    const int sl = pair_slot(w, t, jb);
                    const int i = 32 * w + 8 * jb + t;
                    if (i + o < nf) po[i] = flushed ? po[i] + acc[sl] : acc[sl];
                    acc[sl] = 0.f;
                }
        flushed = true;
    };
    bool bad_range = claim_bad, bad_model = false;
    // the rows' zero padding, which the chunks' copies leave as it is
    for (int e = tid; e < kChunk * kRowPad; e += lanes) row[(e / kRowPad) * nwp + d.n_words + (e % kRowPad)] = 0u;

    for (int64_t j0 = 0; j0 < d.n_seg; j0 += kChunk) {
        const int nj = (int)min((int64_t)kChunk, d.n_seg - j0);
        const int ng8 = (nj + kGroup8 - 1) / kGroup8;
        const int ng = 2 * ng8;
        groups_done += ng8;
        // (form for proven windows on the circular track: the lane's first kPreWords row words
        // are loaded before the barrier, so that their latency overlaps the wait for the other
        // waves' groups; they are stored below)
        const int n_src = nj * d.n_words;
        const uint32_t* src = d.bits + j0 * d.n_words;
        uint32_t pre[(kProven && !kEcc) ? kPreWords : 1];
        if constexpr (kProven && !kEcc) {
#pragma unroll
            for (int k = 0; k < kPreWords; ++k) {
                const int e = tid + k * lanes;
                pre[k] = e < n_src ? src[e] : 0u;
            }
        }
        __syncthreads();
        for (int jj = tid; jj < ng * kGroup; jj += lanes) {
            const int64_t J = j0 + min(jj, nj - 1);
            double sp, cp;
            track_sincos(W * d.t_mid[J], sp, cp);
            double D = doppler_factor(d.v + 3 * J, nx, ny, nz);
            if constexpr (kProven) {
                // |v . n| <= |v/c| of the proof (unit n; slack for the rounding of D), finite phase
                if (!((fabs(D - 1.0) <= d.v_claim * (1.0 + 1e-9) + 1e-15) & (fabs(cp) <= 1.0) & (fabs(sp) <= 1.0))) {
                    bad_range = true;
                    D = 1.0;
                    cp = 0.0;
                    sp = 0.0;
                }
            }
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
        // The rows' data words (their kRowPad zero words are written once, before the first chunk):
        // word e of the chunk's rows is word e of the item's rows from segment j0 on (zero past
        // segment nj, the last group's padding) and goes to word wd of row jj (e = jj nw + wd),
        // stepped without a division.  In the form for proven windows on the circular track the
        // lane's first kPreWords words are all loaded before any is stored, so that their
        // latencies overlap (one after another they cost the batched launch 2 %); the other forms
        // keep one load per store, which holds their registers where they were.
        {
            const int nw = d.n_words;
            const int n_e = ng * kGroup * nw;
            int jj = tid / nw, wd = tid - jj * nw;
            const int dq = lanes / nw, dr = lanes - dq * nw;
            if constexpr (kProven && !kEcc) {
#pragma unroll
                for (int k = 0; k < kPreWords; ++k) {
                    if (tid + k * lanes < n_e) row[jj * nwp + wd] = pre[k];
                    jj += dq;
                    wd += dr;
                    if (wd >= nw) { wd -= nw; ++jj; }
                }
                for (int e = tid + kPreWords * lanes; e < n_e; e += lanes) {
                    row[jj * nwp + wd] = e < n_src ? src[e] : 0u;
                    jj += dq;
                    wd += dr;
                    if (wd >= nw) { wd -= nw; ++jj; }
                }
            } else {
                for (int e = tid; e < n_e; e += lanes) {
                    row[jj * nwp + wd] = jj < nj ? d.bits[(j0 + jj) * nw + wd] : 0u;
                    jj += dq;
                    wd += dr;
                    if (wd >= nw) { wd -= nw; ++jj; }
                }
            }
        }
        // The 256-entry tables, 32 entries (two high nibbles) per work item: T8[16 h + l] =
        // Tlo[l] + Thi[h], each half's subset sum taken in segment order from +0 (as a sum over the
        // set bits, one weight at a time, would give it).
        for (int it = tid; it < ng8 * 8; it += lanes) {
            const int g = it >> 3, k8 = it & 7;
            float w8[kGroup8];
#pragma unroll
            for (int u = 0; u < kGroup8; ++u) {
                const int jj = g * kGroup8 + u;
                w8[u] = jj < nj ? (wrow ? wrow[j0 + jj] : 1.f) : 0.f;
            }
            float lo[16];
            lo[0] = 0.f;
#pragma unroll
            for (int u = 0; u < kGroup; ++u)
#pragma unroll
                for (int l = 0; l < (1 << u); ++l) lo[(1 << u) + l] = lo[l] + w8[u];
            // high nibbles 2 k8 (bit 0 clear) and 2 k8 + 1: bits 1..3 from k8
            const float s5 = (k8 & 1) ? w8[5] : 0.f;
            const float s6 = (k8 & 2) ? w8[6] : 0.f;
            const float s7 = (k8 & 4) ? w8[7] : 0.f;
            const float hi0 = ((0.f + s5) + s6) + s7;
            const float hi1 = (((0.f + w8[4]) + s5) + s6) + s7;
            float4* dst = reinterpret_cast<float4*>(sm.T8 + g * 256 + k8 * 32);
#pragma unroll
            for (int q4 = 0; q4 < 8; ++q4) {
                const float hv = q4 < 4 ? hi0 : hi1;
                const int l = (q4 & 3) * 4;
                dst[q4] = make_float4(lo[l] + hv, lo[l + 1] + hv, lo[l + 2] + hv, lo[l + 3] + hv);
            }
        }
        __syncthreads();
        if (!active || claim_bad) continue;

        // this lane's rows: segments 4h .. 4h + 3 of group 0, then eight rows further per group
        const uint32_t* lrow = row + 4 * h * nwp;
        for (int g8 = 0; g8 < ng8; ++g8, lrow += kGroup8 * nwp) {
            const int hg = 2 * g8 + h;
            uint32_t mk[kGroup][3];
            BandTrack tr[kGroup];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const int jj = hg * kGroup + u;
                const double G = tile_G<kEcc>(sm.DC[jj], sm.DS[jj], sm.D[jj], kEcc ? sm.DC2[jj] : 0.0,
                                              kEcc ? sm.DS2[jj] : 0.0, Ac, As, Ac2, As2);
                tr[u] = band_track<kProven>(G, F0, FL, klo, klo + d.n_bins, last, bad_range, bad_model);
            }
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const int at = tr[u].ok ? tr[u].kf - klo_h : pad_h;   // (always ok when proven)
                const uint32_t* rw = lrow + u * nwp + (at >> 5);
                const uint32_t w0 = rw[0], w1 = rw[1], w2 = rw[2], w3 = rw[3];
                mk[u][0] = __builtin_amdgcn_alignbit(w1, w0, at);
                mk[u][1] = __builtin_amdgcn_alignbit(w2, w1, at);
                mk[u][2] = __builtin_amdgcn_alignbit(w3, w2, at);
            }
#pragma unroll
            for (int u = 0; u < kGroup; ++u)
                if (tr[u].ok && tr[u].span != last) band_step(tr[u], F0, last, mk[u][0], mk[u][1], mk[u][2], off);

            // Words from the top (w = 2) down, so that only the word above stays live.  A[t]: the
            // transposed masks; Z[t]: this lane's low nibbles with the partner's high ones.
            const uint32_t T8 = lds_base + (uint32_t)g8 * 1024u;   // LDS address of the group's table
            uint32_t Zup[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int w = 2; w >= 0; --w) {
                uint32_t x0 = mk[0][w], x1 = mk[1][w], x2 = mk[2][w], x3 = mk[3][w];
                uint32_t y0, y1, y2, y3;
                // bit pairs at distance 2 (segments 0, 2 and 1, 3), then single bits at distance 1
                y0 = (x0 & 0x33333333u) | ((x2 << 2) & 0xccccccccu);
                y2 = ((x0 >> 2) & 0x33333333u) | (x2 & 0xccccccccu);
                y1 = (x1 & 0x33333333u) | ((x3 << 2) & 0xccccccccu);
                y3 = ((x1 >> 2) & 0x33333333u) | (x3 & 0xccccccccu);
                x0 = (y0 & 0x55555555u) | ((y1 << 1) & 0xaaaaaaaau);
                x1 = ((y0 >> 1) & 0x55555555u) | (y1 & 0xaaaaaaaau);
                x2 = (y2 & 0x55555555u) | ((y3 << 1) & 0xaaaaaaaau);
                x3 = ((y2 >> 1) & 0x55555555u) | (y3 & 0xaaaaaaaau);
                const uint32_t A[4] = {x0, x1, x2, x3};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const uint32_t p = pair_swap(A[t]);
                    const uint32_t Z = (A[t] & 0x0f0f0f0fu) | (p & 0xf0f0f0f0u);
                    // bytes j of x: bin 32 w + 8 j + 4 h + t (lane 1 takes the word one nibble down)
                    const uint32_t x = __builtin_amdgcn_alignbit(Zup[t], Z, nib);
                    Zup[t] = Z;
                    const uint32_t ye = x & 0x00ff00ffu;                            // bytes 0 and 2
                    const uint32_t yo = __builtin_amdgcn_perm(x, x, 0x0c030c01u);   // bytes 1 and 3
                    acc[pair_slot(w, t, 0)] += lds_at(lut_addr_lo(ye, T8));
                    acc[pair_slot(w, t, 1)] += lds_at(lut_addr_lo(yo, T8));
                    acc[pair_slot(w, t, 2)] += lds_at(lut_addr_hi(ye, T8));
                    if (!(w == 2 && t >= 2)) acc[pair_slot(w, t, 3)] += lds_at(lut_addr_hi(yo, T8));
                }
            }
        }
        if (groups_done % kFlushGroups == 0) flush();
    }
    if (bad_range) raise_status(d.status, BSH_STATUS_RANGE);
    if (bad_model) raise_status(d.status, BSH_STATUS_MODEL);
    if (active && (groups_done % kFlushGroups != 0 || !flushed)) flush();
}

// kMode % kEccMode: 0 = select-and-add, weighted sums only; 1 = select-and-add with counts;
// 2 = table.  kMode >= kEccMode: the same on the ELL1 track of the item's eccentricity pair.
template <int kMode, int kChunk>
constexpr size_t fixed_smem_bytes()
{
    constexpr bool kEcc = mode_ecc(kMode);
    constexpr size_t b = mode_table(kMode) ? sizeof(TileSmemLut<kChunk, kEcc>) : sizeof(TileSmem<kChunk, kEcc>);
    return (b + 15) & ~(size_t)15;
}

// The tile's LDS: the rows, then the fixed structure.
template <int kMode, int kChunk>
__device__ __forceinline__ void run_tile(const ItemDesc& d, int s, int ip, int64_t tile, unsigned char* smem)
{
    constexpr int kM = mode_base(kMode) % kEccMode;
    constexpr bool kEcc = mode_ecc(kMode);
    // rows at offset 0 (a row's words are then addressed by the read instructions' own offsets);
    // the structure follows the item's rows (a multiple of 512 bytes)
    uint32_t* row = reinterpret_cast<uint32_t*>(smem);
    const uint32_t sm_off = (uint32_t)kChunk * (uint32_t)(d.n_words + kRowPad) * 4u;
    unsigned char* st = smem + sm_off;
    if constexpr (kM == 2) {
        using Lut = TileSmemLut<kChunk, kEcc>;
        static_assert(offsetof(Lut, T8) == 0, "tables first");
        count_tile_pair<kChunk, kEcc, mode_proven(kMode)>(d, s, ip, tile, *reinterpret_cast<Lut*>(st), row, smem,
                                                          sm_off);
    } else {
        count_tile<kM == 1, kChunk, kEcc>(d, s, ip, tile, *reinterpret_cast<TileSmem<kChunk, kEcc>*>(st), row);
    }
}

// Launch bound: the least waves per SIMD the register allocation must allow.  The circular
// table variant comes out at 155-168 registers, three waves, with the bound at two: bounding it
// to three makes the ILP scheduler keep two table reads in flight instead of eight (22 % slower).
// The ELL1 table variant needs 171-183 registers unbounded (two waves); bounded to three it
// spills a few and is faster (200 Hz band 2.05 -> 1.88 ms, batched launch 651 -> 462 ms on 256
// items).  The select variants hold 90 partial sums (and counts): one.
template <int kMode>
constexpr int min_blocks() { return mode_base(kMode) == kEccMode + 2 ? 3 : (mode_table(kMode) ? 2 : 1); }

// Instantiate a kernel template for every (mode, chunk) of the select variants (modes 0, 1 and
// their ELL1 forms 3, 4) or of the table variant (modes 2, 5) and call f with the chosen one.  The
// two families are compiled in different sources (bsh_count_table.hip holds the table variant).
#define BSH_DISPATCH_SELECT(MODE, CHUNK, F)                                                   \
    switch ((MODE) * 1000 + (CHUNK)) {                                                        \
    case 128: F(0, 128); break;                                                               \
    case 256: F(0, 256); break;                                                               \
    case 512: F(0, 512); break;                                                               \
    case 1128: F(1, 128); break;                                                              \
    case 1256: F(1, 256); break;                                                              \
    case 1512: F(1, 512); break;                                                              \
    case 3128: F(3, 128); break;                                                              \
    case 3256: F(3, 256); break;                                                              \
    case 3512: F(3, 512); break;                                                              \
    case 4128: F(4, 128); break;                                                              \
    case 4256: F(4, 256); break;                                                              \
    case 4512: F(4, 512); break;                                                              \
    default: return fail_inval("kernel mode / chunk");                                        \
    }

#define BSH_DISPATCH_TABLE(MODE, CHUNK, F)                                                    \
    switch ((MODE) * 1000 + (CHUNK)) {                                                        \
    case 2128: F(2, 128); break;                                                              \
    case 2256: F(2, 256); break;                                                              \
    case 2512: F(2, 512); break;                                                              \
    case 5128: F(5, 128); break;                                                              \
    case 5256: F(5, 256); break;                                                              \
    case 5512: F(5, 512); break;                                                              \
    case 10128: F(10, 128); break;                                                            \
    case 10256: F(10, 256); break;                                                            \
    case 10512: F(10, 512); break;                                                            \
    case 13128: F(13, 128); break;                                                            \
    case 13256: F(13, 256); break;                                                            \
    case 13512: F(13, 512); break;                                                            \
    default: return fail_inval("kernel mode / chunk");                                        \
    }

inline bool is_table_mode(int mode) { return mode_table(mode); }

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
    case 10128: BSH_FIXED_SMEM(10, 128); break;
    case 10256: BSH_FIXED_SMEM(10, 256); break;
    case 10512: BSH_FIXED_SMEM(10, 512); break;
    case 13128: BSH_FIXED_SMEM(13, 128); break;
    case 13256: BSH_FIXED_SMEM(13, 256); break;
    case 13512: BSH_FIXED_SMEM(13, 512); break;
    default: return 0;
    }
    return fixed + row_bytes(chunk, n_words);
}
#undef BSH_FIXED_SMEM

}  // namespace bsh
