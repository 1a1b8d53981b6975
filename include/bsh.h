/*
 * bsh.h -- C ABI of libbsh.so, the MI355X (gfx950) semi-coherent Hough search for
 * continuous gravitational waves from neutron stars in circular binary orbits
 * (Covas & Sintes, "BinarySkyHough", arXiv:1904.04873).
 *
 * The search evaluates, for every template theta = (sky n, f0, a_p, P, t_asc) and every
 * short-FFT segment J, the frequency track of eq:frequencyevoFinal (Sec. II) in the
 * product form used by eq:hough1 (Sec. IV.B):
 *
 *     x_J = f(t_J) Tc = F (1 + v_J.n) (1 - a_p W cos(W (t_J - t_asc))),   F = f0 Tc, W = 2 pi / P
 *
 * rounds it to the nearest DFT bin k_J = floor(x_J + 1/2) (bin k <-> frequency k/Tc, Sec. IV.A),
 * and sums a per-segment quantity along the track: the weighted peak (stage 1, number count
 * of eq:hough2) or the weighted normalized power (stage 2, eq:hough3).
 *
 * Conventions shared by every call
 *   - Pointers are device pointers unless a field name ends in _host.  The caller allocates
 *     every buffer and keeps it alive until the stream has finished the call.
 *   - Every call that launches work is asynchronous on `stream` (a hipStream_t, NULL = the
 *     null stream) and returns once the work is queued.
 *   - Return value: BSH_OK or a negative code.  BSH_EINVAL (bad pointer, shape or
 *     non-finite parameter) and BSH_ERANGE found on the host are reported before anything
 *     is launched.  BSH_EHIP reports a HIP runtime error; bsh_last_error() gives the text
 *     (thread-local, valid until the next call on the same thread).
 *   - `status` (where present) is a device int32 that the caller zeroes and later reads:
 *     kernels OR in BSH_STATUS_RANGE when a track leaves the staged row [k_lo, k_lo+n_bins)
 *     or, in a stage-1 launch whose window the host has proven (see bsh_hough_count_ex), when a
 *     segment's |v.n| or a template's a_p W (1 + e) exceeds that proof's bound (no track is
 *     clamped into the row; the outputs of that call are then not meaningful) and
 *     BSH_STATUS_MODEL when a track's drift across the f0 band exceeds one
 *     bin (parameters outside the model's validity), and BSH_STATUS_INPUT when a candidate
 *     names a sky pixel outside [0, n_sky) (that candidate's outputs are then 0) or a
 *     post-processing input is invalid (a significance that is not finite and positive, or a
 *     cluster label that does not name a root).
 *   - Template index of the stage-1 grid (f0 fastest):
 *         idx = ((s * n_bin) + b) * n_f0 + i,   b = tasc_off[ia * n_per + ip] + j
 *     with s the sky pixel, i the f0 bin (F = k0 + i), ia/ip the a_p/P indices and j the
 *     t_asc point of that (a_p, P) cell.
 *   - Candidates (stage 2) are rows of cand_params[n][4] = (F = f0 Tc, a_p in light-seconds,
 *     P in s, t_asc in s) with a sky pixel cand_sky[n]; they need not lie on the grid.
 *     Taking F rather than f0 keeps grid templates bit-identical between the two stages.
 *
 * No exception crosses this ABI.  No call allocates device memory except bsh_plan_create,
 * which allocates the plan's own tables, queue and top-k workspaces (released by
 * bsh_plan_destroy); every other call works in caller-given buffers and workspaces whose sizes
 * the *_workspace functions give.
 */
#ifndef BSH_H_
#define BSH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BSH_OK 0
#define BSH_EINVAL (-1)
#define BSH_ERANGE (-2)
#define BSH_EHIP (-3)
#define BSH_ENOMEM (-4)

#define BSH_STATUS_RANGE 1
#define BSH_STATUS_MODEL 2
#define BSH_STATUS_INPUT 4

#define BSH_MAX_PER 256     /* largest number of orbital periods in one grid */
#define BSH_MAX_F0 90       /* stage-1 f0 bins per band (a 0.1 Hz band at Tc = 900 s) */
#define BSH_MAX_WORDS 16    /* longest staged peakgram row: 512 bins */

typedef void* bsh_stream;

/* Per-segment inputs of one work item (Sec. IV.A).  n_seg segments of length t_coh. */
typedef struct bsh_segments {
    int64_t n_seg;
    double t_coh;               /* coherent time Tc (s), > 0 */
    const double* t_mid;        /* [n_seg] segment mid-times (s), same origin as t_asc */
    const double* v_over_c;     /* [n_seg][3] detector velocity / c, same frame as the sky vectors */
    const float* weight;        /* [n_seg] or [n_sky][n_seg] segment weights (eq:weigths) */
    int32_t weight_per_sky;     /* 1: weight is [n_sky][n_seg] */
    int32_t n_bins;             /* staged row width, 1 .. 32*BSH_MAX_WORDS */
    int64_t k_lo;               /* absolute bin of column 0 */
    const uint32_t* peak_bits;  /* [n_seg][(n_bins+31)/32] peakgram, bit b of word w = column 32w+b;
                                   NULL for calls that read only power */
    const float* power;         /* [n_seg][n_bins] normalized power (eq:HoughPower); NULL for
                                   calls that read only peak_bits */
    double v_max_host;          /* max |v/c| over the segments, or 0 if unknown (host value;
                                   enables the host-side window check) */
} bsh_segments;

/* Stage-1 template grid of one band (Sec. IV.C, resolution and ranges). */
typedef struct bsh_grid {
    int32_t n_sky;
    const double* sky;            /* [n_sky][3] unit vectors */
    int64_t k0;                   /* first f0 bin: f0_i = (k0 + i) / Tc */
    int32_t n_f0;                 /* 1 .. BSH_MAX_F0 */
    int32_t n_ap;
    int32_t n_per;                /* 1 .. BSH_MAX_PER */
    const double* a_p;            /* [n_ap] projected semi-major axes (light-seconds) */
    const double* period;         /* [n_per] orbital periods (s) */
    const int64_t* tasc_off;      /* [n_ap*n_per+1] prefix offsets of each cell's t_asc points */
    const double* t_asc;          /* [n_bin] times of ascending node (s) */
    const double* a_p_host;       /* host copies of the three small tables above */
    const double* period_host;
    const int64_t* tasc_off_host;
    double ecc_c, ecc_s;          /* (e cos w, e sin w) of every template of the grid: the
                                     low-eccentricity (ELL1) track of eq:frequencyevo (Sec. II),
                                     see bsh_power_stat_ecc; (0, 0) is the circular track, bit for
                                     bit.  A search over eccentricity runs one grid per pair.
                                     Finite, with e cos w ^2 + e sin w ^2 < 0.25. */
} bsh_grid;

/* Numeric ranges from which bsh_grid_build enumerates one band's grid. */
typedef struct bsh_grid_spec {
    int64_t k0;
    int32_t n_f0;
    double t_coh;
    double ap_lo, ap_hi;          /* a_p values: lo + i*((hi-lo)/(n-1)), last = hi */
    int32_t n_ap;
    double per_lo, per_hi;        /* P values (s), same rule */
    int32_t n_per;
    int32_t tasc_fixed;           /* > 0: that many t_asc points in every cell */
    double tasc_rule_m;           /* else N = clamp(ceil(m * Tc * f_hi * a_p * W), min, max) */
    int32_t tasc_min, tasc_max;
} bsh_grid_spec;

/* Library version (major*10000 + minor*100 + patch). */
int bsh_version(void);

/* Text of the last error on this thread ("" if none). */
const char* bsh_last_error(void);

/*
 * Template-bank enumeration for one band (host only; Sec. IV.C):
 *   f0 on bin centres (delta f = 1/Tc); a_p and P on inclusive uniform lists;
 *   t_asc_j = t_mid - P/2 + j (P/N) so that t_mid - P/2 <= t_asc < t_mid + P/2;
 *   N per cell fixed, or from the spacing of eq:binaryres as N = m Tc f_hi a_p W, evaluated
 *   left to right and clamped (f_hi = (k0 + n_f0)/Tc).
 * Writes host arrays a_p[n_ap], period[n_per], tasc_off[n_ap*n_per+1] and, if t_asc is not
 * NULL, t_asc[*n_bin_out] (BSH_ENOMEM if t_asc_cap is too small).  Cells are a_p-major.
 */
int bsh_grid_build(const bsh_grid_spec* spec, double t_mid, double* a_p, double* period,
                   int64_t* tasc_off, double* t_asc, int64_t t_asc_cap, int64_t* n_bin_out);

/*
 * Normalized power (eq:HoughPower, Sec. IV.A): rho_k = P_k / <n_k>^2 with the noise level
 * <n_k>^2 = median(P_{k-m} .. P_{k+m}) / beta, window = 2m+1 (odd; the paper uses 101) and
 * beta = sum_{i=m+1}^{2m+1} 1/i, the expected median of 2m+1 unit exponentials, so that noise
 * normalizes to unit mean.  raw [n_seg][n_raw] un-normalized SFT powers (n_raw <= 4096);
 * rho_out [n_seg][n_raw - 2m], column c centred on raw column c + m;
 * rho = (float)((P * beta) / median) evaluated in double precision.  A window that holds a NaN
 * has a NaN median, so its output is NaN.
 */
int bsh_normalize(const float* raw, int64_t n_seg, int32_t n_raw, int32_t window, float* rho_out,
                  bsh_stream stream);

/*
 * Peakgram (Sec. IV.A): bits[J][w] bit b = [power[J][32w+b] > rho_th], compared in double
 * precision; unused high bits of the last word are zero.
 * power [n_seg][n_bins] float32, bits [n_seg][(n_bins+31)/32] uint32.
 */
int bsh_peakgram(const float* power, int64_t n_seg, int32_t n_bins, double rho_th,
                 uint32_t* bits, bsh_stream stream);

/*
 * Stage-1 weighted number count over every template of `grid` (Sec. IV.C eq:hough2; the
 * GPU loop K1 of Sec. IV.B), reading seg->peak_bits.
 *   wsum_out [n_sky*n_bin*n_f0]: sum_J w_J p_J  (FP32, at least 64 partial sums per template)
 *   count_out (may be NULL): sum_J p_J (uint32)
 * Either output may be NULL but not both.  Requires n_per <= BSH_MAX_PER, n_f0 <= BSH_MAX_F0.
 * A grid with a nonzero (ecc_c, ecc_s) is counted on the ELL1 track of bsh_power_stat_ecc.
 */
int bsh_hough_count(const bsh_segments* seg, const bsh_grid* grid, uint32_t* count_out,
                    float* wsum_out, int32_t* status, bsh_stream stream);

/*
 * Same as bsh_hough_count with an explicit tile shape and accumulation variant: `lanes` binary
 * templates per block (64, 128, 256 or 512), `chunk` segments staged in LDS per pass (128, 256
 * or 512), and `variant`:
 *   BSH_VARIANT_SELECT  every peak bit selects its weight, which is added (and counted);
 *   BSH_VARIANT_TABLE   segments in groups of eight, whose 256 subset sums of weights are looked
 *                       up with the eight peak bits as index;
 *   BSH_VARIANT_AUTO    the table (the default of bsh_hough_count).
 * Counts with the table (AUTO or TABLE, fewer than 2^24 segments) are the table's sums with every
 * weight one, exact in FP32 and so the same counts bit for bit, computed in a launch of their own
 * (after the weighted sums' launch when both are asked for).  Results do not depend on the tile
 * shape; the two variants' weighted sums agree to FP32 rounding, their counts exactly.
 * When seg->v_max_host > 0 the host bounds every track: |G - 1| <= v + A + v A with v =
 * v_max_host and A = max a_p W (1 + e) over the grid.  If the staged row covers that bound (else
 * BSH_ERANGE, as always) and the band's drift (n_f0 - 1)(v + A + v A) is below half a bin, the
 * table variant runs without its per-track range and drift tests: instead every staged segment's
 * |v.n| and every template's a_p W (1 + e) are tested against v and A (device copies against the
 * host's bound), and a violation raises BSH_STATUS_RANGE.  Results are the same bit for bit.
 */
#define BSH_VARIANT_AUTO 0
#define BSH_VARIANT_SELECT 1
#define BSH_VARIANT_TABLE 2

/* 1 when the table variant's launches for (seg, grid) take the form for proven windows (see
 * above), 0 when they test every track, negative on invalid arguments.  Host-only. */
int32_t bsh_count_window_proven(const bsh_segments* seg, const bsh_grid* grid);
int bsh_hough_count_ex(const bsh_segments* seg, const bsh_grid* grid, int32_t lanes, int32_t chunk,
                       int32_t variant, uint32_t* count_out, float* wsum_out, int32_t* status,
                       bsh_stream stream);

/*
 * Stage 1 with its per-band top-list and bounded memory (Sec. IV.C: only the best N_C
 * templates of a band go on to the second stage, so the full map is never needed; eq:RAM1
 * counts the map memory this avoids).  The grid's sky pixels are counted in passes of
 * sky_per_pass pixels (0: all at once) into a map inside the workspace; after each pass the
 * pass's top-k is merged into the running list, which is exact because the best k of a union
 * are among the best k of each part.  Results equal bsh_topk over the full bsh_hough_count
 * map (default tile and accumulation), bit for bit.
 *   spec->k: list length; out_score[k], out_index[k] as bsh_topk (template index as above;
 *   the tail is -inf / -1 when the grid has fewer than k templates).
 *   ws / ws_bytes: at least bsh_hough_count_topk_workspace(grid, spec) bytes: one pass's map
 *   (sky_per_pass x n_bin x n_f0 floats) plus O(k).  When there are several passes, each must
 *   hold at least k templates (BSH_EINVAL otherwise).
 */
typedef struct bsh_topk_spec {
    int32_t k;
    int32_t sky_per_pass;
} bsh_topk_spec;

size_t bsh_hough_count_topk_workspace(const bsh_grid* grid, const bsh_topk_spec* spec);
int bsh_hough_count_topk(const bsh_segments* seg, const bsh_grid* grid, const bsh_topk_spec* spec,
                         float* out_score, int64_t* out_index, void* ws, size_t ws_bytes,
                         int32_t* status, bsh_stream stream);

/*
 * Exact top-k under the total order (score descending, index ascending) (Sec. IV.C
 * top-lists).  score [n]; index [n] int64 or NULL for 0..n-1 (indices must be distinct and
 * non-negative).
 * Writes out_score[k], out_index[k] sorted; if n < k the tail is -inf / -1.
 * ws / ws_bytes: device workspace of at least bsh_topk_workspace(n, k) bytes.
 * Scores must not be NaN.  Merging per-item lists is a call with their concatenation.
 */
size_t bsh_topk_workspace(int64_t n, int32_t k);
int bsh_topk(const float* score, const int64_t* index, int64_t n, int32_t k,
             float* out_score, int64_t* out_index, void* ws, size_t ws_bytes, bsh_stream stream);

/*
 * Many independent top-k lists in the same launches: segment g is score[offsets[g] ..
 * offsets[g+1]) and its list goes to out_score[g*k .. g*k+k), out_index likewise.
 * offsets: device [n_segs+1] and a host copy (for launch sizing); each segment shorter than
 * 2^32 - 1.  index NULL: entry e of segment g gets the implicit index
 * (g << index_shift) | (e - offsets[g]) (just the position when index_shift is 0).
 * Workspace: bsh_topk_segmented_workspace(n_segs, k) bytes.  n_segs <= 65535.
 * Given at least bsh_topk_segmented_candidate_workspace(n_segs, k) bytes (for n_segs >= 2,
 * 12 bytes per segment and candidate slot more: C = 32768 slots for k <= 2048, else 8 k rounded
 * up to a multiple of 1024 if that is larger), a call whose longest segment exceeds C entries
 * first selects candidates: per segment, the key of a set rank among 32768 sampled entries
 * (512 runs of 64 consecutive ones, run r from r (length - 64) / 511, integer division) as a
 * threshold aiming at C / 4 entries at or above it, one pass that copies those entries (up to
 * C), and the selection over that copy; a segment whose copy holds fewer than min(k, length) or
 * overflowed takes the ordinary passes instead.  The lists are the same either way, bit for bit.
 */
size_t bsh_topk_segmented_workspace(int32_t n_segs, int32_t k);
size_t bsh_topk_segmented_candidate_workspace(int32_t n_segs, int32_t k);
int bsh_topk_segmented(const float* score, const int64_t* index, const int64_t* offsets,
                       const int64_t* offsets_host, int32_t n_segs, int32_t k, int32_t index_shift,
                       float* out_score, int64_t* out_index, void* ws, size_t ws_bytes,
                       bsh_stream stream);

/*
 * bsh_topk without allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * results as bsh_topk, bit for bit, but no workspace argument: the workspace is a static device
 * array of bsh_topk_noalloc_max_bytes() bytes (8 MiB; enough for k up to about 2.3e5), one per
 * GPU, held until the process ends.  k beyond what it holds: BSH_ENOMEM, nothing launched.
 * The call allocates nothing and calls no allocating routine.  Every call on one GPU shares that
 * GPU's array (each call clears the state it needs on the stream first), so calls that overlap
 * in time on one GPU (on different streams, or from different threads) race and must not be
 * issued; calls on different GPUs are independent.
 */
size_t bsh_topk_noalloc_max_bytes(void);
int bsh_topk_noalloc(const float* score, const int64_t* index, int64_t n, int32_t k,
                     float* out_score, int64_t* out_index, bsh_stream stream);

/*
 * Stage-1 template index -> candidate row (sky pixel, F = k0+i, a_p, P, t_asc).
 * index [n] int64 (entries < 0 give sky -1 and zero parameters); cand_sky [n]; cand_params [n][4].
 */
int bsh_decode_templates(const bsh_grid* grid, const int64_t* index, int64_t n,
                         int32_t* cand_sky, double* cand_params, bsh_stream stream);

/*
 * Stage-2 statistic on the exact track for n candidates (Sec. IV.C eq:hough3; the GPU
 * loop K2 of Sec. IV.B).  sky [n_sky][3]; candidates as above; with weight_per_sky the
 * weight row of the candidate's pixel is used.
 *   mode 0: P_out[c] = sum_J w_J rho_{J,k_J} (nearest bin, needs seg->power); when
 *           seg->peak_bits is set, count_out / wsum_out (each may be NULL) get the
 *           stage-1 count and weighted count of the same track;
 *   mode 1: P_out[c] = sum_J w_J ((1-a) rho_{J,k'} + a rho_{J,k'+1}), k' = floor(x_J),
 *           a = x_J - k' (bin-interpolated extension, piecewise linear in the parameters).
 * P_out may be NULL in mode 0 when only counts are wanted.
 */
int bsh_power_stat(const bsh_segments* seg, const double* sky, int32_t n_sky, const int32_t* cand_sky,
                   const double* cand_params, int64_t n, int32_t mode, float* P_out,
                   uint32_t* count_out, float* wsum_out, int32_t* status, bsh_stream stream);

/*
 * Vector-Jacobian product of the mode-1 statistic:
 *   grad_params[c][q] = grad_P[c] * dP_lin/dtheta_q,  theta = (F, a_p, P, t_asc), FP64.
 * At an exact integer x the right-hand interval is used.  grad_P may be NULL (all ones).
 */
int bsh_power_stat_grad(const bsh_segments* seg, const double* sky, int32_t n_sky,
                        const int32_t* cand_sky,
                        const double* cand_params, int64_t n, const double* grad_P,
                        double* grad_params, int32_t* status, bsh_stream stream);

/*
 * The mode-1 statistic (the bin-interpolated extension of Sec. IV.C eq:hough3) and its
 * vector-Jacobian product in one pass over the segments (both come from the same track and
 * the same two row values per segment), for gradient ascent of P_lin, which needs both every
 * step:
 *   P_out[c] = P_lin of bsh_power_stat mode 1 (its FP32 terms summed in runs as there, the
 *              partial sums of the candidate's threads then added in FP64: equal to the
 *              mode-1 result within the FP32 summation bound, not bit for bit);
 *   grad_params as bsh_power_stat_grad, bit for bit.
 * P_out and grad_params must not be NULL; grad_P may be NULL (all ones).  Status bits,
 * errors and the right-hand derivative at integer x are those of bsh_power_stat_grad.
 */
int bsh_power_stat_value_and_grad(const bsh_segments* seg, const double* sky, int32_t n_sky,
                                  const int32_t* cand_sky, const double* cand_params, int64_t n,
                                  const double* grad_P, float* P_out, double* grad_params,
                                  int32_t* status, bsh_stream stream);

/*
 * Stage-2 statistic on the low-eccentricity (ELL1) track of eq:frequencyevo (Sec. II), for
 * orbits the circular model only approximates (Sec. IV.E bounds when that matters):
 *   x = F (1 + v.n) (1 - a_p W [cos psi + (e cos w) cos 2psi - (e sin w) sin 2psi]),
 *   psi = W (t - t_asc).
 * With C2, S2 = cos, sin of 2 W t (from those of W t by the double-angle formulas), the
 * bracket's eccentric part is C2 A_c2 + S2 A_s2 with A_c2 = a_p W (ec c2 + es s2),
 * A_s2 = a_p W (ec s2 - es c2), c2, s2 = cos, sin of 2 W t_asc; the track is evaluated as
 * G = [circular G] - fma(D C2, A_c2, (D S2) A_s2), the order the stage-1 count uses for a grid
 * with an eccentricity pair, so that grid templates select the same bins in both stages.
 * cand_params [n][6] = (F, a_p, P, t_asc, e cos w, e sin w); modes and outputs as
 * bsh_power_stat (counts of the same track in mode 0 when seg->peak_bits is set; P_out may then
 * be NULL).  With zero eccentricity every output equals bsh_power_stat's bit for bit.
 */
int bsh_power_stat_ecc(const bsh_segments* seg, const double* sky, int32_t n_sky,
                       const int32_t* cand_sky, const double* cand_params, int64_t n, int32_t mode,
                       float* P_out, uint32_t* count_out, float* wsum_out, int32_t* status,
                       bsh_stream stream);

/*
 * Vector-Jacobian product of the mode-1 statistic on the ELL1 track (the interpolated extension
 * of eq:hough3 on the track of bsh_power_stat_ecc), with respect to all six parameters:
 *   grad_params[c][q] = grad_P[c] * dP_lin/dtheta_q, theta = (F, a_p, P, t_asc, e cos w, e sin w),
 * FP64, [n][6].  With E = cos psi + ec cos 2psi - es sin 2psi and E' = dE/dpsi,
 *   dx/dF = D B, dx/da_p = -F D W E, dx/dP = F D a_p (W/P)(E + psi E'), dx/dt_asc = F D a_p W^2 E',
 *   dx/d(e cos w) = -F D a_p W cos 2psi, dx/d(e sin w) = F D a_p W sin 2psi.
 * P_out may be NULL; when given it also gets P_lin from the same pass (as
 * bsh_power_stat_value_and_grad).  grad_P may be NULL (all ones).  At zero eccentricity the first
 * four columns are bsh_power_stat_grad's within FP64 rounding.
 */
int bsh_power_stat_grad_ecc(const bsh_segments* seg, const double* sky, int32_t n_sky,
                            const int32_t* cand_sky, const double* cand_params, int64_t n,
                            const double* grad_P, float* P_out, double* grad_params, int32_t* status,
                            bsh_stream stream);

/*
 * Absolute bins k_J of each candidate's track: bins_out [n][n_seg] int32.  The same
 * evaluation as bsh_power_stat; for inspection and for placing injected signals.  No row
 * is read, so no window applies; a bad sky index gives bins of -1 and BSH_STATUS_INPUT.
 */
int bsh_track_bins(const bsh_segments* seg, const double* sky, int32_t n_sky, const int32_t* cand_sky,
                   const double* cand_params, int64_t n, int32_t* bins_out, int32_t* status,
                   bsh_stream stream);

/*
 * Batched stage 1 over many work items of uneven size (independent band x sky-patch jobs,
 * eq:cost of Sec. IV.F).  An item is one segment set, one band grid (index into grids[]) and
 * the pixels [sky_lo, sky_lo + n_sky) of that grid's sky table; items must be ordered by band.
 * Item i's stage-1 map (as bsh_hough_count would write it) goes to
 * maps[off_i .. off_i + n_sky*n_bin*n_f0) with off_i the running sum over earlier items;
 * bsh_items_map_floats gives the total.  Global template index of an item's entry at
 * position q of its map: (i << 40) | q.
 */
typedef struct bsh_item {
    bsh_segments seg;
    int32_t grid;
    int32_t sky_lo;
    int32_t n_sky;
    int32_t band;
} bsh_item;

typedef struct bsh_plan_opts {
    int32_t lanes;        /* tile shape as in bsh_hough_count_ex (0: default 256) */
    int32_t chunk;        /* (0: default 256) */
    int32_t k_item;       /* top-k of every item's map (0: maps only) */
    int32_t k_band;       /* top-k per band over its items' lists (0: none) */
    int32_t use_graph;    /* 1: capture one run in a HIP graph at creation, replay it */
    int32_t lpt;          /* 1: queue units longest-first */
    int32_t blocks;       /* persistent blocks (0: CUs x resident blocks per CU) */
    int32_t variant;      /* accumulation variant as in bsh_hough_count_ex */
    int32_t persistent;   /* 0: one block per unit of the queue, dispatched in queue order;
                             1: persistent blocks that pull units from an atomic queue counter;
                             < 0: the persistent blocks when as many of them are resident per CU
                             as blocks of the one-block-per-unit form, else one block per unit
                             (bsh_plan_persistent tells which) */
} bsh_plan_opts;

typedef struct bsh_plan bsh_plan;

int64_t bsh_items_map_floats(const bsh_item* items, int32_t n_items, const bsh_grid* grids,
                             int32_t n_grids);

/*
 * Build a plan: validates every item on the host, builds the unit queue (one unit per
 * item x pixel x period x tile) and, with use_graph, captures one run.  The plan owns its
 * device tables and top-k workspaces (allocated here, freed by bsh_plan_destroy); every
 * pointer passed in (items' tables, grids, maps, item lists [n_items][k_item], band lists
 * [n_bands][k_band], status) must stay valid for the plan's life.  Two runs of one plan, or
 * other work on the same arrays, must not overlap in time.
 *
 * Bounded memory: maps_floats may be smaller than bsh_items_map_floats (but not smaller than
 * the largest item's map); the items are then split, in order, into passes whose maps fit in
 * `maps` together, each pass one count launch followed by its items' lists, and `maps`
 * is reused (it then holds the last pass's maps after a run).  This needs k_item > 0; the item
 * and band lists are the same as with room for every map, because the best k of a band are
 * among the best k of each of its items.  At most 65535 items.
 */
int bsh_plan_create(const bsh_item* items, int32_t n_items, const bsh_grid* grids, int32_t n_grids,
                    int32_t n_bands, const bsh_plan_opts* opts, float* maps, int64_t maps_floats,
                    float* item_score, int64_t* item_index, float* band_score, int64_t* band_index,
                    int32_t* status, bsh_plan** plan);

/* One batched run: the count launch(es), per-item lists, per-band lists (one graph launch). */
int bsh_plan_run(bsh_plan* plan, bsh_stream stream);

/* The same results from one plain launch (plus its own top-k) per item, in item order. */
int bsh_plan_run_plain(bsh_plan* plan, bsh_stream stream);

/* The count launches of a run alone (every pass, no lists; not graph-captured):
 * the maps of the last pass, for timing the count kernel on its own. */
int bsh_plan_run_count(bsh_plan* plan, bsh_stream stream);

/* Number of queued units, blocks per launch (the persistent blocks, or the largest pass's unit
 * count with one block per unit), launch form (1: persistent blocks, 0: one block per unit) and
 * passes of a plan (-1 for NULL).  bsh_plan_proven: 1 when the count launches take the form of
 * the table kernel for proven windows, i.e. every item with segments gave v_max_host > 0 and a
 * staged row that covers its tracks' bound with the band's drift below half a bin, so that the
 * per-track range checks are left out (the bound itself is checked per staged segment and
 * template, and a violation raises BSH_STATUS_RANGE); 0 otherwise (-1 for NULL). */
int64_t bsh_plan_units(const bsh_plan* plan);
int32_t bsh_plan_blocks(const bsh_plan* plan);
int32_t bsh_plan_persistent(const bsh_plan* plan);
int32_t bsh_plan_proven(const bsh_plan* plan);
int32_t bsh_plan_passes(const bsh_plan* plan);

int bsh_plan_destroy(bsh_plan* plan);

/* ------------------------------------------------------------------ post-processing
 *
 * The steps after the search (Sec. V.E) on the top-lists: coincidences between two lists,
 * clustering of one list, and significance-weighted centroids with the most significant
 * cluster of the list (one per 0.1 Hz band).  Templates are rows [n][6] FP64 of
 * (f in Hz, x, y, a_p in lt-s, Omega = 2 pi / P in rad/s, t_asc in s); x and y project the
 * sky direction on the plane of the detector's orbital velocity (the ecliptic).
 *
 * Distance (eq:postdist): d^2 = sum over the six parameters of (difference / resolution)^2 with
 * delta f = 1/Tc and delta Theta = c/(v Tc f P_F) (Sec. IV.C) and the binary resolutions of
 * eq:binaryres, each point-dependent resolution taken as the mean of its values at the two
 * templates.  "Closer than w" means d^2 < w^2 evaluated in FP64 in the fixed operation order
 * written in bsh_post.hip, so that the decisions are reproducible.
 */
typedef struct bsh_post_params {
    double t_coh;         /* Tc in s */
    double t_obs;         /* observation time in s (delta Omega) */
    double m_a;           /* mismatch parameters of eq:binaryres */
    double m_omega;
    double m_t;
    double pixel_factor;  /* P_F of the sky resolution */
    double v_over_c;      /* |v|/c of the sky resolution (the orbital speed, about 1e-4) */
} bsh_post_params;

/*
 * Post-processing rows of stage-2 candidates: rows_out[i] = (F/Tc, sky[s][0], sky[s][1], a_p,
 * 2 pi / P, t_asc) for s = cand_sky[i] (cand_params as bsh_power_stat; sky indices are not
 * range-checked here: they must come from the search).
 */
int bsh_post_rows(const double* sky, const int32_t* cand_sky, const double* cand_params, int64_t n,
                  double t_coh, double* rows_out, bsh_stream stream);

/*
 * Significance of stage-1 or stage-2 scores (eq:hough2, eq:hough3) for noise with normalized
 * power p(rho) = exp(-rho): with W1 = sum_J w_J and W2 = sum_J w_J^2 over weight[n_seg],
 *   kind 0 (s_H): (n_w - p0 W1) / sqrt(p0 (1 - p0) W2),  p0 = exp(-rho_th)
 *   kind 1 (s_P): (P - W1) / sqrt(W2)
 * sig_out [n] FP64.
 */
int bsh_significance(const float* score, int64_t n, const float* weight, int64_t n_seg, int32_t kind,
                     double rho_th, double* sig_out, bsh_stream stream);

/* Device workspace bytes of bsh_coincidences for a first list of na rows. */
size_t bsh_coincidences_workspace(int64_t na);

/*
 * Coincidences between two top-lists (Sec. V.E, step 1): every pair (i of a, j of b) with
 * d < window, in (i, j) order.  Pair q gets pairs_out[q] = (i, j), the significance-weighted
 * centroid rows_out[q] = (s_a[i] row_a[i] + s_b[j] row_b[j]) / (s_a[i] + s_b[j]) and the
 * significance sig_out[q] = s_a[i] + s_b[j].  Only the first `cap` pairs are written;
 * *n_pairs_out (device int64) receives the full count.
 */
int bsh_coincidences(const bsh_post_params* pp, const double* rows_a, const double* sig_a, int64_t na,
                     const double* rows_b, const double* sig_b, int64_t nb, double window, int64_t cap,
                     int64_t* pairs_out, double* rows_out, double* sig_out, int64_t* n_pairs_out,
                     void* ws, size_t ws_bytes, bsh_stream stream);

/*
 * Clusters of one list (Sec. V.E, step 2): templates closer than `window` share a cluster and
 * clusters that share a template merge, i.e. the connected components of the "d < window"
 * graph.  label_out[i] = smallest index of i's cluster (int32; n < 2^31).
 */
int bsh_cluster(const bsh_post_params* pp, const double* rows, int64_t n, double window,
                int32_t* label_out, bsh_stream stream);

/* Device workspace bytes of bsh_cluster_centroids for n rows. */
size_t bsh_cluster_centroids_workspace(int64_t n);

/*
 * Per cluster of `label` (as bsh_cluster writes it: every label is the index of a member
 * labelled by itself): the most significant member top_out[r] (lowest index on ties); if
 * cut > 0, the members closer than `cut` to it (the option-B cut of step 2; the top member is
 * always kept); and over the kept members the summed significance weight_out[r] and the
 * significance-weighted centroid centroid_out[r][6] (step 3).  Row r of each output is set for
 * cluster roots r; other rows get weight 0, centroid 0 and top -1.  best_out[0] = root of the
 * cluster with the largest summed significance (lowest root on ties).  Significances must be
 * finite and positive, and labels valid, else BSH_STATUS_INPUT is raised.  The sums use
 * device atomics, so their rounding may differ between runs in the last bits.
 */
int bsh_cluster_centroids(const bsh_post_params* pp, const double* rows, const double* sig,
                          const int32_t* label, int64_t n, double cut, double* centroid_out,
                          double* weight_out, int32_t* top_out, int32_t* best_out, int32_t* status,
                          void* ws, size_t ws_bytes, bsh_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* BSH_H_ */
