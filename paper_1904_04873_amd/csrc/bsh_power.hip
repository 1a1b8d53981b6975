// Stage-2 statistics on the exact track (Sec. IV.C eq:hough3; the GPU loop K2 of Sec. IV.B)
// and the vector-Jacobian product of the bin-interpolated extension.
//
// One wave64 per candidate; lanes stride over segments so the per-segment tables are read
// with coalesced loads, each lane keeps its own partial sum (at most n_seg/64 terms) and a
// wave reduction adds the 64 partials.  The orbit factor is evaluated exactly as in the
// stage-1 kernel (cos(W (t - t_asc)) through the sum formula from cos/sin of W t and
// W t_asc), so a grid template selects the same bins in both stages.
#include "bsh_internal.h"

namespace {

using namespace bsh;

constexpr int kWaves = 4;            // candidates per block
constexpr int kThreads = 64 * kWaves;

__global__ __launch_bounds__(kThreads) void power_stat_kernel(
    const double* __restrict__ t_mid, const double* __restrict__ v, const float* __restrict__ w,
    int32_t w_per_sky, const float* __restrict__ power, const uint32_t* __restrict__ bits,
    int32_t n_words, int32_t n_bins, int64_t k_lo, int64_t n_seg, const double* __restrict__ sky,
    int32_t n_sky, const int32_t* __restrict__ cand_sky, const double* __restrict__ cand, int64_t n,
    int32_t mode, float* __restrict__ P_out, uint32_t* __restrict__ count_out,
    float* __restrict__ wsum_out, int32_t* status)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (c >= n) return;
    const int32_t s = cand_sky[c];
    if (s < 0 || s >= n_sky) {
        if (lane == 0) {
            if (P_out) P_out[c] = 0.f;
            if (count_out) count_out[c] = 0u;
            if (wsum_out) wsum_out[c] = 0.f;
            raise_status(status, BSH_STATUS_INPUT);
        }
        return;
    }
    const Cand cd = load_cand(cand + 4 * c);
    const double nx = sky[3 * s], ny = sky[3 * s + 1], nz = sky[3 * s + 2];
    const float* wr = w + (w_per_sky ? (int64_t)s * n_seg : 0);
    const double klo = (double)k_lo;
    float P = 0.f, ws = 0.f;
    uint32_t cnt = 0u;
    bool bad = false;
    for (int64_t J = lane; J < n_seg; J += 64) {
        double st, ct;
        sincos(cd.W * t_mid[J], &st, &ct);
        const double D = doppler_factor(v + 3 * J, nx, ny, nz);
        const double G = track_G(D, D * ct, D * st, cd.Ac, cd.As);
        const float wj = wr[J];
        if (mode == 0) {
            const int col = (int)(track_bin(cd.F, G) - klo);
            if (col < 0 || col >= n_bins) { bad = true; continue; }
            if (power) P += wj * power[J * n_bins + col];
            if (bits) {
                const uint32_t bit = (bits[J * n_words + (col >> 5)] >> (col & 31)) & 1u;
                cnt += bit;
                ws += bit ? wj : 0.f;
            }
        } else {
            const double x = cd.F * G;
            const double kf = floor(x);
            const int col = (int)(kf - klo);
            if (col < 0 || col + 1 >= n_bins) { bad = true; continue; }
            const float a = (float)(x - kf);
            const float* row = power + J * n_bins + col;
            P += wj * ((1.f - a) * row[0] + a * row[1]);
        }
    }
    if (bad) raise_status(status, BSH_STATUS_RANGE);
    P = wave_sum(P);
    ws = wave_sum(ws);
    cnt = wave_sum(cnt);
    if (lane == 0) {
        if (P_out) P_out[c] = P;
        if (count_out) count_out[c] = cnt;
        if (wsum_out) wsum_out[c] = ws;
    }
}

__global__ __launch_bounds__(kThreads) void power_grad_kernel(
    const double* __restrict__ t_mid, const double* __restrict__ v, const float* __restrict__ w,
    int32_t w_per_sky, const float* __restrict__ power, int32_t n_bins, int64_t k_lo, int64_t n_seg,
    const double* __restrict__ sky, int32_t n_sky, const int32_t* __restrict__ cand_sky,
    const double* __restrict__ cand, int64_t n, const double* __restrict__ grad_P,
    double* __restrict__ grad, int32_t* status)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (c >= n) return;
    const int32_t s = cand_sky[c];
    if (s < 0 || s >= n_sky) {
        if (lane < 4) grad[4 * c + lane] = 0.0;
        if (lane == 0) raise_status(status, BSH_STATUS_INPUT);
        return;
    }
    const Cand cd = load_cand(cand + 4 * c);
    const double nx = sky[3 * s], ny = sky[3 * s + 1], nz = sky[3 * s + 2];
    const float* wr = w + (w_per_sky ? (int64_t)s * n_seg : 0);
    const double klo = (double)k_lo;
    const double WoP = cd.W / cd.P;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
    bool bad = false;
    for (int64_t J = lane; J < n_seg; J += 64) {
        const double t = t_mid[J];
        double st, ct, cphi, sphi;
        sincos(cd.W * t, &st, &ct);
        orbit_phase(ct, st, cd, cphi, sphi);
        const double D = doppler_factor(v + 3 * J, nx, ny, nz);
        const double B = 1.0 - cd.apW * cphi;
        const double x = cd.F * track_G(D, D * ct, D * st, cd.Ac, cd.As);
        const double kf = floor(x);
        const int col = (int)(kf - klo);
        if (col < 0 || col + 1 >= n_bins) { bad = true; continue; }
        const float* row = power + J * n_bins + col;
        const double S = (double)wr[J] * ((double)row[1] - (double)row[0]);
        const double FD = cd.F * D;
        g0 += S * (D * B);
        g1 += S * (-FD * cd.W * cphi);
        g2 += S * (FD * cd.ap * WoP * (cphi - cd.W * (t - cd.ta) * sphi));
        g3 += S * (-FD * cd.apW * cd.W * sphi);
    }
    if (bad) raise_status(status, BSH_STATUS_RANGE);
    g0 = wave_sum(g0);
    g1 = wave_sum(g1);
    g2 = wave_sum(g2);
    g3 = wave_sum(g3);
    if (lane == 0) {
        const double sc = grad_P ? grad_P[c] : 1.0;
        grad[4 * c + 0] = sc * g0;
        grad[4 * c + 1] = sc * g1;
        grad[4 * c + 2] = sc * g2;
        grad[4 * c + 3] = sc * g3;
    }
}


// Low-eccentricity (ELL1) track of eq:frequencyevo in the product form: the orbit factor gains
// (e cos w) cos 2psi - (e sin w) sin 2psi inside the a_p W bracket; cos 2psi and sin 2psi come
// from cos psi and sin psi.  At e = 0 it is bit-identical to the circular track.
__global__ __launch_bounds__(kThreads) void power_stat_ecc_kernel(
    const double* __restrict__ t_mid, const double* __restrict__ v, const float* __restrict__ w,
    int32_t w_per_sky, const float* __restrict__ power, int32_t n_bins, int64_t k_lo, int64_t n_seg,
    const double* __restrict__ sky, int32_t n_sky, const int32_t* __restrict__ cand_sky,
    const double* __restrict__ cand, int64_t n, int32_t mode, float* __restrict__ P_out, int32_t* status)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (c >= n) return;
    const int32_t s = cand_sky[c];
    if (s < 0 || s >= n_sky) {
        if (lane == 0) {
            P_out[c] = 0.f;
            raise_status(status, BSH_STATUS_INPUT);
        }
        return;
    }
    const double* th = cand + 6 * c;
    const Cand cd = load_cand(th);
    const double ec = th[4], es = th[5];
    const double nx = sky[3 * s], ny = sky[3 * s + 1], nz = sky[3 * s + 2];
    const float* wr = w + (w_per_sky ? (int64_t)s * n_seg : 0);
    const double klo = (double)k_lo;
    float P = 0.f;
    bool bad = false;
    for (int64_t J = lane; J < n_seg; J += 64) {
        double st, ct, cphi, sphi;
        sincos(cd.W * t_mid[J], &st, &ct);
        orbit_phase(ct, st, cd, cphi, sphi);
        const double c2 = (cphi - sphi) * (cphi + sphi);
        const double s2 = 2.0 * (sphi * cphi);
        const double D = doppler_factor(v + 3 * J, nx, ny, nz);
        // the circular G minus D a_p W (e cos w cos 2psi - e sin w sin 2psi); for e = 0 the
        // subtracted term is zero and G is the circular track's bit for bit
        const double G = track_G(D, D * ct, D * st, cd.Ac, cd.As) - (D * cd.apW) * (ec * c2 - es * s2);
        const float wj = wr[J];
        if (mode == 0) {
            const int col = (int)(track_bin(cd.F, G) - klo);
            if (col < 0 || col >= n_bins) { bad = true; continue; }
            P += wj * power[J * n_bins + col];
        } else {
            const double x = cd.F * G;
            const double kf = floor(x);
            const int col = (int)(kf - klo);
            if (col < 0 || col + 1 >= n_bins) { bad = true; continue; }
            const float a = (float)(x - kf);
            const float* row = power + J * n_bins + col;
            P += wj * ((1.f - a) * row[0] + a * row[1]);
        }
    }
    if (bad) raise_status(status, BSH_STATUS_RANGE);
    P = wave_sum(P);
    if (lane == 0) P_out[c] = P;
}

}  // namespace

extern "C" int bsh_power_stat(const bsh_segments* seg, const double* sky, int32_t n_sky,
                              const int32_t* cand_sky, const double* cand_params, int64_t n,
                              int32_t mode, float* P_out, uint32_t* count_out, float* wsum_out,
                              int32_t* status, bsh_stream stream)
{
    clear_error();
    if (mode != 0 && mode != 1) return fail_inval("mode must be 0 or 1");
    const bool want_counts = count_out || wsum_out;
    if (mode == 1 && want_counts) return fail_inval("counts are a mode-0 output");
    if (!P_out && !want_counts) return fail_inval("no output");
    int rc = check_segments(seg, want_counts, P_out != nullptr);
    if (rc) return rc;
    if (n < 0) return fail_inval("n < 0");
    if (n_sky < 1) return fail_inval("n_sky < 1");
    if (n == 0) return BSH_OK;
    if (!sky || !cand_sky || !cand_params) return fail_inval("NULL pointer");
    const int64_t blocks = (n + kWaves - 1) / kWaves;
    if (blocks > 0x7fffffff) return fail_inval("too many candidates");
    hipLaunchKernelGGL(power_stat_kernel, dim3((unsigned)blocks), dim3(kThreads), 0,
                       (hipStream_t)stream, seg->t_mid, seg->v_over_c, seg->weight,
                       seg->weight_per_sky, P_out ? seg->power : nullptr,
                       want_counts ? seg->peak_bits : nullptr, words_for(seg->n_bins), seg->n_bins,
                       seg->k_lo, seg->n_seg, sky, n_sky, cand_sky, cand_params, n, mode, P_out,
                       count_out, wsum_out, status);
    return check_launch("bsh_power_stat");
}

extern "C" int bsh_power_stat_grad(const bsh_segments* seg, const double* sky, int32_t n_sky,
                                   const int32_t* cand_sky, const double* cand_params, int64_t n,
                                   const double* grad_P, double* grad_params, int32_t* status,
                                   bsh_stream stream)
{
    clear_error();
    int rc = check_segments(seg, false, true);
    if (rc) return rc;
    if (n < 0) return fail_inval("n < 0");
    if (n_sky < 1) return fail_inval("n_sky < 1");
    if (n == 0) return BSH_OK;
    if (!sky || !cand_sky || !cand_params || !grad_params) return fail_inval("NULL pointer");
    const int64_t blocks = (n + kWaves - 1) / kWaves;
    if (blocks > 0x7fffffff) return fail_inval("too many candidates");
    hipLaunchKernelGGL(power_grad_kernel, dim3((unsigned)blocks), dim3(kThreads), 0,
                       (hipStream_t)stream, seg->t_mid, seg->v_over_c, seg->weight,
                       seg->weight_per_sky, seg->power, seg->n_bins, seg->k_lo, seg->n_seg, sky,
                       n_sky, cand_sky, cand_params, n, grad_P, grad_params, status);
    return check_launch("bsh_power_stat_grad");
}

extern "C" int bsh_power_stat_ecc(const bsh_segments* seg, const double* sky, int32_t n_sky,
                                  const int32_t* cand_sky, const double* cand_params, int64_t n,
                                  int32_t mode, float* P_out, int32_t* status, bsh_stream stream)
{
    clear_error();
    if (mode != 0 && mode != 1) return fail_inval("mode must be 0 or 1");
    if (!P_out) return fail_inval("P_out is NULL");
    int rc = check_segments(seg, false, true);
    if (rc) return rc;
    if (n < 0) return fail_inval("n < 0");
    if (n_sky < 1) return fail_inval("n_sky < 1");
    if (n == 0) return BSH_OK;
    if (!sky || !cand_sky || !cand_params) return fail_inval("NULL pointer");
    const int64_t blocks = (n + kWaves - 1) / kWaves;
    if (blocks > 0x7fffffff) return fail_inval("too many candidates");
    hipLaunchKernelGGL(power_stat_ecc_kernel, dim3((unsigned)blocks), dim3(kThreads), 0,
                       (hipStream_t)stream, seg->t_mid, seg->v_over_c, seg->weight, seg->weight_per_sky,
                       seg->power, seg->n_bins, seg->k_lo, seg->n_seg, sky, n_sky, cand_sky, cand_params,
                       n, mode, P_out, status);
    return check_launch("bsh_power_stat_ecc");
}
