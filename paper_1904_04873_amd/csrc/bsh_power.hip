// Stage-2 statistics on the exact track (Sec. IV.C eq:hough3; the GPU loop K2 of Sec. IV.B)
// and the vector-Jacobian product of the bin-interpolated extension.
//
// A block serves kC candidates; its kC x kP threads split each candidate's segments by phase
// (thread (c, p) takes J = p, p + kP, ...), so the kC lanes of one phase read one power row
// and one set of segment tables per step and a wave touches 64 / kC rows at once.  Each
// thread sums its terms in runs of at most kRun (the run totals added in order), and the kP
// partial sums of a candidate are added by a pairwise tree in LDS: a fixed order, and an FP32
// error below (kRun + n_seg / (kP kRun) + log2 kP) ulps of the total.  Shapes (measured on the
// 4000-segment workload): 8 x 64 for the statistics, whose 10^4-candidate calls need many
// waves, 8 x 32 for the adjoint.  The orbit factor is evaluated exactly as in the stage-1
// kernel (cos(W (t - t_asc)) through the sum formula from cos/sin of W t and W t_asc), so a
// grid template selects the same bins in both stages.
#include "bsh_internal.h"

namespace {

using namespace bsh;

constexpr int kRun = 64;             // terms per run of a thread's FP32 sum
constexpr int kStatC = 8, kStatP = 64;
constexpr int kGradC = 8, kGradP = 32;

// FP32 sum of a thread's terms in runs of kRun.
struct RunSum {
    float total = 0.f, run = 0.f;
    int n = 0;
    __device__ __forceinline__ void add(float x)
    {
        run += x;
        if (++n == kRun) {
            total += run;
            run = 0.f;
            n = 0;
        }
    }
    __device__ __forceinline__ float value() const { return total + run; }
};

// The candidate's total over the kP threads serving it, by a pairwise tree over the phases
// in LDS; valid in the phase-0 thread.  Every thread of the block calls this.
template <int kC, int kP, typename T>
__device__ __forceinline__ T phase_sum(T v, T* red)
{
    const int cl = threadIdx.x % kC, p = threadIdx.x / kC;
    __syncthreads();
    red[p * kC + cl] = v;
    __syncthreads();
#pragma unroll
    for (int half = kP / 2; half > 0; half /= 2) {
        if (p < half) red[p * kC + cl] += red[(p + half) * kC + cl];
        __syncthreads();
    }
    return red[cl];
}

__device__ __forceinline__ bool cand_sky_ok(const int32_t* cand_sky, int64_t c, int64_t n, int32_t n_sky,
                                            int32_t& s)
{
    s = c < n ? cand_sky[c] : 0;
    return c < n && s >= 0 && s < n_sky;
}

// kEcc: candidates are (F, a_p, P, t_asc, e cos w, e sin w) rows on the ELL1 track (track_G_ecc);
// with zero eccentricity every result is the circular kernel's bit for bit.
template <bool kEcc>
__global__ __launch_bounds__(kStatC * kStatP) void power_stat_kernel(
    const double* __restrict__ t_mid, const double* __restrict__ v, const float* __restrict__ w,
    int32_t w_per_sky, const float* __restrict__ power, const uint32_t* __restrict__ bits,
    int32_t n_words, int32_t n_bins, int64_t k_lo, int64_t n_seg, const double* __restrict__ sky,
    int32_t n_sky, const int32_t* __restrict__ cand_sky, const double* __restrict__ cand, int64_t n,
    int32_t mode, float* __restrict__ P_out, uint32_t* __restrict__ count_out,
    float* __restrict__ wsum_out, int32_t* status)
{
    __shared__ float redf[kStatC * kStatP];
    __shared__ uint32_t redu[kStatC * kStatP];
    const int cl = threadIdx.x % kStatC, p = threadIdx.x / kStatC;
    const int64_t c = (int64_t)blockIdx.x * kStatC + cl;
    int32_t s;
    const bool ok = cand_sky_ok(cand_sky, c, n, n_sky, s);
    RunSum P, ws;
    uint32_t cnt = 0u;
    bool bad = false;
    if (ok) {
        const double* th = cand + (kEcc ? 6 : 4) * c;
        const Cand cd = load_cand(th);
        double Ac2 = 0.0, As2 = 0.0;
        if constexpr (kEcc) ecc_coeffs(cd.apW, cd.cb, cd.sb, th[4], th[5], Ac2, As2);
        const double nx = sky[3 * s], ny = sky[3 * s + 1], nz = sky[3 * s + 2];
        const float* wr = w + (w_per_sky ? (int64_t)s * n_seg : 0);
        const double klo = (double)k_lo;
        for (int64_t J = p; J < n_seg; J += kStatP) {
            double st, ct;
            track_sincos(cd.W * t_mid[J], st, ct);
            const double D = doppler_factor(v + 3 * J, nx, ny, nz);
            double G;
            if constexpr (kEcc) {
                double c2, s2;
                double_angle(ct, st, c2, s2);
                G = track_G_ecc(D, D * ct, D * st, cd.Ac, cd.As, D * c2, D * s2, Ac2, As2);
            } else {
                G = track_G(D, D * ct, D * st, cd.Ac, cd.As);
            }
            const float wj = wr[J];
            if (mode == 0) {
                const int col = (int)(track_bin(cd.F, G) - klo);
                if (col < 0 || col >= n_bins) { bad = true; continue; }
                if (power) P.add(wj * power[J * n_bins + col]);
                if (bits) {
                    const uint32_t bit = (bits[J * n_words + (col >> 5)] >> (col & 31)) & 1u;
                    cnt += bit;
                    ws.add(bit ? wj : 0.f);
                }
            } else {
                const double x = cd.F * G;
                const double kf = floor(x);
                const int col = (int)(kf - klo);
                if (col < 0 || col + 1 >= n_bins) { bad = true; continue; }
                const float a = (float)(x - kf);
                const float* row = power + J * n_bins + col;
                P.add(wj * ((1.f - a) * row[0] + a * row[1]));
            }
        }
    }
    if (bad) raise_status(status, BSH_STATUS_RANGE);
    if (c < n && !ok && p == 0) raise_status(status, BSH_STATUS_INPUT);
    const float Pt = phase_sum<kStatC, kStatP>(P.value(), redf);
    const float wt = phase_sum<kStatC, kStatP>(ws.value(), redf);
    const uint32_t ct = phase_sum<kStatC, kStatP>(cnt, redu);
    if (p == 0 && c < n) {
        if (P_out) P_out[c] = Pt;
        if (count_out) count_out[c] = ct;
        if (wsum_out) wsum_out[c] = wt;
    }
}

// kValue: also P_lin itself (the mode-1 statistic) from the same gathers, so that a gradient
// step needs one pass over the segments instead of a forward and a backward pass.  The gradient
// is the same computation, in the same order, with or without it.
// kEcc: (F, a_p, P, t_asc, e cos w, e sin w) rows on the ELL1 track and six gradient columns,
// with E = cos psi + ec cos 2psi - es sin 2psi, E' = -sin psi - 2 ec sin 2psi - 2 es cos 2psi
// in place of cos psi and -sin psi (at zero eccentricity the same numbers, bit for bit).
template <bool kValue, bool kEcc>
__global__ __launch_bounds__(kGradC * kGradP) void power_grad_kernel(
    const double* __restrict__ t_mid, const double* __restrict__ v, const float* __restrict__ w,
    int32_t w_per_sky, const float* __restrict__ power, int32_t n_bins, int64_t k_lo, int64_t n_seg,
    const double* __restrict__ sky, int32_t n_sky, const int32_t* __restrict__ cand_sky,
    const double* __restrict__ cand, int64_t n, const double* __restrict__ grad_P,
    double* __restrict__ grad, float* __restrict__ P_out, int32_t* status)
{
    __shared__ double red[kGradC * kGradP];
    const int cl = threadIdx.x % kGradC, p = threadIdx.x / kGradC;
    const int64_t c = (int64_t)blockIdx.x * kGradC + cl;
    int32_t s;
    const bool ok = cand_sky_ok(cand_sky, c, n, n_sky, s);
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0, g4 = 0.0, g5 = 0.0;
    RunSum P;
    bool bad = false;
    if (ok) {
        const double* th = cand + (kEcc ? 6 : 4) * c;
        const Cand cd = load_cand(th);
        const double ec = kEcc ? th[4] : 0.0, es = kEcc ? th[5] : 0.0;
        double Ac2 = 0.0, As2 = 0.0;
        if constexpr (kEcc) ecc_coeffs(cd.apW, cd.cb, cd.sb, ec, es, Ac2, As2);
        const double nx = sky[3 * s], ny = sky[3 * s + 1], nz = sky[3 * s + 2];
        const float* wr = w + (w_per_sky ? (int64_t)s * n_seg : 0);
        const double klo = (double)k_lo;
        const double WoP = cd.W / cd.P;
        for (int64_t J = p; J < n_seg; J += kGradP) {
            const double t = t_mid[J];
            double st, ct, cphi, sphi;
            track_sincos(cd.W * t, st, ct);
            orbit_phase(ct, st, cd, cphi, sphi);
            const double D = doppler_factor(v + 3 * J, nx, ny, nz);
            // E and E' (cos psi and -sin psi on the circular track)
            double E = cphi, Ep = -sphi, c2p = 0.0, s2p = 0.0, x;
            if constexpr (kEcc) {
                double c2, s2;
                double_angle(ct, st, c2, s2);
                x = cd.F * track_G_ecc(D, D * ct, D * st, cd.Ac, cd.As, D * c2, D * s2, Ac2, As2);
                double_angle(cphi, sphi, c2p, s2p);
                E = cphi + (ec * c2p - es * s2p);
                Ep = -sphi - 2.0 * (ec * s2p) - 2.0 * (es * c2p);
            } else {
                x = cd.F * track_G(D, D * ct, D * st, cd.Ac, cd.As);
            }
            const double B = 1.0 - cd.apW * E;
            const double kf = floor(x);
            const int col = (int)(kf - klo);
            if (col < 0 || col + 1 >= n_bins) { bad = true; continue; }
            const float* row = power + J * n_bins + col;
            if (kValue) {
                const float a = (float)(x - kf);
                P.add(wr[J] * ((1.f - a) * row[0] + a * row[1]));
            }
            const double S = (double)wr[J] * ((double)row[1] - (double)row[0]);
            const double FD = cd.F * D;
            g0 += S * (D * B);
            if constexpr (kEcc) {
                const double psi = cd.W * (t - cd.ta);
                g1 += S * (-FD * cd.W * E);
                g2 += S * (FD * cd.ap * WoP * (E + psi * Ep));
                g3 += S * (FD * cd.apW * cd.W * Ep);
                g4 += S * (-FD * cd.apW * c2p);
                g5 += S * (FD * cd.apW * s2p);
            } else {
                g1 += S * (-FD * cd.W * cphi);
                g2 += S * (FD * cd.ap * WoP * (cphi - cd.W * (t - cd.ta) * sphi));
                g3 += S * (-FD * cd.apW * cd.W * sphi);
            }
        }
    }
    if (bad) raise_status(status, BSH_STATUS_RANGE);
    if (c < n && !ok && p == 0) raise_status(status, BSH_STATUS_INPUT);
    g0 = phase_sum<kGradC, kGradP>(g0, red);
    g1 = phase_sum<kGradC, kGradP>(g1, red);
    g2 = phase_sum<kGradC, kGradP>(g2, red);
    g3 = phase_sum<kGradC, kGradP>(g3, red);
    if constexpr (kEcc) {
        g4 = phase_sum<kGradC, kGradP>(g4, red);
        g5 = phase_sum<kGradC, kGradP>(g5, red);
    }
    float Pt = 0.f;
    if (kValue) {
        // the doubles' LDS tree holds the float partial sums too (converted exactly)
        Pt = (float)phase_sum<kGradC, kGradP>((double)P.value(), red);
    }
    if (p == 0 && c < n) {
        const double sc = ok ? (grad_P ? grad_P[c] : 1.0) : 0.0;
        constexpr int kCols = kEcc ? 6 : 4;
        grad[kCols * c + 0] = sc * g0;
        grad[kCols * c + 1] = sc * g1;
        grad[kCols * c + 2] = sc * g2;
        grad[kCols * c + 3] = sc * g3;
        if constexpr (kEcc) {
            grad[kCols * c + 4] = sc * g4;
            grad[kCols * c + 5] = sc * g5;
        }
        if (kValue) P_out[c] = Pt;
    }
}


}  // namespace

namespace {

template <bool kEcc>
int launch_stat(const bsh_segments* seg, const double* sky, int32_t n_sky, const int32_t* cand_sky,
                const double* cand_params, int64_t n, int32_t mode, float* P_out, uint32_t* count_out,
                float* wsum_out, int32_t* status, bsh_stream stream, const char* what)
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
    const int64_t blocks = (n + kStatC - 1) / kStatC;
    if (blocks > 0x7fffffff) return fail_inval("too many candidates");
    hipLaunchKernelGGL(power_stat_kernel<kEcc>, dim3((unsigned)blocks), dim3(kStatC * kStatP), 0,
                       (hipStream_t)stream, seg->t_mid, seg->v_over_c, seg->weight,
                       seg->weight_per_sky, P_out ? seg->power : nullptr,
                       want_counts ? seg->peak_bits : nullptr, words_for(seg->n_bins), seg->n_bins,
                       seg->k_lo, seg->n_seg, sky, n_sky, cand_sky, cand_params, n, mode, P_out,
                       count_out, wsum_out, status);
    return check_launch(what);
}

}  // namespace

extern "C" int bsh_power_stat(const bsh_segments* seg, const double* sky, int32_t n_sky,
                              const int32_t* cand_sky, const double* cand_params, int64_t n,
                              int32_t mode, float* P_out, uint32_t* count_out, float* wsum_out,
                              int32_t* status, bsh_stream stream)
{
    return launch_stat<false>(seg, sky, n_sky, cand_sky, cand_params, n, mode, P_out, count_out, wsum_out,
                              status, stream, "bsh_power_stat");
}

extern "C" int bsh_power_stat_ecc(const bsh_segments* seg, const double* sky, int32_t n_sky,
                                  const int32_t* cand_sky, const double* cand_params, int64_t n,
                                  int32_t mode, float* P_out, uint32_t* count_out, float* wsum_out,
                                  int32_t* status, bsh_stream stream)
{
    return launch_stat<true>(seg, sky, n_sky, cand_sky, cand_params, n, mode, P_out, count_out, wsum_out,
                             status, stream, "bsh_power_stat_ecc");
}

namespace {

template <bool kEcc>
int launch_grad(const bsh_segments* seg, const double* sky, int32_t n_sky, const int32_t* cand_sky,
                const double* cand_params, int64_t n, const double* grad_P, double* grad_params,
                float* P_out, int32_t* status, bsh_stream stream, const char* what)
{
    clear_error();
    int rc = check_segments(seg, false, true);
    if (rc) return rc;
    if (n < 0) return fail_inval("n < 0");
    if (n_sky < 1) return fail_inval("n_sky < 1");
    if (n == 0) return BSH_OK;
    if (!sky || !cand_sky || !cand_params || !grad_params) return fail_inval("NULL pointer");
    const int64_t blocks = (n + kGradC - 1) / kGradC;
    if (blocks > 0x7fffffff) return fail_inval("too many candidates");
    auto kernel = P_out ? power_grad_kernel<true, kEcc> : power_grad_kernel<false, kEcc>;
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kGradC * kGradP), 0, (hipStream_t)stream,
                       seg->t_mid, seg->v_over_c, seg->weight, seg->weight_per_sky, seg->power,
                       seg->n_bins, seg->k_lo, seg->n_seg, sky, n_sky, cand_sky, cand_params, n, grad_P,
                       grad_params, P_out, status);
    return check_launch(what);
}

}  // namespace

extern "C" int bsh_power_stat_grad(const bsh_segments* seg, const double* sky, int32_t n_sky,
                                   const int32_t* cand_sky, const double* cand_params, int64_t n,
                                   const double* grad_P, double* grad_params, int32_t* status,
                                   bsh_stream stream)
{
    return launch_grad<false>(seg, sky, n_sky, cand_sky, cand_params, n, grad_P, grad_params, nullptr, status,
                              stream, "bsh_power_stat_grad");
}

extern "C" int bsh_power_stat_value_and_grad(const bsh_segments* seg, const double* sky, int32_t n_sky,
                                             const int32_t* cand_sky, const double* cand_params, int64_t n,
                                             const double* grad_P, float* P_out, double* grad_params,
                                             int32_t* status, bsh_stream stream)
{
    if (!P_out && n > 0) {
        clear_error();
        return fail_inval("P_out is NULL");
    }
    return launch_grad<false>(seg, sky, n_sky, cand_sky, cand_params, n, grad_P, grad_params, P_out, status,
                              stream, "bsh_power_stat_value_and_grad");
}

extern "C" int bsh_power_stat_grad_ecc(const bsh_segments* seg, const double* sky, int32_t n_sky,
                                       const int32_t* cand_sky, const double* cand_params, int64_t n,
                                       const double* grad_P, float* P_out, double* grad_params,
                                       int32_t* status, bsh_stream stream)
{
    return launch_grad<true>(seg, sky, n_sky, cand_sky, cand_params, n, grad_P, grad_params, P_out, status,
                             stream, "bsh_power_stat_grad_ecc");
}
