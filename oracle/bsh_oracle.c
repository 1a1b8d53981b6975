/*
 * TEST INFRASTRUCTURE ONLY -- the CPU oracle of the binary Hough search.
 *
 * Plain, slow, FP64 definitions of what the search computes, written from
 * Covas & Sintes, "BinarySkyHough" (arXiv:1904.04873).  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load this file's
 * library; the GPU library shares no code with it.
 *
 * Definitions (product form of the zero-eccentricity frequency track):
 *   x_J(theta) = f(t_J) * Tc = F * (1 + v_J.n) * (1 - a_p * Omega * cos(Omega (t_J - t_asc)))
 *     with F = f0 * Tc, Omega = 2 pi / P                [Sec. II, eq:frequencyevoFinal;
 *                                                         product form as in eq:hough1]
 *   k_J = floor(x_J + 1/2)     nearest DFT bin, bin k <-> k / Tc   [Sec. IV.A, DFT]
 *   peak  p_J = [rho_{J,k_J} > rho_th]                              [Sec. IV.A]
 *   number count n = sum_J w_J p_J (weighted), count = sum_J p_J    [Sec. IV.C, eq:hough2]
 *   power  P = sum_J w_J rho_{J,k_J}                                [Sec. IV.C, eq:hough3]
 *   interpolated power P_lin = sum_J w_J ((1-a) rho_{J,k'} + a rho_{J,k'+1}),
 *     k' = floor(x_J), a = x_J - k'  (an extension of eq:hough3; not in the paper)
 *
 * Every evaluation follows one fixed expression order (d = (vx nx + vy ny) + vz nz,
 * D = 1 + d, W = 2pi/P, phi = W (t - t_asc), B = 1 - (a_p W) cos phi, G = D B,
 * x = F G) and must be compiled without floating-point contraction.
 * Evaluations with x within NEAR_TIE of a half-integer are counted as near-ties:
 * there a differently ordered but equally accurate evaluation may pick the
 * neighbouring bin.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

#define TWO_PI 6.283185307179586
#define NEAR_TIE 1e-9

#define ORC_OK 0
#define ORC_ERANGE (-2)

/* Doppler factor of segment J towards sky direction n (eq:frequencyevoFinal, v.n/c term). */
static double doppler_factor(const double* v, const double* n)
{
    double d = v[0] * n[0] + v[1] * n[1];
    d = d + v[2] * n[2];
    return 1.0 + d;
}

/* Binary-orbit factor at time t (eq:frequencyevoFinal, a_p Omega cos term). */
static double orbit_factor(double t, double a_p, double period, double t_asc)
{
    double w = TWO_PI / period;
    double phi = w * (t - t_asc);
    return 1.0 - (a_p * w) * cos(phi);
}

/* Additive form of the same track: 1 + v.n - a_p Omega cos(...)  (reading c1 alternative). */
static double additive_factor(double d_factor, double b_factor)
{
    return (d_factor - 1.0) + b_factor;
}

static int is_near_tie(double x)
{
    double y = x + 0.5;
    double f = y - floor(y);
    return (f < NEAR_TIE) || (f > 1.0 - NEAR_TIE);
}

/*
 * Stage-1 number count over the full template grid (Sec. IV.C; K1 of Sec. IV.B).
 * Template index: idx = ((s * n_bin) + b) * n_f0 + i with b = tasc_off[ia*n_per+ip] + j.
 * power: [n_seg][n_bins] normalized power; the peak test is applied here.
 * Outputs per template: count, weighted count (FP64), number of near-tie segments
 * and the weight carried by them.  Returns ORC_ERANGE if a bin leaves the row.
 */
int orc_hough_count(int64_t n_seg, const double* t_mid, const double* v_over_c,
                    const float* weight, int32_t weight_per_sky,
                    int64_t k_lo, int32_t n_bins, const float* power, double rho_th,
                    int32_t n_sky, const double* sky, int64_t k0, int32_t n_f0,
                    int32_t n_ap, const double* a_p, int32_t n_per, const double* period,
                    const int64_t* tasc_off, const double* t_asc, int32_t additive,
                    uint32_t* count_out, double* nw_out, uint32_t* ntie_out, double* ntie_w_out)
{
    const int64_t n_bin = tasc_off[(int64_t)n_ap * n_per];
    int err = ORC_OK;
    double* D = (double*)malloc(sizeof(double) * (size_t)(n_seg > 0 ? n_seg : 1));
    if (!D) return -4;
    for (int32_t s = 0; s < n_sky; ++s) {
        const float* w = weight + (weight_per_sky ? (int64_t)s * n_seg : 0);
        /* loop invariant of the sky pixel: D per segment */
        for (int64_t J = 0; J < n_seg; ++J) D[J] = doppler_factor(v_over_c + 3 * J, sky + 3 * s);
        #pragma omp parallel reduction(min:err)
        {
            double* B = (double*)malloc(sizeof(double) * (size_t)(n_seg > 0 ? n_seg : 1));
            #pragma omp for schedule(static)
            for (int64_t b = 0; b < n_bin; ++b) {
                /* locate the (a_p, P) cell of binary template b */
                int64_t cell = 0;
                while (tasc_off[cell + 1] <= b) ++cell;
                const double ap = a_p[cell / n_per];
                const double per = period[cell % n_per];
                const double ta = t_asc[b];
                /* loop invariant of the binary template: B per segment */
                for (int64_t J = 0; J < n_seg; ++J) B[J] = orbit_factor(t_mid[J], ap, per, ta);
                for (int32_t i = 0; i < n_f0; ++i) {
                    const double F = (double)(k0 + i);
                    uint32_t cnt = 0, nt = 0;
                    double nw = 0.0, ntw = 0.0;
                    for (int64_t J = 0; J < n_seg; ++J) {
                        double G = additive ? additive_factor(D[J], B[J]) : D[J] * B[J];
                        double x = F * G;
                        double kk = floor(x + 0.5);
                        int64_t c = (int64_t)kk - k_lo;
                        if (c < 0 || c >= n_bins) { err = ORC_ERANGE; continue; }
                        int p = power[J * n_bins + c] > rho_th;
                        cnt += (uint32_t)p;
                        nw += p ? (double)w[J] : 0.0;
                        if (is_near_tie(x)) { nt += 1; ntw += (double)w[J]; }
                    }
                    const int64_t idx = (((int64_t)s * n_bin) + b) * n_f0 + i;
                    if (count_out) count_out[idx] = cnt;
                    if (nw_out) nw_out[idx] = nw;
                    if (ntie_out) ntie_out[idx] = nt;
                    if (ntie_w_out) ntie_w_out[idx] = ntw;
                }
            }
            free(B);
        }
    }
    free(D);
    return err;
}

/*
 * Per-candidate frequency track: continuous x_J and bin k_J (absolute) for
 * each candidate (sky index, F = f0 Tc, a_p, P, t_asc).  out_x / out_k are
 * [n_cand][n_seg]; either may be NULL.
 */
void orc_track(int64_t n_seg, const double* t_mid, const double* v_over_c,
               const double* sky, int64_t n_cand, const int32_t* cand_sky,
               const double* cand, int32_t additive, double* out_x, int64_t* out_k)
{
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n_cand; ++c) {
        const double* th = cand + 4 * c;
        for (int64_t J = 0; J < n_seg; ++J) {
            double D = doppler_factor(v_over_c + 3 * J, sky + 3 * cand_sky[c]);
            double B = orbit_factor(t_mid[J], th[1], th[2], th[3]);
            double G = additive ? additive_factor(D, B) : D * B;
            double x = th[0] * G;
            if (out_x) out_x[c * n_seg + J] = x;
            if (out_k) out_k[c * n_seg + J] = (int64_t)floor(x + 0.5);
        }
    }
}

/*
 * Per-candidate statistics on the exact track (Sec. IV.C, eq:hough2 / eq:hough3):
 *   mode 0: P = sum w rho at the nearest bin, plus count and weighted count of peaks;
 *   mode 1: P_lin, the bin-interpolated power.
 * weight is [n_seg] or [n_sky][n_seg].  Any output pointer may be NULL.
 */
int orc_power_stat(int64_t n_seg, const double* t_mid, const double* v_over_c,
                   const float* weight, int32_t weight_per_sky,
                   int64_t k_lo, int32_t n_bins, const float* power, double rho_th,
                   const double* sky, int64_t n_cand, const int32_t* cand_sky,
                   const double* cand, int32_t mode,
                   double* p_out, uint32_t* count_out, double* nw_out, uint32_t* ntie_out)
{
    int err = ORC_OK;
    #pragma omp parallel for schedule(static) reduction(min:err)
    for (int64_t c = 0; c < n_cand; ++c) {
        const double* th = cand + 4 * c;
        const float* w = weight + (weight_per_sky ? (int64_t)cand_sky[c] * n_seg : 0);
        double P = 0.0, nw = 0.0;
        uint32_t cnt = 0, nt = 0;
        for (int64_t J = 0; J < n_seg; ++J) {
            double D = doppler_factor(v_over_c + 3 * J, sky + 3 * cand_sky[c]);
            double B = orbit_factor(t_mid[J], th[1], th[2], th[3]);
            double x = th[0] * (D * B);
            const float* row = power + J * n_bins;
            if (mode == 0) {
                int64_t col = (int64_t)floor(x + 0.5) - k_lo;
                if (col < 0 || col >= n_bins) { err = ORC_ERANGE; continue; }
                double rho = (double)row[col];
                P += (double)w[J] * rho;
                if (rho > rho_th) { cnt += 1; nw += (double)w[J]; }
                if (is_near_tie(x)) nt += 1;
            } else {
                double kf = floor(x);
                int64_t col = (int64_t)kf - k_lo;
                if (col < 0 || col + 1 >= n_bins) { err = ORC_ERANGE; continue; }
                double a = x - kf;
                P += (double)w[J] * ((1.0 - a) * (double)row[col] + a * (double)row[col + 1]);
            }
        }
        if (p_out) p_out[c] = P;
        if (count_out) count_out[c] = cnt;
        if (nw_out) nw_out[c] = nw;
        if (ntie_out) ntie_out[c] = nt;
    }
    return err;
}

/*
 * Gradient of P_lin with respect to (F, a_p, P, t_asc), scaled by grad_p[c].
 * With S_J = w_J (rho_{k'+1} - rho_{k'}) and the track x = F D B,
 *   dx/dF     = D B
 *   dx/da_p   = -F D W cos(phi)
 *   dx/dP     =  F D a_p (W / P) (cos(phi) - W (t - t_asc) sin(phi))
 *   dx/dt_asc = -F D a_p W^2 sin(phi)
 * (differentiating the product-form track; the t_asc term is minus the orbital
 * part of the frequency derivative of eq:derivative, scaled by F D).  At an
 * exact integer x the right-hand interval [k', k'+1] is used.
 */
int orc_power_grad(int64_t n_seg, const double* t_mid, const double* v_over_c,
                   const float* weight, int32_t weight_per_sky,
                   int64_t k_lo, int32_t n_bins, const float* power,
                   const double* sky, int64_t n_cand, const int32_t* cand_sky,
                   const double* cand, const double* grad_p, double* grad_out, double* abs_out)
{
    int err = ORC_OK;
    #pragma omp parallel for schedule(static) reduction(min:err)
    for (int64_t c = 0; c < n_cand; ++c) {
        const double* th = cand + 4 * c;
        const double F = th[0], ap = th[1], per = th[2], ta = th[3];
        const float* w = weight + (weight_per_sky ? (int64_t)cand_sky[c] * n_seg : 0);
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;   /* sums of |term|, for tolerances */
        for (int64_t J = 0; J < n_seg; ++J) {
            double D = doppler_factor(v_over_c + 3 * J, sky + 3 * cand_sky[c]);
            double W = TWO_PI / per;
            double dt = t_mid[J] - ta;
            double phi = W * dt;
            double cp = cos(phi), sp = sin(phi);
            double B = 1.0 - (ap * W) * cp;
            double x = F * (D * B);
            double kf = floor(x);
            int64_t col = (int64_t)kf - k_lo;
            if (col < 0 || col + 1 >= n_bins) { err = ORC_ERANGE; continue; }
            const float* row = power + J * n_bins;
            double S = (double)w[J] * ((double)row[col + 1] - (double)row[col]);
            double t0 = S * (D * B);
            double t1 = S * (-F * D * W * cp);
            double t2 = S * (F * D * ap * (W / per) * (cp - W * dt * sp));
            double t3 = S * (-F * D * ap * W * W * sp);
            g0 += t0; g1 += t1; g2 += t2; g3 += t3;
            a0 += fabs(t0); a1 += fabs(t1); a2 += fabs(t2); a3 += fabs(t3);
        }
        const double s = grad_p ? grad_p[c] : 1.0;
        grad_out[4 * c + 0] = s * g0;
        grad_out[4 * c + 1] = s * g1;
        grad_out[4 * c + 2] = s * g2;
        grad_out[4 * c + 3] = s * g3;
        if (abs_out) {
            abs_out[4 * c + 0] = fabs(s) * a0;
            abs_out[4 * c + 1] = fabs(s) * a1;
            abs_out[4 * c + 2] = fabs(s) * a2;
            abs_out[4 * c + 3] = fabs(s) * a3;
        }
    }
    return err;
}

/*
 * Low-eccentricity (ELL1) track, eq:frequencyevo (Sec. II), in the product form:
 *   x = F (1 + v.n) (1 - a_p W [cos psi + (e cos w) cos 2psi - (e sin w) sin 2psi]),
 *   psi = W (t - t_asc).
 * Candidates are rows (F, a_p, P, t_asc, e cos w, e sin w).  Outputs as orc_track, and the
 * nearest-bin power P = sum w rho (mode 0) or the interpolated power (mode 1) per candidate.
 */
static double orbit_factor_ecc(double t, double a_p, double period, double t_asc, double ec, double es)
{
    double w = TWO_PI / period;
    double psi = w * (t - t_asc);
    double c1 = cos(psi);
    double c2 = cos(2.0 * psi);
    double s2 = sin(2.0 * psi);
    return 1.0 - (a_p * w) * (c1 + (ec * c2 - es * s2));
}

void orc_track_ecc(int64_t n_seg, const double* t_mid, const double* v_over_c, const double* sky,
                   int64_t n_cand, const int32_t* cand_sky, const double* cand, double* out_x,
                   int64_t* out_k)
{
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n_cand; ++c) {
        const double* th = cand + 6 * c;
        for (int64_t J = 0; J < n_seg; ++J) {
            double D = doppler_factor(v_over_c + 3 * J, sky + 3 * cand_sky[c]);
            double B = orbit_factor_ecc(t_mid[J], th[1], th[2], th[3], th[4], th[5]);
            double x = th[0] * (D * B);
            if (out_x) out_x[c * n_seg + J] = x;
            if (out_k) out_k[c * n_seg + J] = (int64_t)floor(x + 0.5);
        }
    }
}

int orc_power_stat_ecc(int64_t n_seg, const double* t_mid, const double* v_over_c,
                       const float* weight, int32_t weight_per_sky, int64_t k_lo, int32_t n_bins,
                       const float* power, const double* sky, int64_t n_cand,
                       const int32_t* cand_sky, const double* cand, int32_t mode, double* p_out,
                       uint32_t* ntie_out)
{
    int err = ORC_OK;
    #pragma omp parallel for schedule(static) reduction(min:err)
    for (int64_t c = 0; c < n_cand; ++c) {
        const double* th = cand + 6 * c;
        const float* w = weight + (weight_per_sky ? (int64_t)cand_sky[c] * n_seg : 0);
        double P = 0.0;
        uint32_t nt = 0;
        for (int64_t J = 0; J < n_seg; ++J) {
            double D = doppler_factor(v_over_c + 3 * J, sky + 3 * cand_sky[c]);
            double B = orbit_factor_ecc(t_mid[J], th[1], th[2], th[3], th[4], th[5]);
            double x = th[0] * (D * B);
            const float* row = power + J * n_bins;
            if (mode == 0) {
                int64_t col = (int64_t)floor(x + 0.5) - k_lo;
                if (col < 0 || col >= n_bins) { err = ORC_ERANGE; continue; }
                P += (double)w[J] * (double)row[col];
                if (is_near_tie(x)) nt += 1;
            } else {
                double kf = floor(x);
                int64_t col = (int64_t)kf - k_lo;
                if (col < 0 || col + 1 >= n_bins) { err = ORC_ERANGE; continue; }
                double a = x - kf;
                P += (double)w[J] * ((1.0 - a) * (double)row[col] + a * (double)row[col + 1]);
            }
        }
        if (p_out) p_out[c] = P;
        if (ntie_out) ntie_out[c] = nt;
    }
    return err;
}

/*
 * Stage-1 number count on the ELL1 track for one eccentricity pair (ec, es) = (e cos w, e sin w)
 * shared by every template of the grid: the same template order, outputs and near-tie
 * bookkeeping as orc_hough_count, with the orbit factor of orbit_factor_ecc (product form).
 */
int orc_hough_count_ecc(int64_t n_seg, const double* t_mid, const double* v_over_c,
                        const float* weight, int32_t weight_per_sky,
                        int64_t k_lo, int32_t n_bins, const float* power, double rho_th,
                        int32_t n_sky, const double* sky, int64_t k0, int32_t n_f0,
                        int32_t n_ap, const double* a_p, int32_t n_per, const double* period,
                        const int64_t* tasc_off, const double* t_asc, double ec, double es,
                        uint32_t* count_out, double* nw_out, uint32_t* ntie_out, double* ntie_w_out)
{
    const int64_t n_bin = tasc_off[(int64_t)n_ap * n_per];
    int err = ORC_OK;
    for (int32_t s = 0; s < n_sky; ++s) {
        const float* w = weight + (weight_per_sky ? (int64_t)s * n_seg : 0);
        #pragma omp parallel for schedule(static) reduction(min:err)
        for (int64_t b = 0; b < n_bin; ++b) {
            int64_t cell = 0;
            while (tasc_off[cell + 1] <= b) ++cell;
            const double ap = a_p[cell / n_per];
            const double per = period[cell % n_per];
            const double ta = t_asc[b];
            for (int32_t i = 0; i < n_f0; ++i) {
                const double F = (double)(k0 + i);
                uint32_t cnt = 0, nt = 0;
                double nw = 0.0, ntw = 0.0;
                for (int64_t J = 0; J < n_seg; ++J) {
                    double D = doppler_factor(v_over_c + 3 * J, sky + 3 * s);
                    double B = orbit_factor_ecc(t_mid[J], ap, per, ta, ec, es);
                    double x = F * (D * B);
                    int64_t c = (int64_t)floor(x + 0.5) - k_lo;
                    if (c < 0 || c >= n_bins) { err = ORC_ERANGE; continue; }
                    int p = power[J * n_bins + c] > rho_th;
                    cnt += (uint32_t)p;
                    nw += p ? (double)w[J] : 0.0;
                    if (is_near_tie(x)) { nt += 1; ntw += (double)w[J]; }
                }
                const int64_t idx = (((int64_t)s * n_bin) + b) * n_f0 + i;
                if (count_out) count_out[idx] = cnt;
                if (nw_out) nw_out[idx] = nw;
                if (ntie_out) ntie_out[idx] = nt;
                if (ntie_w_out) ntie_w_out[idx] = ntw;
            }
        }
    }
    return err;
}

/*
 * Gradient of P_lin on the ELL1 track with respect to (F, a_p, P, t_asc, e cos w, e sin w),
 * scaled by grad_p[c].  With psi = W (t - t_asc), E = cos psi + ec cos 2psi - es sin 2psi
 * (so that B = 1 - a_p W E) and E' = dE/dpsi = -sin psi - 2 ec sin 2psi - 2 es cos 2psi:
 *   dx/dF     = D B
 *   dx/da_p   = -F D W E
 *   dx/dP     =  F D a_p (W / P) (E + psi E')      (dW/dP = -W/P, dpsi/dP = -psi/P)
 *   dx/dt_asc =  F D a_p W^2 E'                    (dpsi/dt_asc = -W)
 *   dx/d(ec)  = -F D a_p W cos 2psi
 *   dx/d(es)  =  F D a_p W sin 2psi
 * derived by hand from the track of orbit_factor_ecc; at e = 0 the first four are the terms of
 * orc_power_grad.  S_J, the right-hand interval at an exact integer x and abs_out as there.
 */
int orc_power_grad_ecc(int64_t n_seg, const double* t_mid, const double* v_over_c,
                       const float* weight, int32_t weight_per_sky,
                       int64_t k_lo, int32_t n_bins, const float* power,
                       const double* sky, int64_t n_cand, const int32_t* cand_sky,
                       const double* cand, const double* grad_p, double* grad_out, double* abs_out)
{
    int err = ORC_OK;
    #pragma omp parallel for schedule(static) reduction(min:err)
    for (int64_t c = 0; c < n_cand; ++c) {
        const double* th = cand + 6 * c;
        const double F = th[0], ap = th[1], per = th[2], ta = th[3], ec = th[4], es = th[5];
        const float* w = weight + (weight_per_sky ? (int64_t)cand_sky[c] * n_seg : 0);
        double g[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t J = 0; J < n_seg; ++J) {
            double D = doppler_factor(v_over_c + 3 * J, sky + 3 * cand_sky[c]);
            double W = TWO_PI / per;
            double psi = W * (t_mid[J] - ta);
            double c1 = cos(psi), s1 = sin(psi);
            double c2 = cos(2.0 * psi), s2 = sin(2.0 * psi);
            double E = c1 + (ec * c2 - es * s2);
            double Ep = -s1 - 2.0 * (ec * s2) - 2.0 * (es * c2);
            double B = 1.0 - (ap * W) * E;
            double x = F * (D * B);
            double kf = floor(x);
            int64_t col = (int64_t)kf - k_lo;
            if (col < 0 || col + 1 >= n_bins) { err = ORC_ERANGE; continue; }
            const float* row = power + J * n_bins;
            double S = (double)w[J] * ((double)row[col + 1] - (double)row[col]);
            double FD = F * D;
            double t[6];
            t[0] = S * (D * B);
            t[1] = S * (-FD * W * E);
            t[2] = S * (FD * ap * (W / per) * (E + psi * Ep));
            t[3] = S * (FD * ap * W * W * Ep);
            t[4] = S * (-FD * ap * W * c2);
            t[5] = S * (FD * ap * W * s2);
            for (int q = 0; q < 6; ++q) {
                g[q] += t[q];
                a[q] += fabs(t[q]);
            }
        }
        const double sc = grad_p ? grad_p[c] : 1.0;
        for (int q = 0; q < 6; ++q) {
            grad_out[6 * c + q] = sc * g[q];
            if (abs_out) abs_out[6 * c + q] = fabs(sc) * a[q];
        }
    }
    return err;
}

/* Peakgram: bit c of row J set iff rho_{J,c} > rho_th (Sec. IV.A), bit b of word w = column 32w+b. */
void orc_peakgram(int64_t n_seg, int32_t n_bins, const float* power, double rho_th,
                  int32_t n_words, uint32_t* bits)
{
    for (int64_t J = 0; J < n_seg; ++J) {
        for (int32_t w = 0; w < n_words; ++w) bits[J * n_words + w] = 0u;
        for (int32_t c = 0; c < n_bins; ++c)
            if ((double)power[J * n_bins + c] > rho_th)
                bits[J * n_words + c / 32] |= 1u << (c % 32);
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
