// Internal helpers of libbsh: error state, argument checks and the device-side
// evaluation of the frequency track.  Not part of the public ABI (include/bsh.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/bsh.h"

namespace bsh {

// Nearest double to 2 pi; the orbital angular frequency is W = TWO_PI / P.
constexpr double kTwoPi = 6.283185307179586;

// ---------------------------------------------------------------- host error state

void set_error(const char* fmt, ...);
void clear_error();

inline int fail_inval(const char* what)
{
    set_error("invalid argument: %s", what);
    return BSH_EINVAL;
}

inline int check_launch(const char* where)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: %s", where, hipGetErrorString(e));
        return BSH_EHIP;
    }
    return BSH_OK;
}

inline int words_for(int32_t n_bins) { return (n_bins + 31) / 32; }

// Host-side validation of a segment table; `need_bits` / `need_power` select the rows.
int check_segments(const bsh_segments* seg, bool need_bits, bool need_power);
// Host-side validation of a grid (small host tables are read).
int check_grid(const bsh_grid* g);
// Conservative host check that every stage-1 track stays inside the staged row.
int check_window(const bsh_segments* seg, const bsh_grid* g);
// True when v_max_host is given, the staged row covers every track's bound with the margin of
// check_window, and the band's offsets drift by less than half a bin (at most one f0-shift
// step); *v and *apw receive the bounds on |v/c| and a_p W (1 + e) that the proof used.
bool proven_window(const bsh_segments* seg, const bsh_grid* g, double* v, double* apw);

// Segmented exact top-k (bsh_topk.hip): offsets on the device, longest segment from the host.
// With implicit indices (index NULL) the written indices are index_base + ((g << shift) | position);
// the order among a segment's entries does not depend on the base.
size_t topk_workspace_bytes(int32_t n_segs, int32_t k);
// A workspace of this size lets a segmented call with long segments take the candidate pass.
size_t topk_candidate_workspace_bytes(int32_t n_segs, int32_t k);
int topk_segmented(const float* score, const int64_t* index, const int64_t* offsets, int32_t n_segs,
                   int64_t max_len, int32_t shift, int32_t k, float* out_score, int64_t* out_index,
                   void* ws, size_t ws_bytes, hipStream_t stream, int64_t index_base = 0);

// ---------------------------------------------------------------- device track

// sin and cos of an orbital phase x (|x| < 2^20 rad; the tracks' phases stay below 10^3) by
// Cody and Waite's additive range reduction: k = nearest integer to x 2/pi, r = x - k pi/2
// with pi/2 split into three doubles, the first two of 33 significant bits (so k times them is
// exact for |k| < 2^20 and the first subtraction is exact), then the Taylor series of sin and
// cos at r in [-pi/4, pi/4] through r^15/15! and r^16/16! (the first omitted terms are below
// 5e-17 and 3e-18) and the quadrant k mod 4.  Every kernel takes cos and sin of W t and of
// W t_asc from here, so all of them see the same values.
__device__ __forceinline__ void track_sincos(double x, double& s, double& c)
{
    constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
    constexpr double kP1 = 0x1.921fb544p+0;
    constexpr double kP2 = 0x1.0b4611a6p-34;
    constexpr double kP3 = 0x1.3198a2e037073p-69;
    const double k = rint(x * kTwoOverPi);
    double r = fma(-k, kP1, x);
    r = fma(-k, kP2, r);
    r = fma(-k, kP3, r);
    const double r2 = r * r;
    double ps = -0x1.ae7f3e733b81fp-41;          // -1/15!
    ps = fma(ps, r2, 0x1.6124613a86d09p-33);     //  1/13!
    ps = fma(ps, r2, -0x1.ae64567f544e4p-26);    // -1/11!
    ps = fma(ps, r2, 0x1.71de3a556c734p-19);     //  1/9!
    ps = fma(ps, r2, -0x1.a01a01a01a01ap-13);    // -1/7!
    ps = fma(ps, r2, 0x1.1111111111111p-7);      //  1/5!
    ps = fma(ps, r2, -0x1.5555555555555p-3);     // -1/3!
    const double sr = fma(r * r2, ps, r);
    double pc = 0x1.ae7f3e733b81fp-45;           //  1/16!
    pc = fma(pc, r2, -0x1.93974a8c07c9dp-37);    // -1/14!
    pc = fma(pc, r2, 0x1.1eed8eff8d898p-29);     //  1/12!
    pc = fma(pc, r2, -0x1.27e4fb7789f5cp-22);    // -1/10!
    pc = fma(pc, r2, 0x1.a01a01a01a01ap-16);     //  1/8!
    pc = fma(pc, r2, -0x1.6c16c16c16c17p-10);    // -1/6!
    pc = fma(pc, r2, 0x1.5555555555555p-5);      //  1/4!
    pc = fma(pc, r2, -0.5);                      // -1/2!
    const double cr = fma(r2, pc, 1.0);
    // x = k pi/2 + r: quadrant 1 swaps sin and cos, quadrants 2 and 3 flip the signs
    const int q = (int)k & 3;
    const double s0 = (q & 1) ? cr : sr;
    const double c0 = (q & 1) ? sr : cr;
    s = (q & 2) ? -s0 : s0;
    c = ((q + 1) & 2) ? -c0 : c0;
}

// Doppler factor D = 1 + v.n, one fixed operation order (no contraction: the library is
// built with -ffp-contract=off).
__device__ __forceinline__ double doppler_factor(const double* v, double nx, double ny, double nz)
{
    double d = v[0] * nx + v[1] * ny;
    d = d + v[2] * nz;
    return 1.0 + d;
}

// A candidate template (F = f0 Tc, a_p, P, t_asc) with the quantities every segment reuses:
// W = 2 pi / P, a_p W, cos / sin of W t_asc and A_c = a_p W cos(W t_asc), A_s = a_p W sin(W t_asc).
struct Cand {
    double F, ap, P, ta, W, apW, cb, sb, Ac, As;
};

__device__ __forceinline__ Cand load_cand(const double* cand)
{
    Cand c;
    c.F = cand[0];
    c.ap = cand[1];
    c.P = cand[2];
    c.ta = cand[3];
    c.W = kTwoPi / c.P;
    c.apW = c.ap * c.W;
    track_sincos(c.W * c.ta, c.sb, c.cb);
    c.Ac = c.apW * c.cb;
    c.As = c.apW * c.sb;
    return c;
}

// cos and sin of the orbital phase W (t - t_asc), from cos / sin of W t and W t_asc by the
// angle-difference formulas (for the eccentric track and the derivatives; bins come from
// track_G).
__device__ __forceinline__ void orbit_phase(double ct, double st, const Cand& c, double& cphi,
                                            double& sphi)
{
    cphi = fma(ct, c.cb, st * c.sb);
    sphi = fma(st, c.cb, -(ct * c.sb));
}

// The track x = F G with G = D (1 - a_p W cos(W (t - t_asc)))  (eq:frequencyevoFinal, product
// form).  Expanding cos by the angle-difference formula, G = D - (D C A_c + D S A_s) with
// C, S = cos, sin of W t (per segment) and A_c, A_s of the template; it is evaluated in this
// one order, D - fma(D C, A_c, (D S) A_s), by every kernel (the stage-1 kernel stages D C and
// D S once per block), so all of them select identical bins.
__device__ __forceinline__ double track_G(double D, double DC, double DS, double Ac, double As)
{
    return D - fma(DC, Ac, DS * As);
}

// Low-eccentricity (ELL1) track of eq:frequencyevo: the orbit bracket gains
// (e cos w) cos 2psi - (e sin w) sin 2psi, psi = W (t - t_asc).  Expanding cos 2psi and sin 2psi
// by the angle-difference formulas in 2 W t and 2 W t_asc, its a_p W multiple is
// C2 A_c2 + S2 A_s2 with C2, S2 = cos, sin(2 W t) (per segment) and the template's
// A_c2 = a_p W (ec c2 + es s2), A_s2 = a_p W (ec s2 - es c2), c2, s2 = cos, sin(2 W t_asc).
// Both double angles come from cos / sin of the single angle, in this one order.
__device__ __forceinline__ void double_angle(double c, double s, double& c2, double& s2)
{
    c2 = (c - s) * (c + s);
    s2 = 2.0 * (s * c);
}

__device__ __forceinline__ void ecc_coeffs(double apW, double cb, double sb, double ec, double es, double& Ac2,
                                           double& As2)
{
    double c2, s2;
    double_angle(cb, sb, c2, s2);
    Ac2 = apW * (ec * c2 + es * s2);
    As2 = apW * (ec * s2 - es * c2);
}

// G on the ELL1 track: the circular G minus D (C2 A_c2 + S2 A_s2), evaluated as
// track_G(...) - fma(D C2, A_c2, (D S2) A_s2) by every kernel.  With zero eccentricity A_c2 and
// A_s2 are zeros and G is the circular track_G bit for bit.
__device__ __forceinline__ double track_G_ecc(double D, double DC, double DS, double Ac, double As, double DC2,
                                              double DS2, double Ac2, double As2)
{
    return track_G(D, DC, DS, Ac, As) - fma(DC2, Ac2, DS2 * As2);
}

// Nearest bin of the track: floor(F G + 1/2), with F G + 1/2 rounded once.
__device__ __forceinline__ double track_bin(double F, double G) { return floor(fma(F, G, 0.5)); }

__device__ __forceinline__ void raise_status(int32_t* status, int32_t bit)
{
    if (status) atomicOr(status, bit);
}

// Wave64 sum (all lanes end with the total).
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace bsh
