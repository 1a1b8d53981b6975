"""TEST INFRASTRUCTURE ONLY: the CPU oracle of the binary Hough search.

A plain, slow, FP64 reference written from Covas & Sintes, "BinarySkyHough"
(arXiv:1904.04873).  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library never
does, and the two share no code.  The heavy loops live in ``bsh_oracle.c``
(plain C, no floating-point contraction, OpenMP over templates); the grid
enumeration, significances and top-k selection are written here in NumPy.

Functions and the passage each follows:

* ``grid_tables``      -- template bank: f0 on bin centres (delta f = 1/Tc),
                          a_p and P value lists, t_asc spread over one period
                          around mid-time (Sec. IV.C "Resolution" and "Range
                          of parameter space"; spacing rule eq:binaryres).
* ``hough_count``      -- stage-1 weighted number count (Sec. IV.C, eq:hough2).
* ``power_stat``       -- stage-2 weighted power on the exact track (eq:hough3),
                          nearest bin or the bin-interpolated extension.
* ``power_grad``       -- gradient of the interpolated power (extension).
* ``track``            -- the frequency track x_J = f(t_J) Tc and its bins
                          (eq:frequencyevoFinal, product form).
* ``track_ecc`` / ``power_stat_ecc`` / ``hough_count_ecc`` / ``power_grad_ecc`` --
                          the low-eccentricity (ELL1) track of eq:frequencyevo, the
                          stage-2 power on it, the stage-1 count of a grid with one
                          eccentricity pair, and the interpolated power's gradient with
                          respect to the six track parameters.
* ``normalize``        -- normalized power rho = |x|^2 / <n>^2 with the noise level from a
                          running median over 101 bins (eq:HoughPower).
* ``peakgram``         -- thresholded peakgram (Sec. IV.A).
* ``significance_h`` / ``significance_p`` -- eq:hough2 / eq:hough3 with the
                          noise moments that follow from p(rho) = exp(-rho).
* ``topk``             -- best k under (score descending, index ascending).

Every function is pinned by the CPU tests.  The two significance normalizations
(whose constants the paper defers to the SkyHough paper) are pinned by the noise law
of Sec. IV.F: under p(rho) = exp(-rho) both have mean 0 and variance 1 for any weights.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bsh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TWO_PI = 6.283185307179586
NEAR_TIE = 1e-9
P_PEAK_DEFAULT_TH = 1.6


def build(force: bool = False) -> str:
    """Compile the oracle's C part (gcc, FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_hough_count.argtypes = [i64, P, P, P, i32, i64, i32, P, f64, i32, P, i64, i32,
                                      i32, P, i32, P, P, P, i32, P, P, P, P]
        L.orc_hough_count.restype = ctypes.c_int
        L.orc_track.argtypes = [i64, P, P, P, i64, P, P, i32, P, P]
        L.orc_track.restype = None
        L.orc_power_stat.argtypes = [i64, P, P, P, i32, i64, i32, P, f64, P, i64, P, P, i32,
                                     P, P, P, P]
        L.orc_power_stat.restype = ctypes.c_int
        L.orc_power_grad.argtypes = [i64, P, P, P, i32, i64, i32, P, P, i64, P, P, P, P, P]
        L.orc_power_grad.restype = ctypes.c_int
        L.orc_track_ecc.argtypes = [i64, P, P, P, i64, P, P, P, P]
        L.orc_track_ecc.restype = None
        L.orc_power_stat_ecc.argtypes = [i64, P, P, P, i32, i64, i32, P, P, i64, P, P, i32, P, P]
        L.orc_power_stat_ecc.restype = ctypes.c_int
        L.orc_hough_count_ecc.argtypes = [i64, P, P, P, i32, i64, i32, P, f64, i32, P, i64, i32,
                                          i32, P, i32, P, P, P, f64, f64, P, P, P, P]
        L.orc_hough_count_ecc.restype = ctypes.c_int
        L.orc_power_grad_ecc.argtypes = [i64, P, P, P, i32, i64, i32, P, P, i64, P, P, P, P, P]
        L.orc_power_grad_ecc.restype = ctypes.c_int
        L.orc_peakgram.argtypes = [i64, i32, P, f64, i32, P]
        L.orc_peakgram.restype = None
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class OracleRangeError(RuntimeError):
    """A frequency track left the staged row of bins."""


# --------------------------------------------------------------------------
# template bank (Sec. IV.C: delta f = 1/Tc; t_asc in [t_mid - P/2, t_mid + P/2))
# --------------------------------------------------------------------------

def linspace_inclusive(lo: float, hi: float, n: int) -> np.ndarray:
    """n values lo + i*((hi-lo)/(n-1)), the last one set to hi exactly."""
    if n == 1:
        return np.array([lo], dtype=np.float64)
    step = (hi - lo) / (n - 1)
    out = np.array([lo + i * step for i in range(n)], dtype=np.float64)
    out[-1] = hi
    return out


def tasc_points(spec, a_p: float, period: float) -> int:
    """t_asc points of one (a_p, P) cell.

    The spacing of eq:binaryres, delta t_asc = sqrt(6 m_t)/(pi Tc f a_p Omega^2),
    spread over one period gives P / delta t_asc = 2 pi^2 Tc f a_p Omega / sqrt(6 m_t);
    with the constant m = 2 pi^2 / sqrt(6 m_t) this is m Tc f a_p Omega, taken at the
    band's upper edge and clamped (reading of the garbled per-cell rule).
    """
    if spec.tasc_fixed:
        return int(spec.tasc_fixed)
    omega = TWO_PI / period
    n = math.ceil(spec.tasc_rule_m * spec.t_coh * spec.f_hi * a_p * omega)
    return int(min(max(n, spec.tasc_min), spec.tasc_max))


def grid_tables(spec, t_mid: float):
    """(a_p[n_ap], P[n_per], tasc_off[n_ap*n_per+1], t_asc[n_bin]) for one band.

    Cells are ordered a_p-major; inside a cell t_asc_j = t_mid - P/2 + j (P/N).
    """
    a_p = linspace_inclusive(spec.ap_lo, spec.ap_hi, spec.n_ap)
    per = linspace_inclusive(spec.per_lo, spec.per_hi, spec.n_per)
    counts = [tasc_points(spec, float(a), float(p)) for a in a_p for p in per]
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    t_asc = np.empty(int(off[-1]), dtype=np.float64)
    for ia in range(spec.n_ap):
        for ip in range(spec.n_per):
            cell = ia * spec.n_per + ip
            n = counts[cell]
            P = float(per[ip])
            base = t_mid - 0.5 * P
            step = P / n
            for j in range(n):
                t_asc[off[cell] + j] = base + j * step
    return a_p, per, off, t_asc


def decode_index(idx: np.ndarray, n_bin: int, n_f0: int, off: np.ndarray, n_per: int):
    """Template index -> (sky, b, i, a_p index, P index)."""
    idx = np.asarray(idx, dtype=np.int64)
    i = idx % n_f0
    sb = idx // n_f0
    b = sb % n_bin
    s = sb // n_bin
    cell = np.searchsorted(off, b, side="right") - 1
    return s, b, i, cell // n_per, cell % n_per


# --------------------------------------------------------------------------
# thin ctypes wrappers over the C definitions
# --------------------------------------------------------------------------

def hough_count(seg, sky: np.ndarray, k0: int, n_f0: int, a_p, per, off, t_asc,
                rho_th: float = P_PEAK_DEFAULT_TH, additive: bool = False,
                weight_per_sky: bool = False):
    """Stage-1 count over every template: (count u32, n_w f64, near-tie count, near-tie weight)."""
    t = _c(seg.t_mid, np.float64)
    v = _c(seg.v_over_c, np.float64)
    w = _c(seg.weight, np.float32)
    pw = _c(seg.power, np.float32)
    sky = _c(sky, np.float64)
    a_p, per, off, t_asc = (_c(a_p, np.float64), _c(per, np.float64), _c(off, np.int64),
                            _c(t_asc, np.float64))
    n_t = sky.shape[0] * int(off[-1]) * n_f0
    cnt = np.zeros(n_t, np.uint32)
    nw = np.zeros(n_t, np.float64)
    nt = np.zeros(n_t, np.uint32)
    ntw = np.zeros(n_t, np.float64)
    rc = lib().orc_hough_count(t.size, _p(t), _p(v), _p(w), int(weight_per_sky), seg.k_lo,
                               seg.n_bins, _p(pw), rho_th, sky.shape[0], _p(sky), k0, n_f0,
                               a_p.size, _p(a_p), per.size, _p(per), _p(off), _p(t_asc),
                               int(additive), _p(cnt), _p(nw), _p(nt), _p(ntw))
    if rc != 0:
        raise OracleRangeError("a track left the staged bins")
    return cnt, nw, nt, ntw


def track(seg, sky: np.ndarray, cand_sky, cand: np.ndarray, additive: bool = False):
    """Continuous x = f(t_J) Tc and absolute bins for each candidate, both [n_cand, n_seg]."""
    t = _c(seg.t_mid, np.float64)
    v = _c(seg.v_over_c, np.float64)
    sky = _c(sky, np.float64)
    cand = _c(cand, np.float64).reshape(-1, 4)
    cs = _c(cand_sky, np.int32).reshape(-1)
    x = np.empty((cand.shape[0], t.size), np.float64)
    k = np.empty((cand.shape[0], t.size), np.int64)
    lib().orc_track(t.size, _p(t), _p(v), _p(sky), cand.shape[0], _p(cs), _p(cand),
                    int(additive), _p(x), _p(k))
    return x, k


def power_stat(seg, sky, cand_sky, cand, mode: int = 0, rho_th: float = P_PEAK_DEFAULT_TH,
               weight_per_sky: bool = False):
    """Per candidate: (P or P_lin, count, n_w, near-tie count)."""
    t = _c(seg.t_mid, np.float64)
    v = _c(seg.v_over_c, np.float64)
    w = _c(seg.weight, np.float32)
    pw = _c(seg.power, np.float32)
    sky = _c(sky, np.float64)
    cand = _c(cand, np.float64).reshape(-1, 4)
    cs = _c(cand_sky, np.int32).reshape(-1)
    n = cand.shape[0]
    P = np.zeros(n, np.float64)
    cnt = np.zeros(n, np.uint32)
    nw = np.zeros(n, np.float64)
    nt = np.zeros(n, np.uint32)
    rc = lib().orc_power_stat(t.size, _p(t), _p(v), _p(w), int(weight_per_sky), seg.k_lo,
                              seg.n_bins, _p(pw), rho_th, _p(sky), n, _p(cs), _p(cand),
                              int(mode), _p(P), _p(cnt), _p(nw), _p(nt))
    if rc != 0:
        raise OracleRangeError("a track left the staged bins")
    return P, cnt, nw, nt


def power_grad(seg, sky, cand_sky, cand, grad_p=None, weight_per_sky: bool = False,
               with_abs: bool = False):
    """d P_lin / d(F, a_p, P, t_asc) per candidate, [n, 4] float64 (times grad_p if given).

    With ``with_abs`` also returns the sums of the absolute per-segment terms, the scale
    against which a differently ordered summation is compared."""
    t = _c(seg.t_mid, np.float64)
    v = _c(seg.v_over_c, np.float64)
    w = _c(seg.weight, np.float32)
    pw = _c(seg.power, np.float32)
    sky = _c(sky, np.float64)
    cand = _c(cand, np.float64).reshape(-1, 4)
    cs = _c(cand_sky, np.int32).reshape(-1)
    n = cand.shape[0]
    g = np.zeros((n, 4), np.float64)
    a = np.zeros((n, 4), np.float64) if with_abs else None
    gp = None if grad_p is None else _c(grad_p, np.float64)
    rc = lib().orc_power_grad(t.size, _p(t), _p(v), _p(w), int(weight_per_sky), seg.k_lo,
                              seg.n_bins, _p(pw), _p(sky), n, _p(cs), _p(cand), _p(gp), _p(g), _p(a))
    if rc != 0:
        raise OracleRangeError("a track left the staged bins")
    return (g, a) if with_abs else g


def track_ecc(seg, sky, cand_sky, cand: np.ndarray):
    """ELL1 track: x and bins [n_cand, n_seg] for rows (F, a_p, P, t_asc, e cos w, e sin w)."""
    t = _c(seg.t_mid, np.float64)
    v = _c(seg.v_over_c, np.float64)
    sky = _c(sky, np.float64)
    cand = _c(cand, np.float64).reshape(-1, 6)
    cs = _c(cand_sky, np.int32).reshape(-1)
    x = np.empty((cand.shape[0], t.size), np.float64)
    k = np.empty((cand.shape[0], t.size), np.int64)
    lib().orc_track_ecc(t.size, _p(t), _p(v), _p(sky), cand.shape[0], _p(cs), _p(cand), _p(x), _p(k))
    return x, k


def power_stat_ecc(seg, sky, cand_sky, cand, mode: int = 0, weight_per_sky: bool = False):
    """Stage-2 power on the ELL1 track: (P, near-tie count) per candidate."""
    t = _c(seg.t_mid, np.float64)
    v = _c(seg.v_over_c, np.float64)
    w = _c(seg.weight, np.float32)
    pw = _c(seg.power, np.float32)
    sky = _c(sky, np.float64)
    cand = _c(cand, np.float64).reshape(-1, 6)
    cs = _c(cand_sky, np.int32).reshape(-1)
    n = cand.shape[0]
    P = np.zeros(n, np.float64)
    nt = np.zeros(n, np.uint32)
    rc = lib().orc_power_stat_ecc(t.size, _p(t), _p(v), _p(w), int(weight_per_sky), seg.k_lo, seg.n_bins,
                                  _p(pw), _p(sky), n, _p(cs), _p(cand), int(mode), _p(P), _p(nt))
    if rc != 0:
        raise OracleRangeError("a track left the staged bins")
    return P, nt


def hough_count_ecc(seg, sky, k0: int, n_f0: int, a_p, per, off, t_asc, ec: float, es: float,
                    rho_th: float = P_PEAK_DEFAULT_TH, weight_per_sky: bool = False):
    """Stage-1 count on the ELL1 track with one (e cos w, e sin w) pair for the whole grid:
    (count u32, n_w f64, near-tie count, near-tie weight), template order as hough_count."""
    t = _c(seg.t_mid, np.float64)
    v = _c(seg.v_over_c, np.float64)
    w = _c(seg.weight, np.float32)
    pw = _c(seg.power, np.float32)
    sky = _c(sky, np.float64)
    a_p, per, off, t_asc = (_c(a_p, np.float64), _c(per, np.float64), _c(off, np.int64),
                            _c(t_asc, np.float64))
    n_t = sky.shape[0] * int(off[-1]) * n_f0
    cnt = np.zeros(n_t, np.uint32)
    nw = np.zeros(n_t, np.float64)
    nt = np.zeros(n_t, np.uint32)
    ntw = np.zeros(n_t, np.float64)
    rc = lib().orc_hough_count_ecc(t.size, _p(t), _p(v), _p(w), int(weight_per_sky), seg.k_lo,
                                   seg.n_bins, _p(pw), rho_th, sky.shape[0], _p(sky), k0, n_f0,
                                   a_p.size, _p(a_p), per.size, _p(per), _p(off), _p(t_asc),
                                   float(ec), float(es), _p(cnt), _p(nw), _p(nt), _p(ntw))
    if rc != 0:
        raise OracleRangeError("a track left the staged bins")
    return cnt, nw, nt, ntw


def power_grad_ecc(seg, sky, cand_sky, cand, grad_p=None, weight_per_sky: bool = False,
                   with_abs: bool = False):
    """d P_lin / d(F, a_p, P, t_asc, e cos w, e sin w) on the ELL1 track, [n, 6] float64."""
    t = _c(seg.t_mid, np.float64)
    v = _c(seg.v_over_c, np.float64)
    w = _c(seg.weight, np.float32)
    pw = _c(seg.power, np.float32)
    sky = _c(sky, np.float64)
    cand = _c(cand, np.float64).reshape(-1, 6)
    cs = _c(cand_sky, np.int32).reshape(-1)
    n = cand.shape[0]
    g = np.zeros((n, 6), np.float64)
    a = np.zeros((n, 6), np.float64) if with_abs else None
    gp = None if grad_p is None else _c(grad_p, np.float64)
    rc = lib().orc_power_grad_ecc(t.size, _p(t), _p(v), _p(w), int(weight_per_sky), seg.k_lo,
                                  seg.n_bins, _p(pw), _p(sky), n, _p(cs), _p(cand), _p(gp), _p(g), _p(a))
    if rc != 0:
        raise OracleRangeError("a track left the staged bins")
    return (g, a) if with_abs else g


def median_bias(window: int) -> float:
    """Expected median of `window` (odd) i.i.d. Exp(1) values: sum_{i=m+1}^{2m+1} 1/i, window = 2m+1."""
    m = (window - 1) // 2
    return float(sum(1.0 / i for i in range(m + 1, 2 * m + 2)))


def normalize(raw: np.ndarray, window: int = 101) -> np.ndarray:
    """eq:HoughPower: rho_k = P_k / <n_k>^2 with <n_k>^2 = median(P_{k-m..k+m}) / beta, beta the
    expected median of `window` unit exponentials.  Output column c is raw column c + m;
    rho = (float32)((P * beta) / median) evaluated in double precision."""
    from numpy.lib.stride_tricks import sliding_window_view
    raw = np.asarray(raw, np.float32)
    m = (window - 1) // 2
    med = np.median(sliding_window_view(raw, window, axis=1), axis=2)      # exact: odd window
    beta = median_bias(window)
    centre = raw[:, m:raw.shape[1] - m].astype(np.float64)
    return ((centre * beta) / med.astype(np.float64)).astype(np.float32)


def peakgram(power: np.ndarray, rho_th: float = P_PEAK_DEFAULT_TH) -> np.ndarray:
    """Bit-packed peakgram [n_seg, ceil(n_bins/32)] uint32 (bit b of word w = column 32w+b)."""
    pw = _c(power, np.float32)
    n_seg, n_bins = pw.shape
    n_words = (n_bins + 31) // 32
    bits = np.zeros((n_seg, n_words), np.uint32)
    lib().orc_peakgram(n_seg, n_bins, _p(pw), rho_th, n_words, _p(bits))
    return bits


# --------------------------------------------------------------------------
# significances and top-k (Sec. IV.C)
# --------------------------------------------------------------------------

def peak_probability(rho_th: float = P_PEAK_DEFAULT_TH) -> float:
    """P(rho > rho_th) for the Gaussian-noise law p(rho) = exp(-rho) (Sec. V.F)."""
    return math.exp(-rho_th)


def significance_h(n_w, w: np.ndarray, rho_th: float = P_PEAK_DEFAULT_TH):
    """s_H = (n - <n>)/sigma_H with Bernoulli(p0) peaks: <n> = p0 sum w, sigma^2 = p0(1-p0) sum w^2."""
    p0 = peak_probability(rho_th)
    w = np.asarray(w, np.float64)
    return (np.asarray(n_w, np.float64) - p0 * w.sum()) / math.sqrt(p0 * (1 - p0) * (w * w).sum())


def significance_p(P, w: np.ndarray):
    """s_P = (P - <P>)/sigma_P with Exp(1) powers: <P> = sum w, sigma^2 = sum w^2."""
    w = np.asarray(w, np.float64)
    return (np.asarray(P, np.float64) - w.sum()) / math.sqrt((w * w).sum())


def topk(score: np.ndarray, k: int, index: Optional[np.ndarray] = None
         ) -> Tuple[np.ndarray, np.ndarray]:
    """The k best entries under (score descending, index ascending): (scores, indices)."""
    score = np.asarray(score)
    index = np.arange(score.size, dtype=np.int64) if index is None else np.asarray(index, np.int64)
    order = np.lexsort((index, -score.astype(np.float64)))[:k]
    return score[order], index[order]
