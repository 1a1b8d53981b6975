"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's own formula as its expectation:
each expected value comes from a special case with a textbook answer, an
equation the paper prints separately (the phase model, the frequency
derivative, the Doppler bin count), brute force at 50 digits, a
finite-difference of an independent quantity, or a statistical law.
"""
import json
import math
import os

import numpy as np
import pytest

import bsh_synth as S
import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
TC = S.T_COH


def _grid_from(a_p, per, t_asc_cells):
    """Explicit grid tables from per-cell t_asc lists (cells a_p-major)."""
    a_p = np.asarray(a_p, np.float64)
    per = np.asarray(per, np.float64)
    counts = [len(c) for c in t_asc_cells]
    off = np.zeros(len(counts) + 1, np.int64)
    off[1:] = np.cumsum(counts)
    return a_p, per, off, np.concatenate([np.asarray(c, np.float64) for c in t_asc_cells])


def _segments(n, k0, n_f0, margin, seed, v=None, span_days=60.0, weight=None):
    rng = np.random.default_rng(seed)
    t0 = np.sort(rng.uniform(0, span_days * S.DAY, n))
    t = t0 + 0.5 * TC
    vv = S.velocity_over_c(t) if v is None else np.broadcast_to(np.asarray(v, np.float64), (n, 3)).copy()
    k_lo, n_bins = S.band_window(k0, n_f0, margin)
    w = S.lognormal_weights(rng, n) if weight is None else np.full(n, weight, np.float32)
    return S.Segments(t_mid=t, v_over_c=vv, weight=w, power=S.exp1_powers(rng, n, n_bins),
                      k_lo=k_lo, n_bins=n_bins)


# ---------------------------------------------------------------- constants

def test_paper_constants():
    assert GOLD["t_coh_s"]["value"] == S.T_COH
    assert GOLD["rho_th"]["value"] == S.RHO_TH
    assert abs(O.peak_probability(1.6) - GOLD["peak_probability_at_1p6"]["value"]) < 1e-15
    # 90 frequency templates per 0.1 Hz band at delta f = 1/Tc (Sec. IV.F)
    assert round(0.1 * GOLD["t_coh_s"]["value"]) == GOLD["n_f0_per_0p1Hz_band"]["value"]
    for cfg in (S.config1(), S.config2()):
        assert cfg.grids[0].n_f0 == 90


# ---------------------------------------------------------------- track formula

def test_track_orbit_extremes_at_special_phases():
    """v = 0: f(t_asc) = f0 (1 - a_p W), f(t_asc + P/2) = f0 (1 + a_p W), f(t_asc +- P/4) = f0."""
    F, ap, P, ta = 90012.0, 2.5, 20 * S.DAY, 3.0e6
    W = 2 * math.pi / P
    times = np.array([ta, ta + P / 2, ta + P / 4, ta - P / 4, ta + P])
    seg = S.Segments(t_mid=times, v_over_c=np.zeros((5, 3)), weight=np.ones(5, np.float32),
                     power=np.zeros((5, 1), np.float32), k_lo=0, n_bins=1)
    x, _ = O.track(seg, np.array([[0, 0, 1.0]]), [0], np.array([[F, ap, P, ta]]))
    x = x[0]
    assert x[0] == pytest.approx(F * (1 - ap * W), abs=1e-9)
    assert x[1] == pytest.approx(F * (1 + ap * W), abs=1e-9)
    assert x[2] == pytest.approx(F, abs=1e-9)
    assert x[3] == pytest.approx(F, abs=1e-9)
    assert x[4] == pytest.approx(x[0], abs=1e-9)


def test_track_doppler_bins_match_n0():
    """a_p = 0, v parallel to n: the shift in bins equals n0 = f v / (c delta f) (Sec. IV.B)."""
    vabs = 1.0e-4
    F = 270000.0
    seg = S.Segments(t_mid=np.array([0.0, 0.0]), v_over_c=np.array([[vabs, 0, 0], [-vabs, 0, 0]]),
                     weight=np.ones(2, np.float32), power=np.zeros((2, 1), np.float32),
                     k_lo=0, n_bins=1)
    x, _ = O.track(seg, np.array([[1.0, 0.0, 0.0]]), [0], np.array([[F, 0.0, S.DAY, 0.0]]))
    f0 = F / TC
    n0 = f0 * vabs / (1.0 / TC)
    assert x[0, 0] - F == pytest.approx(n0, rel=1e-12)
    assert F - x[0, 1] == pytest.approx(n0, rel=1e-12)


def test_track_is_time_derivative_of_phase_model():
    """f(t) = (1/2pi) d phi/dt with phi from eq:phaseMethod (e = 0, r.n = v.n t for constant v).

    The phase model is a different printed equation than the frequency track;
    central differences of the phase must reproduce the oracle's x / Tc.  The
    additive flag reproduces it exactly; the canonical product form differs by
    the second-order term f0 (v.n) a_p W cos, under 1e-3 bins here.
    """
    f0, ap, P, ta = 300.04, 3.1, 17 * S.DAY, 1.1e6
    v = np.array([0.6e-4, -0.7e-4, 0.2e-4])
    n = np.array([0.48, 0.6, 0.64])
    n = n / np.linalg.norm(n)
    W = 2 * math.pi / P
    times = np.linspace(0.3e6, 2.5e6, 23)

    def phase(t):  # cycles; eq:phaseMethod with e = 0
        return f0 * (t + (v @ n) * t - ap * math.sin(W * (t - ta)))

    h = 1.0
    f_num = np.array([(phase(t + h) - phase(t - h)) / (2 * h) for t in times])
    seg = S.Segments(t_mid=times, v_over_c=np.tile(v, (times.size, 1)), weight=np.ones(times.size, np.float32),
                     power=np.zeros((times.size, 1), np.float32), k_lo=0, n_bins=1)
    cand = np.array([[f0 * TC, ap, P, ta]])
    x_add, _ = O.track(seg, n[None, :], [0], cand, additive=True)
    x_prod, _ = O.track(seg, n[None, :], [0], cand)
    assert np.max(np.abs(x_add[0] - f_num * TC)) < 2e-4
    assert np.max(np.abs(x_prod[0] - f_num * TC)) < 1e-3
    assert np.max(np.abs(x_prod[0] - x_add[0])) > 1e-6   # the two forms really differ


def test_track_derivative_matches_eq_derivative():
    """d f/dt of the track equals f0 a_p W^2 sin(W (t - t_asc)) (eq:derivative, constant v)."""
    F, ap, P, ta = 180033.0, 1.7, 23 * S.DAY, 0.7e6
    W = 2 * math.pi / P
    times = np.linspace(1e5, 2.4e6, 31)
    h = 30.0
    seg_p = S.Segments(t_mid=times + h, v_over_c=np.zeros((31, 3)), weight=np.ones(31, np.float32),
                       power=np.zeros((31, 1), np.float32), k_lo=0, n_bins=1)
    seg_m = S.Segments(t_mid=times - h, v_over_c=np.zeros((31, 3)), weight=np.ones(31, np.float32),
                       power=np.zeros((31, 1), np.float32), k_lo=0, n_bins=1)
    sky = np.array([[0, 0, 1.0]])
    cand = np.array([[F, ap, P, ta]])
    xp, _ = O.track(seg_p, sky, [0], cand)
    xm, _ = O.track(seg_m, sky, [0], cand)
    fdot_num = (xp[0] - xm[0]) / (2 * h) / TC
    fdot_paper = (F / TC) * ap * W * W * np.sin(W * (times - ta))
    assert np.max(np.abs(fdot_num - fdot_paper)) < 1e-6 * np.max(np.abs(fdot_paper))


def test_bins_brute_force_50_digits():
    """Bins of the oracle equal floor(x + 1/2) evaluated in 50-digit arithmetic."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    seg = _segments(6, 1000, 3, 4, seed=11)
    sky = S.fibonacci_sphere(3)
    rng = np.random.default_rng(5)
    cand = np.stack([1000 + rng.uniform(0, 3, 12), rng.uniform(0.1, 3, 12),
                     rng.uniform(15, 45, 12) * S.DAY, rng.uniform(0, 3e6, 12)], axis=1)
    cs = rng.integers(0, 3, 12)
    x, k = O.track(seg, sky, cs, cand)
    two_pi = 2 * mp.pi
    for c in range(12):
        Fm, apm, Pm, tam = (mp.mpf(float(v)) for v in cand[c])
        nvec = [mp.mpf(float(v)) for v in sky[cs[c]]]
        for J in range(seg.n_seg):
            vv = [mp.mpf(float(q)) for q in seg.v_over_c[J]]
            t = mp.mpf(float(seg.t_mid[J]))
            W = two_pi / Pm
            xe = Fm * (1 + sum(a * b for a, b in zip(vv, nvec))) * (1 - apm * W * mp.cos(W * (t - tam)))
            assert abs(float(xe) - x[c, J]) < 1e-9
            assert int(mp.floor(xe + mp.mpf("0.5"))) == k[c, J]


# ---------------------------------------------------------------- stage-1 count

def test_count_brute_force_tiny_grid():
    """Counts and weighted counts on a 4-segment, 3-f0, 2x2x2 grid against a 50-digit evaluation."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    seg = _segments(4, 1000, 3, 4, seed=3)
    seg.power[:] = np.random.default_rng(9).exponential(1.0, seg.power.shape).astype(np.float32)
    sky = S.fibonacci_sphere(2)
    a_p = [0.7, 2.9]
    per = [16 * S.DAY, 31 * S.DAY]
    cells = [[1.0e5, 9.0e5], [2.0e5, 1.3e6], [3.0e5, 4.0e5], [5.0e5, 2.2e6]]
    a_p, per, off, ta = _grid_from(a_p, per, cells)
    cnt, nw, nt, _ = O.hough_count(seg, sky, 1000, 3, a_p, per, off, ta)
    assert nt.sum() == 0
    idx = 0
    for s in range(2):
        for b in range(off[-1]):
            cell = np.searchsorted(off, b, side="right") - 1
            ap, P = a_p[cell // 2], per[cell % 2]
            for i in range(3):
                c_exp, w_exp = 0, 0.0
                for J in range(4):
                    W = 2 * mp.pi / mp.mpf(float(P))
                    d = sum(mp.mpf(float(u)) * mp.mpf(float(q)) for u, q in zip(seg.v_over_c[J], sky[s]))
                    xe = (1000 + i) * (1 + d) * (1 - mp.mpf(float(ap)) * W *
                                                  mp.cos(W * (mp.mpf(float(seg.t_mid[J])) - mp.mpf(float(ta[b])))))
                    col = int(mp.floor(xe + mp.mpf("0.5"))) - seg.k_lo
                    if seg.power[J, col] > 1.6:
                        c_exp += 1
                        w_exp += float(seg.weight[J])
                assert cnt[idx] == c_exp
                assert nw[idx] == pytest.approx(w_exp, rel=1e-12)
                idx += 1


def test_count_no_motion_is_column_popcount():
    """v = 0 and a_p = 0: x = F exactly, so count_i is the number of peaks in column k0 + i."""
    seg = _segments(50, 5000, 20, 3, seed=4, v=[0, 0, 0], weight=1.0)
    a_p, per, off, ta = _grid_from([0.0], [20 * S.DAY], [[0.0, 1e6, 2e6]])
    cnt, nw, nt, _ = O.hough_count(seg, S.fixed_pixel(), 5000, 20, a_p, per, off, ta)
    col = (seg.power > 1.6).sum(axis=0)[3:23]
    for b in range(3):
        assert np.array_equal(cnt[b * 20:(b + 1) * 20], col)
    assert nt.sum() == 0


def test_count_ap_zero_independent_of_orbit():
    """a_p = 0 reduces to the isolated-star count (f1 = 0): independent of P and t_asc."""
    seg = _segments(200, 20000, 30, 6, seed=5)
    a_p, per, off, ta = _grid_from([0.0], [15 * S.DAY, 40 * S.DAY],
                                   [[0.0, 3.3e5, 2.9e6], [1.0e6, 7.7e6]])
    cnt, nw, nt, _ = O.hough_count(seg, S.fixed_pixel(), 20000, 30, a_p, per, off, ta)
    cnt = cnt.reshape(5, 30)
    nw = nw.reshape(5, 30)
    for b in range(1, 5):
        assert np.array_equal(cnt[b], cnt[0])
        assert np.array_equal(nw[b], nw[0])


def test_count_noiseless_injection():
    """rho = 0 except 2 on the true template's track: count = N and n_w = sum w there, 0 elsewhere far away."""
    seg = _segments(300, 180000, 90, 22, seed=6)
    seg.power[:] = 0
    g = S.GridSpec(k0=180000, n_f0=90, ap_lo=0.5, ap_hi=2.5, n_ap=3, per_lo=15 * S.DAY,
                   per_hi=30 * S.DAY, n_per=2, tasc_fixed=5)
    a_p, per, off, ta = O.grid_tables(g, seg.t_span_mid())
    b_true, i_true = 17, 41
    cell = np.searchsorted(off, b_true, side="right") - 1
    cand = np.array([[180000 + i_true, a_p[cell // 2], per[cell % 2], ta[b_true]]])
    _, k = O.track(seg, S.fixed_pixel(), [0], cand)
    seg.power[np.arange(seg.n_seg), k[0] - seg.k_lo] = 2.0
    cnt, nw, nt, _ = O.hough_count(seg, S.fixed_pixel(), 180000, 90, a_p, per, off, ta)
    idx = b_true * 90 + i_true
    assert cnt[idx] == seg.n_seg
    assert nw[idx] == pytest.approx(float(seg.weight.astype(np.float64).sum()), rel=1e-12)
    assert cnt.argmax() == idx


def test_count_tasc_period_and_sign_invariance():
    """t_asc -> t_asc + P and (a_p, t_asc) -> (-a_p, t_asc + P/2) leave every bin unchanged (near-ties aside)."""
    seg = _segments(400, 90000, 90, 12, seed=8)
    P = 21 * S.DAY
    base = [0.4e6, 1.1e6, 2.7e6]
    a1 = _grid_from([1.3], [P], [base])
    a2 = _grid_from([1.3], [P], [[t + P for t in base]])
    a3 = _grid_from([-1.3], [P], [[t + P / 2 for t in base]])
    r1 = O.hough_count(seg, S.fixed_pixel(), 90000, 90, *a1)
    r2 = O.hough_count(seg, S.fixed_pixel(), 90000, 90, *a2)
    r3 = O.hough_count(seg, S.fixed_pixel(), 90000, 90, *a3)
    ok = (r1[2] == 0) & (r2[2] == 0) & (r3[2] == 0)
    assert ok.mean() > 0.99
    assert np.array_equal(r1[0][ok], r2[0][ok])
    assert np.array_equal(r1[0][ok], r3[0][ok])


def test_count_bins_stay_inside_bound():
    """Every bin lies within k0 - m .. k0 + n_f0 - 1 + m, m = F_hi (|v| + a_p W + |v| a_p W) (Sec. IV.B n0)."""
    w = S.config1()
    seg, g = w.segments[0], w.grids[0]
    a_p, per, off, ta = O.grid_tables(g, seg.t_span_mid())
    vmax = np.linalg.norm(seg.v_over_c, axis=1).max()
    apw = (a_p[:, None] * 2 * np.pi / per[None, :]).max()
    m = (g.k0 + g.n_f0) * (vmax + apw + vmax * apw)
    rng = np.random.default_rng(0)
    bs = rng.integers(0, off[-1], 64)
    cells = np.searchsorted(off, bs, side="right") - 1
    cand = np.stack([g.k0 + rng.integers(0, 90, 64).astype(np.float64), a_p[cells // g.n_per],
                     per[cells % g.n_per], ta[bs]], axis=1)
    _, k = O.track(seg, w.sky, np.zeros(64, np.int32), cand)
    assert k.min() >= g.k0 - m - 1 and k.max() <= g.k0 + 89 + m + 1
    assert k.min() - seg.k_lo >= 0 and k.max() - seg.k_lo < seg.n_bins


def test_count_noise_mean_matches_peak_probability():
    """Under Exp(1) noise the mean count is N exp(-rho_th) and the mean n_w is exp(-rho_th) sum w."""
    p0 = O.peak_probability(1.6)
    counts, nws, sw = [], [], []
    for s in range(40):
        seg = _segments(250, 30000, 2, 6, seed=100 + s)
        a_p, per, off, ta = _grid_from([1.0], [20 * S.DAY], [[1e6]])
        c, nw, _, _ = O.hough_count(seg, S.fixed_pixel(), 30000, 1, a_p, per, off, ta)
        counts.append(c[0]); nws.append(nw[0]); sw.append(seg.weight.astype(np.float64).sum())
    N = 250
    sd_mean = math.sqrt(N * p0 * (1 - p0) / 40)
    assert abs(np.mean(counts) - N * p0) < 4.5 * sd_mean
    assert abs(np.mean(np.array(nws) / np.array(sw)) - p0) < 4.5 * math.sqrt(p0 * (1 - p0) / N / 40) * 1.2


# ---------------------------------------------------------------- stage 2 and its extension

def _cands(seg, n, k0, seed, sky_n=1):
    rng = np.random.default_rng(seed)
    return (np.stack([k0 + rng.uniform(0, 89, n), rng.uniform(0.01, 3, n),
                      rng.uniform(15, 45, n) * S.DAY, rng.uniform(0, 3e6, n)], axis=1),
            rng.integers(0, sky_n, n).astype(np.int32))


def test_power_unit_powers_give_weight_sum():
    """rho = 1 everywhere: P = P_lin = sum w exactly."""
    seg = _segments(500, 180000, 90, 22, seed=12)
    seg.power[:] = 1.0
    cand, cs = _cands(seg, 20, 180000, 1)
    sw = seg.weight.astype(np.float64).sum()
    for mode in (0, 1):
        P = O.power_stat(seg, S.fixed_pixel(), cs, cand, mode=mode)[0]
        assert np.allclose(P, sw, rtol=1e-13, atol=0)


def test_power_ramp_is_linear_in_track():
    """rho_{J,c} = c + k_lo (the absolute bin): P_lin = sum w x and P = sum w round(x)."""
    seg = _segments(300, 90000, 90, 12, seed=13)
    seg.power[:] = (np.arange(seg.n_bins, dtype=np.float64) + seg.k_lo)[None, :].astype(np.float32)
    # float32 holds integers of this size exactly
    cand, cs = _cands(seg, 15, 90000, 2)
    x, k = O.track(seg, S.fixed_pixel(), cs, cand)
    w = seg.weight.astype(np.float64)
    P_lin = O.power_stat(seg, S.fixed_pixel(), cs, cand, mode=1)[0]
    P_near = O.power_stat(seg, S.fixed_pixel(), cs, cand, mode=0)[0]
    assert np.allclose(P_lin, x @ w, rtol=1e-13)
    assert np.allclose(P_near, k.astype(np.float64) @ w, rtol=1e-13)


def test_power_count_matches_grid_count():
    """Per-candidate count / n_w at grid templates equals the full-grid stage-1 count."""
    w = S.config1()
    seg, g = w.segments[0], w.grids[0]
    a_p, per, off, ta = O.grid_tables(g, seg.t_span_mid())
    cnt, nw, _, _ = O.hough_count(seg, w.sky, g.k0, g.n_f0, a_p, per, off, ta)
    idx = np.random.default_rng(1).integers(0, cnt.size, 200)
    s, b, i, ia, ip = O.decode_index(idx, int(off[-1]), 90, off, g.n_per)
    cand = np.stack([(g.k0 + i).astype(np.float64), a_p[ia], per[ip], ta[b]], axis=1)
    _, c2, nw2, _ = O.power_stat(seg, w.sky, s.astype(np.int32), cand, mode=0)
    assert np.array_equal(c2, cnt[idx])
    assert np.allclose(nw2, nw[idx], rtol=1e-13)


def _steps(g):
    return np.array([1.0, (g.ap_hi - g.ap_lo) / (g.n_ap - 1), (g.per_hi - g.per_lo) / (g.n_per - 1)])


def test_grad_ramp_closed_form():
    """Ramp power makes P_lin = sum w x(theta): its gradient is the FD of sum w x, kink-free."""
    seg = _segments(400, 180000, 90, 22, seed=14)
    seg.power[:] = (np.arange(seg.n_bins, dtype=np.float64) + seg.k_lo)[None, :].astype(np.float32)
    cand, cs = _cands(seg, 6, 180000, 3)
    g = O.power_grad(seg, S.fixed_pixel(), cs, cand)
    w = seg.weight.astype(np.float64)
    # no kinks here, so steps are chosen to balance truncation against rounding of x ~ 1.8e5
    hs = np.array([1e-2, 5e-3, 0.5e-3 * S.DAY, 300.0])
    for q in range(4):
        cp, cm = cand.copy(), cand.copy()
        cp[:, q] += hs[q]
        cm[:, q] -= hs[q]
        xp, _ = O.track(seg, S.fixed_pixel(), cs, cp)
        xm, _ = O.track(seg, S.fixed_pixel(), cs, cm)
        fd = ((xp - xm) @ w) / (2 * hs[q])   # difference per segment before summing
        assert np.allclose(g[:, q], fd, rtol=2e-6, atol=1e-9 * np.abs(fd).max())


def test_grad_frozen_bin_fd():
    """Noise powers: with the bins k'_J frozen at theta, central FD matches the analytic gradient."""
    seg = _segments(400, 180000, 90, 22, seed=15)
    cand, cs = _cands(seg, 5, 180000, 4)
    g = O.power_grad(seg, S.fixed_pixel(), cs, cand)
    w = seg.weight.astype(np.float64)
    x0, _ = O.track(seg, S.fixed_pixel(), cs, cand)
    kf = np.floor(x0)
    rows = np.arange(seg.n_seg)

    def plin_frozen(c):
        x, _ = O.track(seg, S.fixed_pixel(), cs, c)
        a = x - kf
        col = (kf - seg.k_lo).astype(np.int64)
        r0 = seg.power[rows[None, :], col].astype(np.float64)
        r1 = seg.power[rows[None, :], col + 1].astype(np.float64)
        return ((1 - a) * r0 + a * r1) @ w

    # h = 1e-3 grid step (1/Tc in F, the a_p and P spacings, P/64 in t_asc), where rounding
    # of x ~ 1.8e5 limits the FD to ~1e-5; and larger steps, allowed because the bins are
    # frozen, where it reaches 1e-6
    for hs, tol in ((np.array([1e-3, 1e-3 * 0.05, 1e-3 * 0.5 * S.DAY, 1e-3 * 3e3]), 2e-5),
                    (np.array([1e-2, 5e-3, 0.5e-3 * S.DAY, 300.0]), 1e-6)):
        for q in range(4):
            cp, cm = cand.copy(), cand.copy()
            cp[:, q] += hs[q]
            cm[:, q] -= hs[q]
            fd = (plin_frozen(cp) - plin_frozen(cm)) / (2 * hs[q])
            scale = np.abs(fd).max() + 1e-30
            assert np.max(np.abs(g[:, q] - fd)) <= tol * scale


def test_grad_tasc_is_minus_orbital_fdot():
    """One segment, v = 0, ramp power: dP_lin/dt_asc = -w Tc * (orbital term of eq:derivative)."""
    t = 1.9e6
    seg = S.Segments(t_mid=np.array([t]), v_over_c=np.zeros((1, 3)), weight=np.array([1.7], np.float32),
                     power=(np.arange(60, dtype=np.float32) + 179970)[None, :], k_lo=179970, n_bins=60)
    F, ap, P, ta = 180010.0, 2.2, 19 * S.DAY, 0.4e6
    W = 2 * math.pi / P
    g = O.power_grad(seg, np.array([[0, 0, 1.0]]), [0], np.array([[F, ap, P, ta]]))
    fdot_orb = (F / TC) * ap * W * W * math.sin(W * (t - ta))
    assert g[0, 3] == pytest.approx(-1.7 * TC * fdot_orb, rel=1e-10)


# ---------------------------------------------------------------- peakgram, top-k, significance

def test_peakgram_matches_threshold_strictly_above():
    rng = np.random.default_rng(2)
    pw = rng.exponential(1.0, (37, 134)).astype(np.float32)
    pw[3, 7] = np.float32(1.6)          # float32(1.6) is slightly above the double 1.6
    pw[4, 9] = np.nextafter(np.float32(1.6), np.float32(0))
    bits = O.peakgram(pw)
    unpacked = ((bits[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(37, -1)[:, :134]
    assert np.array_equal(unpacked.astype(bool), pw.astype(np.float64) > 1.6)
    assert unpacked[3, 7] == 1 and unpacked[4, 9] == 0


def test_topk_equals_full_sort_with_index_ties():
    rng = np.random.default_rng(3)
    sc = rng.integers(0, 20, 5000).astype(np.float32)
    vals, idx = O.topk(sc, 300)
    order = sorted(range(5000), key=lambda j: (-sc[j], j))[:300]
    assert np.array_equal(idx, np.array(order))
    assert np.array_equal(vals, sc[order])


def test_significance_reduces_to_binomial_for_unit_weights():
    N, p0 = 1000, O.peak_probability(1.6)
    n = np.array([150.0, 201.0, 260.0])
    s = O.significance_h(n, np.ones(N))
    assert np.allclose(s, (n - N * p0) / math.sqrt(N * p0 * (1 - p0)))
    assert O.significance_p(np.array([1000.0]), np.ones(N))[0] == 0.0


# ---------------------------------------------------------------- template bank

def test_grid_template_counts():
    w1, w2 = S.config1(), S.config2(n_per_det=10)
    a1 = O.grid_tables(w1.grids[0], w1.segments[0].t_span_mid())
    a2 = O.grid_tables(w2.grids[0], w2.segments[0].t_span_mid())
    assert a1[2][-1] * 90 == 46080
    assert a2[2][-1] * 90 == 11796480


def test_grid_tasc_rule_follows_binaryres_spacing():
    """P / delta t_asc from eq:binaryres with m_t = (2 pi^2 / m)^2 / 6 equals the rule's count before clamping."""
    g = S.config5(n_pixels=1, n_per_det=2).grids[0]
    m_t = (2 * math.pi ** 2 / g.tasc_rule_m) ** 2 / 6
    for ap in (0.05, 0.9, 3.25):
        for P in (15 * S.DAY, 31 * S.DAY, 45 * S.DAY):
            W = 2 * math.pi / P
            dt = math.sqrt(6 * m_t) / (math.pi * TC * g.f_hi * ap * W * W)
            n_rule = g.tasc_rule_m * TC * g.f_hi * ap * W
            assert P / dt == pytest.approx(n_rule, rel=1e-12)
            n = O.tasc_points(g, ap, P)
            assert n == min(max(math.ceil(n_rule), 4), 256)


def test_grid_tasc_inside_one_period_around_mid():
    """t_mid - P/2 <= t_asc < t_mid + P/2 (Sec. IV.C, range of t_asc)."""
    g = S.config3(build_items=[]).grids[2]
    t_mid = 1.23e6
    a_p, per, off, ta = O.grid_tables(g, t_mid)
    for cell in range(off.size - 1):
        P = per[cell % g.n_per]
        seg = ta[off[cell]:off[cell + 1]]
        assert seg.min() >= t_mid - P / 2 and seg.max() < t_mid + P / 2
        assert np.all(np.diff(seg) > 0)


# ---------------------------------------------------------------- low-eccentricity track

def test_ecc_track_reduces_to_circular_at_zero_eccentricity():
    seg = _segments(200, 180000, 90, 22, seed=31)
    cand, cs = _cands(seg, 30, 180000, 5)
    x_c, k_c = O.track(seg, S.fixed_pixel(), cs, cand)
    ce = np.concatenate([cand, np.zeros((30, 2))], axis=1)
    x_e, k_e = O.track_ecc(seg, S.fixed_pixel(), cs, ce)
    assert np.array_equal(x_e, x_c) and np.array_equal(k_e, k_c)


def test_ecc_track_max_deviation_is_e_f0_ap_omega():
    """|f_ecc - f_circ| reaches e f0 a_p W over an orbit (eq:frequencyevoerror, its maximum)."""
    F, ap, P, ta, e, om = 270040.0, 2.7, 19 * S.DAY, 0.3e6, 0.004, 1.1
    W = 2 * math.pi / P
    t = ta + np.linspace(0, P, 4001)
    seg = S.Segments(t_mid=t, v_over_c=np.zeros((t.size, 3)), weight=np.ones(t.size, np.float32),
                     power=np.zeros((t.size, 1), np.float32), k_lo=0, n_bins=1)
    sky = np.array([[0, 0, 1.0]])
    x_c, _ = O.track(seg, sky, [0], np.array([[F, ap, P, ta]]))
    x_e, _ = O.track_ecc(seg, sky, [0], np.array([[F, ap, P, ta, e * math.cos(om), e * math.sin(om)]]))
    dev = np.abs(x_e - x_c)[0]
    assert dev.max() == pytest.approx(F * ap * W * e, rel=1e-5)
    # at the eccentricity bound of eq:frequencyevoerror2 the deviation is half a bin
    e_max = 1.0 / (2 * TC * (F / TC) * ap * W)
    x_m, _ = O.track_ecc(seg, sky, [0], np.array([[F, ap, P, ta, e_max, 0.0]]))
    assert np.abs(x_m - x_c).max() == pytest.approx(0.5, rel=1e-5)


def test_ecc_track_is_derivative_of_eccentric_phase_model():
    """v = 0: x / Tc equals (1/2pi) d phi/dt of eq:phaseMethod with its two eccentric terms."""
    f0, ap, P, ta, e, om = 250.03, 1.9, 23 * S.DAY, 0.8e6, 0.008, 2.2
    W = 2 * math.pi / P
    ec, es = e * math.cos(om), e * math.sin(om)
    times = np.linspace(0.2e6, 2.6e6, 29)

    def phase(t):   # cycles
        psi = W * (t - ta)
        return f0 * (t - ap * math.sin(psi) - ap * ec / 2 * math.sin(2 * psi) - ap * es / 2 * math.cos(2 * psi))

    h = 1.0
    f_num = np.array([(phase(t + h) - phase(t - h)) / (2 * h) for t in times])
    seg = S.Segments(t_mid=times, v_over_c=np.zeros((times.size, 3)), weight=np.ones(times.size, np.float32),
                     power=np.zeros((times.size, 1), np.float32), k_lo=0, n_bins=1)
    x, _ = O.track_ecc(seg, np.array([[0, 0, 1.0]]), [0], np.array([[f0 * TC, ap, P, ta, ec, es]]))
    assert np.max(np.abs(x[0] - f_num * TC)) < 2e-4


def test_ecc_power_zero_eccentricity_matches_circular_power():
    seg = _segments(300, 180000, 90, 22, seed=32)
    cand, cs = _cands(seg, 40, 180000, 6)
    ce = np.concatenate([cand, np.zeros((40, 2))], axis=1)
    for mode in (0, 1):
        P_c = O.power_stat(seg, S.fixed_pixel(), cs, cand, mode=mode)[0]
        P_e = O.power_stat_ecc(seg, S.fixed_pixel(), cs, ce, mode=mode)[0]
        assert np.array_equal(P_c, P_e)


# ---------------------------------------------------------------- spectrogram normalization

def test_median_bias_matches_expected_exponential_median():
    """beta(2m+1) is the mean of the sample median of 2m+1 unit exponentials (order statistics)."""
    rng = np.random.default_rng(4)
    for window in (3, 11, 101):
        x = rng.standard_exponential((40000, window))
        assert np.median(x, axis=1).mean() == pytest.approx(O.median_bias(window), rel=4e-3)
    assert O.median_bias(101) == pytest.approx(np.log(2), rel=0.01)


def test_normalize_gives_unit_exponential_noise():
    """Exp(1) noise on any smooth floor normalizes to mean 1 with P(rho > 1.6) = e^-1.6 (Sec. IV.A)."""
    raw = S.raw_sft_powers(np.random.default_rng(5), 400, 134 + 100, 180000 - 72)
    rho = O.normalize(raw)
    assert rho.shape == (400, 134)
    assert abs(float(rho.mean()) - 1.0) < 0.01
    assert abs(float((rho > 1.6).mean()) - np.exp(-1.6)) < 0.005
    # a pure scale per segment cancels exactly up to float rounding
    rho2 = O.normalize(raw * np.float32(4.0))
    assert np.array_equal(rho2, rho)


def test_normalize_is_median_of_window_brute_force():
    raw = np.random.default_rng(6).exponential(1.0, (3, 30)).astype(np.float32)
    rho = O.normalize(raw, window=11)
    beta = O.median_bias(11)
    for J in range(3):
        for c in range(20):
            med = sorted(raw[J, c:c + 11].tolist())[5]
            assert rho[J, c] == np.float32((float(raw[J, c + 5]) * beta) / med)


def test_stage2_on_doubled_set_is_sum_over_both_sets():
    """Stage 2 over the segments plus their Tc/2-shifted companions (Sec. IV.C, second step) is
    the sum of the two sets' statistics, in both modes; counts and near-ties add exactly."""
    w = S.config2(n_per_det=5)
    r = np.random.default_rng(3)
    t0, det = S.two_detector_starts(r, (80, 80), 100)
    a = S._segments(t0, det, S.lognormal_weights(r, t0.size), r, w.segments[0].k_lo, w.segments[0].n_bins)
    b = S.half_shifted(a, r)
    u = S.concat_segments(a, b)
    assert b.n_seg > 80
    for d in (0, 1):          # every companion starts Tc/2 after a segment of its detector
        assert np.all(np.isin(b.t_mid[b.detector == d] - 450.0, a.t_mid[a.detector == d]))
    rng = np.random.default_rng(8)
    cand = np.stack([180000 + rng.uniform(0, 89, 300), rng.uniform(0.01, 3, 300),
                     rng.uniform(15, 45, 300) * S.DAY, rng.uniform(0, 3e6, 300)], axis=1)
    cs = np.zeros(300, np.int32)
    for mode in (0, 1):
        pu, cu, nwu, ntu = O.power_stat(u, w.sky, cs, cand, mode=mode)
        pa, ca, nwa, nta = O.power_stat(a, w.sky, cs, cand, mode=mode)
        pb, cb, nwb, ntb = O.power_stat(b, w.sky, cs, cand, mode=mode)
        assert np.allclose(pu, pa + pb, rtol=1e-12, atol=0)
        if mode == 0:
            assert np.array_equal(cu, ca + cb) and np.array_equal(ntu, nta + ntb)
            assert np.allclose(nwu, nwa + nwb, rtol=1e-12, atol=0)


# ---------------------------------------------------------------- significance normalizations

def _noise_draws(n_seg, n_draws, sigma_w, seed):
    """n_draws independent noise realizations of one candidate over n_seg segments: a segment set
    with no detector motion whose rows hold n_draws unit-exponential columns, read by candidates
    with a_p = 0 at F = each column's absolute bin (so x = F exactly and each candidate reads its
    own column).  Weights are log-normal(0, sigma_w) normalized to mean 1."""
    rng = np.random.default_rng(seed)
    k_lo = 50000
    t = np.sort(rng.uniform(0, 60 * S.DAY, n_seg)) + 0.5 * TC
    w = np.exp(sigma_w * rng.standard_normal(n_seg))
    w = (w / w.mean()).astype(np.float32)
    seg = S.Segments(t_mid=t, v_over_c=np.zeros((n_seg, 3)), weight=w,
                     power=rng.standard_exponential((n_seg, n_draws), dtype=np.float32),
                     k_lo=k_lo, n_bins=n_draws)
    cand = np.stack([k_lo + np.arange(n_draws, dtype=np.float64), np.zeros(n_draws),
                     np.full(n_draws, 20 * S.DAY), np.zeros(n_draws)], axis=1)
    P, cnt, nw, nt = O.power_stat(seg, np.array([[0.0, 0.0, 1.0]]), np.zeros(n_draws, np.int32), cand, mode=0)
    assert nt.sum() == 0
    return seg, P, nw


@pytest.mark.parametrize("sigma_w", [0.3, 1.0])
def test_significances_have_unit_normal_moments_under_noise(sigma_w):
    """Under the noise law p(rho) = exp(-rho) (Sec. IV.F) the peaks are Bernoulli(e^-rho_th) and the
    powers Exp(1), so s_H (eq:hough2) and s_P (eq:hough3) have mean 0 and variance 1 whatever the
    weights.  Log-normal weights make sum w and sum w^2 differ (by e^{sigma^2}: 9 % at sigma 0.3,
    a factor 2.7 at sigma 1), so a normalization that mixes them up moves the variance (or the
    mean) far outside the sampling error of 2 x 10^4 draws."""
    n_draws = 20000
    seg, P, nw = _noise_draws(200, n_draws, sigma_w, seed=int(sigma_w * 10) + 3)
    sh = O.significance_h(nw, seg.weight)
    sp = O.significance_p(P, seg.weight)
    # standard errors: mean 1/sqrt(n); variance about sqrt(2/n) (times a kurtosis factor < 1.5)
    se_m = 1.0 / math.sqrt(n_draws)
    se_v = 1.5 * math.sqrt(2.0 / n_draws)
    for s in (sh, sp):
        assert abs(s.mean()) < 5 * se_m, s.mean()
        assert abs(s.var() - 1.0) < 5 * se_v, s.var()
    # the ratio the pin separates, sum w^2 / sum w, is far from 1 at both widths
    w = seg.weight.astype(np.float64)
    assert (w * w).sum() / w.sum() > (2.0 if sigma_w > 0.5 else 1.05)


# ---------------------------------------------------------------- ELL1 stage-2 power at e != 0

def test_ecc_power_ramp_follows_ecc_track():
    """rho_{J,c} = c + k_lo (the absolute bin), e != 0: P_lin = sum w x and P = sum w k with the ELL1
    track's own x and k, for eccentricities up to 0.05 and both orientations of (e cos w, e sin w)."""
    seg = _segments(300, 180000, 90, 22, seed=33)
    seg.power[:] = (np.arange(seg.n_bins, dtype=np.float64) + seg.k_lo)[None, :].astype(np.float32)
    cand, cs = _cands(seg, 30, 180000, 7)
    rng = np.random.default_rng(8)
    e = rng.uniform(0.001, 0.05, 30)
    om = rng.uniform(0, 2 * math.pi, 30)
    ce = np.concatenate([cand, np.stack([e * np.cos(om), e * np.sin(om)], axis=1)], axis=1)
    x, k = O.track_ecc(seg, S.fixed_pixel(), cs, ce)
    w = seg.weight.astype(np.float64)
    P_lin = O.power_stat_ecc(seg, S.fixed_pixel(), cs, ce, mode=1)[0]
    P_near = O.power_stat_ecc(seg, S.fixed_pixel(), cs, ce, mode=0)[0]
    assert np.allclose(P_lin, x @ w, rtol=1e-13)
    assert np.allclose(P_near, k.astype(np.float64) @ w, rtol=1e-13)


def test_ecc_power_one_segment_equals_phase_model_frequency():
    """No detector motion, one segment, ramp powers: P_lin / w is the ELL1 frequency (times Tc) at the
    segment's time, which must equal the central difference of the eccentric phase model of
    eq:phaseMethod (its two e terms) within 2e-4 bins.  Swapping e cos w and e sin w, or the sign of
    either term, moves it by up to e F a_p W, about 0.07 bins here."""
    f0, ap, P = 250.03, 2.6, 16 * S.DAY
    W = 2 * math.pi / P
    F = f0 * TC
    t0 = 1.3e6
    tas = np.linspace(t0 - P / 2, t0 + P / 2, 41)[:-1]
    e, om = 0.05, 0.9
    ec, es = e * math.cos(om), e * math.sin(om)
    k_lo, n_bins = int(F) - 400, 800
    seg = S.Segments(t_mid=np.array([t0]), v_over_c=np.zeros((1, 3)), weight=np.array([0.75], np.float32),
                     power=(np.arange(n_bins, dtype=np.float64) + k_lo)[None, :].astype(np.float32),
                     k_lo=k_lo, n_bins=n_bins)
    ce = np.stack([np.full(tas.size, F), np.full(tas.size, ap), np.full(tas.size, P), tas,
                   np.full(tas.size, ec), np.full(tas.size, es)], axis=1)
    P_lin = O.power_stat_ecc(seg, np.array([[0, 0, 1.0]]), np.zeros(tas.size, np.int32), ce, mode=1)[0]

    def phase(t, ta):   # cycles
        psi = W * (t - ta)
        return f0 * (t - ap * math.sin(psi) - ap * ec / 2 * math.sin(2 * psi) - ap * es / 2 * math.cos(2 * psi))

    h = 1.0
    x_num = np.array([(phase(t0 + h, ta) - phase(t0 - h, ta)) / (2 * h) * TC for ta in tas])
    assert np.max(np.abs(P_lin / 0.75 - x_num)) < 2e-4
    # the e terms really matter at this size
    x_circ = np.array([F * (1 - ap * W * math.cos(W * (t0 - ta))) for ta in tas])
    assert np.max(np.abs(x_num - x_circ)) > 0.05


# ---------------------------------------------------------------- ELL1 stage-1 count and adjoint

def _ecc_rows(cand, seed, e_max=0.05):
    rng = np.random.default_rng(seed)
    e = rng.uniform(0.001, e_max, cand.shape[0])
    om = rng.uniform(0, 2 * math.pi, cand.shape[0])
    return np.concatenate([cand, np.stack([e * np.cos(om), e * np.sin(om)], axis=1)], axis=1)


def test_ecc_count_reduces_to_circular_at_zero_eccentricity():
    """(e cos w, e sin w) = (0, 0): every output of the ELL1 count equals the circular count, bit for bit."""
    seg = _segments(150, 90000, 90, 12, seed=41)
    sky = S.fibonacci_sphere(2)
    a_p, per, off, ta = _grid_from([0.3, 2.1], [17 * S.DAY, 33 * S.DAY],
                                   [[1e5, 8e5], [2e5, 1.5e6, 2.4e6], [3e5], [5e5, 9e5]])
    r_c = O.hough_count(seg, sky, 90000, 90, a_p, per, off, ta)
    r_e = O.hough_count_ecc(seg, sky, 90000, 90, a_p, per, off, ta, 0.0, 0.0)
    for a, b in zip(r_c, r_e):
        assert np.array_equal(a, b)


def test_ecc_count_brute_force_tiny_grid():
    """ELL1 counts on a 4-segment, 3-f0, 2 x 2 x (1..2) grid with e = 0.03 against a 50-digit
    evaluation of the eccentric track (eq:frequencyevo, product form)."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    seg = _segments(4, 1000, 3, 4, seed=42)
    seg.power[:] = np.random.default_rng(10).exponential(1.0, seg.power.shape).astype(np.float32)
    sky = S.fibonacci_sphere(2)
    a_p, per, off, ta = _grid_from([0.9, 3.1], [15 * S.DAY, 27 * S.DAY],
                                   [[1.5e5, 9.5e5], [2.5e5], [3.5e5, 4.5e5], [6.0e5, 2.0e6]])
    ec, es = 0.03 * math.cos(2.0), 0.03 * math.sin(2.0)
    cnt, nw, nt, _ = O.hough_count_ecc(seg, sky, 1000, 3, a_p, per, off, ta, ec, es)
    assert nt.sum() == 0
    ecm, esm = mp.mpf(ec), mp.mpf(es)
    idx = 0
    for s in range(2):
        for b in range(off[-1]):
            cell = np.searchsorted(off, b, side="right") - 1
            ap, P = a_p[cell // 2], per[cell % 2]
            for i in range(3):
                c_exp, w_exp = 0, 0.0
                for J in range(4):
                    W = 2 * mp.pi / mp.mpf(float(P))
                    d = sum(mp.mpf(float(u)) * mp.mpf(float(q)) for u, q in zip(seg.v_over_c[J], sky[s]))
                    psi = W * (mp.mpf(float(seg.t_mid[J])) - mp.mpf(float(ta[b])))
                    E = mp.cos(psi) + ecm * mp.cos(2 * psi) - esm * mp.sin(2 * psi)
                    xe = (1000 + i) * (1 + d) * (1 - mp.mpf(float(ap)) * W * E)
                    col = int(mp.floor(xe + mp.mpf("0.5"))) - seg.k_lo
                    if seg.power[J, col] > 1.6:
                        c_exp += 1
                        w_exp += float(seg.weight[J])
                assert cnt[idx] == c_exp
                assert nw[idx] == pytest.approx(w_exp, rel=1e-12)
                idx += 1


def test_ecc_count_noiseless_injection():
    """rho = 0 except 2 on one template's ELL1 track: that template counts every segment with the
    full weight and is the map's maximum; the circular track of the same template misses peaks."""
    seg = _segments(300, 180000, 90, 22, seed=43)
    seg.power[:] = 0
    g = S.GridSpec(k0=180000, n_f0=90, ap_lo=1.5, ap_hi=3.0, n_ap=3, per_lo=15 * S.DAY,
                   per_hi=20 * S.DAY, n_per=2, tasc_fixed=5)
    a_p, per, off, ta = O.grid_tables(g, seg.t_span_mid())
    ec, es = 0.04, -0.02
    b_true, i_true = 23, 7
    cell = np.searchsorted(off, b_true, side="right") - 1
    row = np.array([[180000 + i_true, a_p[cell // 2], per[cell % 2], ta[b_true], ec, es]])
    _, k = O.track_ecc(seg, S.fixed_pixel(), [0], row)
    seg.power[np.arange(seg.n_seg), k[0] - seg.k_lo] = 2.0
    cnt, nw, _, _ = O.hough_count_ecc(seg, S.fixed_pixel(), 180000, 90, a_p, per, off, ta, ec, es)
    idx = b_true * 90 + i_true
    assert cnt[idx] == seg.n_seg
    assert nw[idx] == pytest.approx(float(seg.weight.astype(np.float64).sum()), rel=1e-12)
    assert cnt.argmax() == idx
    cnt_c, _, _, _ = O.hough_count(seg, S.fixed_pixel(), 180000, 90, a_p, per, off, ta)
    assert cnt_c[idx] < seg.n_seg


def test_ecc_grad_zero_eccentricity_matches_circular():
    seg = _segments(300, 180000, 90, 22, seed=44)
    cand, cs = _cands(seg, 12, 180000, 9)
    ce = np.concatenate([cand, np.zeros((12, 2))], axis=1)
    g_c = O.power_grad(seg, S.fixed_pixel(), cs, cand)
    g_e = O.power_grad_ecc(seg, S.fixed_pixel(), cs, ce)
    assert np.allclose(g_e[:, :4], g_c, rtol=1e-12, atol=1e-12 * np.abs(g_c).max())
    assert np.all(np.abs(g_e[:, 4:]) > 0)


def test_ecc_grad_ramp_closed_form():
    """Ramp power makes P_lin = sum w x on the ELL1 track, so its gradient in all six parameters
    is the central difference of sum w x taken from the track itself (no kinks)."""
    seg = _segments(400, 180000, 90, 22, seed=45)
    seg.power[:] = (np.arange(seg.n_bins, dtype=np.float64) + seg.k_lo)[None, :].astype(np.float32)
    cand, cs = _cands(seg, 6, 180000, 10)
    cand[:, 1] = np.maximum(cand[:, 1], 0.5)
    ce = _ecc_rows(cand, 11)
    g = O.power_grad_ecc(seg, S.fixed_pixel(), cs, ce)
    w = seg.weight.astype(np.float64)
    hs = np.array([1e-2, 5e-3, 0.5e-3 * S.DAY, 300.0, 1e-4, 1e-4])
    for q in range(6):
        cp, cm = ce.copy(), ce.copy()
        cp[:, q] += hs[q]
        cm[:, q] -= hs[q]
        xp, _ = O.track_ecc(seg, S.fixed_pixel(), cs, cp)
        xm, _ = O.track_ecc(seg, S.fixed_pixel(), cs, cm)
        fd = ((xp - xm) @ w) / (2 * hs[q])
        assert np.allclose(g[:, q], fd, rtol=2e-6, atol=1e-9 * np.abs(fd).max()), q


def test_ecc_grad_frozen_bin_fd():
    """Noise powers: with the bins k'_J frozen at theta, the central difference of P_lin on the
    ELL1 track matches the analytic gradient in all six parameters."""
    seg = _segments(400, 180000, 90, 22, seed=46)
    cand, cs = _cands(seg, 5, 180000, 12)
    ce = _ecc_rows(cand, 13)
    g = O.power_grad_ecc(seg, S.fixed_pixel(), cs, ce)
    w = seg.weight.astype(np.float64)
    x0, _ = O.track_ecc(seg, S.fixed_pixel(), cs, ce)
    kf = np.floor(x0)
    rows = np.arange(seg.n_seg)

    def plin_frozen(c):
        x, _ = O.track_ecc(seg, S.fixed_pixel(), cs, c)
        a = x - kf
        col = (kf - seg.k_lo).astype(np.int64)
        r0 = seg.power[rows[None, :], col].astype(np.float64)
        r1 = seg.power[rows[None, :], col + 1].astype(np.float64)
        return ((1 - a) * r0 + a * r1) @ w

    hs = np.array([1e-2, 5e-3, 0.5e-3 * S.DAY, 300.0, 1e-4, 1e-4])
    for q in range(6):
        cp, cm = ce.copy(), ce.copy()
        cp[:, q] += hs[q]
        cm[:, q] -= hs[q]
        fd = (plin_frozen(cp) - plin_frozen(cm)) / (2 * hs[q])
        scale = np.abs(fd).max() + 1e-30
        assert np.max(np.abs(g[:, q] - fd)) <= 1e-6 * scale, q


def test_ecc_grad_tasc_is_minus_eccentric_fdot():
    """One segment, v = 0, ramp power: dP_lin/dt_asc = -w Tc d^2 phi/dt^2 of the orbital part of the
    eccentric phase model (eq:phaseMethod with its two e terms), since the track depends on t and
    t_asc only through t - t_asc.  The second derivative is taken numerically from the phase."""
    t = 1.7e6
    F, ap, P, ta = 180010.0, 2.4, 17 * S.DAY, 0.55e6
    f0 = F / TC
    e, om = 0.04, 2.5
    ec, es = e * math.cos(om), e * math.sin(om)
    W = 2 * math.pi / P
    seg = S.Segments(t_mid=np.array([t]), v_over_c=np.zeros((1, 3)), weight=np.array([1.3], np.float32),
                     power=(np.arange(80, dtype=np.float32) + 179970)[None, :], k_lo=179970, n_bins=80)
    g = O.power_grad_ecc(seg, np.array([[0, 0, 1.0]]), [0], np.array([[F, ap, P, ta, ec, es]]))

    def orbital_phase(tt):   # cycles, without the f0 t term
        psi = W * (tt - ta)
        return -f0 * ap * (math.sin(psi) + ec / 2 * math.sin(2 * psi) + es / 2 * math.cos(2 * psi))

    h = 500.0
    fdot = (orbital_phase(t + h) - 2 * orbital_phase(t) + orbital_phase(t - h)) / (h * h)
    assert g[0, 3] == pytest.approx(-1.3 * TC * fdot, rel=1e-6)
