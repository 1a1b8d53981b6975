"""Pins of the oracle's post-processing (Sec. V.E, eq:postdist) against what the paper fixes.

The resolutions are pinned through the oracle's frequency track (itself pinned elsewhere): moving
one parameter by its resolution moves the track by the number of bins the resolution formulas
promise (exactly, via trig identities, or within a stated first-order bound).  The clustering is
pinned to single-linkage clustering from SciPy, the coincidences and centroids to cases whose
result follows by hand.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle as O
from oracle import post as PP

TC = 900.0
DAY = 86400.0


def _track_x(t, v, f, a_p, period, t_asc, n=(1.0, 0.0, 0.0)):
    seg = SimpleNamespace(t_mid=np.asarray(t, np.float64), v_over_c=np.asarray(v, np.float64))
    cand = np.array([[f * TC, a_p, period, t_asc]])
    x, _ = O.track(seg, np.array([n], np.float64), np.zeros(1, np.int32), cand)
    return x[0]


def _row(f, a_p, period, t_asc, x=0.0, y=0.0):
    return np.array([f, x, y, a_p, 2 * np.pi / period, t_asc])


def test_frequency_term_counts_bins():
    pp = PP.PostParams()
    a = _row(200.0, 1.0, 20 * DAY, 1e6)
    for nb in (1, 3, 7):
        b = a.copy()
        b[0] += nb / TC
        assert abs(PP.distance2(pp, a, b) - nb * nb) < 1e-9


def test_ap_resolution_moves_track_by_promised_bins():
    """Delta a_p = da_p changes x by F W da_p |cos| <= sqrt(6 m_a)/pi bins, reached at cos = +-1."""
    pp = PP.PostParams(m_a=0.4)
    f, a, per = 200.0, 1.5, 17 * DAY
    row = _row(f, a, per, 3e6)
    da = PP.resolutions(pp, row)[0, 1]
    t = np.linspace(0.0, 2 * per, 400001)
    v = np.zeros((t.size, 3))
    dx = _track_x(t, v, f, a + da, per, 3e6) - _track_x(t, v, f, a, per, 3e6)
    want = np.sqrt(6 * 0.4) / np.pi
    assert abs(np.abs(dx).max() / want - 1) < 1e-6


def test_tasc_resolution_moves_track_by_promised_bins():
    """A t_asc shift dt changes x by F a W (cos u - cos(u - W dt)), amplitude 2 F a W sin(W dt/2);
    the resolution sets F a W^2 dt = sqrt(6 m_t)/pi."""
    pp = PP.PostParams(m_t=0.4)
    f, a, per, ta = 300.0, 2.0, 25 * DAY, 5e6
    row = _row(f, a, per, ta)
    dt = PP.resolutions(pp, row)[0, 3]
    W = 2 * np.pi / per
    t = np.linspace(0.0, 2 * per, 400001)
    v = np.zeros((t.size, 3))
    dx = _track_x(t, v, f, a, per, ta + dt) - _track_x(t, v, f, a, per, ta)
    want = np.sqrt(6 * 0.4) / np.pi * (2 * np.sin(W * dt / 2) / (W * dt))
    assert abs(np.abs(dx).max() / want - 1) < 1e-6


def test_omega_resolution_moves_track_by_promised_bins():
    """A period change dW moves x by F a dW (cos u - u sin u), u = W tau, to first order.  With
    T_obs chosen so that u reaches 8.5 pi at the ends (where sin u = +-1), the maximum over
    |tau| <= T_obs/2 is F a W (T_obs/2) dW = sqrt(72 m)/(2 pi) up to 1/(2 u^2)."""
    m = 1e-4
    f, a, per = 200.0, 1.0, 15 * DAY
    t_obs = 8.5 * per
    pp = PP.PostParams(m_omega=m, t_obs=t_obs)
    ta = 70 * DAY
    row = _row(f, a, per, ta)
    dW = PP.resolutions(pp, row)[0, 2]
    W = 2 * np.pi / per
    per2 = 2 * np.pi / (W + dW)
    t = np.linspace(ta - t_obs / 2, ta + t_obs / 2, 800001)
    v = np.zeros((t.size, 3))
    dx = _track_x(t, v, f, a, per2, ta) - _track_x(t, v, f, a, per, ta)
    want = np.sqrt(72 * m) / (2 * np.pi)
    assert abs(np.abs(dx).max() / want - 1) < 2e-3


def test_sky_resolution_moves_track_by_one_over_pixel_factor():
    """Rotating n in the orbital plane by dTheta changes v.n by |v| 2 sin(dTheta/2) at most, so x
    moves by (1/P_F) (2 sin(dTheta/2)/dTheta) bins with |v| = v/c of the resolution."""
    for pf in (1.0, 2.0):
        pp = PP.PostParams(pixel_factor=pf, v_over_c=1e-4)
        f = 250.0
        row = _row(f, 1.0, 20 * DAY, 0.0)
        dth = PP.resolutions(pp, row)[0, 0]
        t = np.linspace(0.0, 365.25 * DAY, 400001)
        ph = 2 * np.pi * t / (365.25 * DAY)
        v = 1e-4 * np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], axis=1)
        phi = 0.7
        n1 = (np.cos(phi), np.sin(phi), 0.0)
        n2 = (np.cos(phi + dth), np.sin(phi + dth), 0.0)
        dx = _track_x(t, v, f, 0.0, 20 * DAY, 0.0, n2) - _track_x(t, v, f, 0.0, 20 * DAY, 0.0, n1)
        want = (1.0 / pf) * (2 * np.sin(dth / 2) / dth)
        assert abs(np.abs(dx).max() / want - 1) < 1e-6


def test_terms_add_in_quadrature_and_distance_is_symmetric():
    pp = PP.PostParams()
    rng = np.random.default_rng(5)
    a = _row(200.0, 1.2, 20 * DAY, 2e6, 0.3, -0.4)
    res = PP.resolutions(pp, a)[0]
    # moves in x, y and t_asc leave every resolution as it is (they depend on f, a_p and
    # Omega only), so their squared terms add
    b_y = a.copy(); b_y[2] -= 2.0 * res[0]
    b_x = a.copy(); b_x[1] += 1.5 * res[0]
    b_t = a.copy(); b_t[5] += 0.5 * res[3]
    both = a.copy(); both[2] -= 2.0 * res[0]; both[1] += 1.5 * res[0]; both[5] += 0.5 * res[3]
    s = PP.distance2(pp, a, b_y) + PP.distance2(pp, a, b_x) + PP.distance2(pp, a, b_t)
    assert abs(s - 6.5) < 1e-9
    assert abs(PP.distance2(pp, a, both) - s) < 1e-9 * s
    assert abs(PP.distance2(pp, a, b_x) - 2.25) < 1e-9
    assert abs(PP.distance2(pp, a, b_t) - 0.25) < 1e-9
    c = np.stack([_row(200 + rng.uniform(0, .1), rng.uniform(.5, 3), rng.uniform(15, 45) * DAY,
                       rng.uniform(0, 1e7), *rng.uniform(-1, 1, 2)) for _ in range(30)])
    D = PP.distance_matrix2(pp, c, c)
    assert np.array_equal(D, D.T) and np.all(np.diag(D) == 0)


def test_mean_resolution_between_points():
    """Two templates differing in a_p only: da_p does not depend on a_p, so d = |Delta a_p|/da_p;
    differing in a_p and t_asc, the t_asc term uses the mean of dt at both a_p values."""
    pp = PP.PostParams()
    a = _row(200.0, 1.0, 20 * DAY, 2e6)
    r = PP.resolutions(pp, a)[0]
    b = a.copy(); b[3] += 2.5 * r[1]
    assert abs(PP.distance2(pp, a, b) - 6.25) < 1e-9
    # dt_asc ~ 1/a_p: at a_p and 3 a_p the mean is (dt + dt/3)/2 = 2 dt/3
    b = a.copy(); b[3] = 3.0; b[5] += r[3]
    qa = (3.0 - 1.0) / r[1]
    assert abs(PP.distance2(pp, a, b) - (qa * qa + 1.5 ** 2)) < 1e-9 * qa * qa


def _cloud(rng, n, pp):
    """Candidates scattered over a few resolution cells so that links and gaps both occur."""
    base = _row(200.05, 1.5, 20 * DAY, 3e6, 0.2, 0.1)
    r = PP.resolutions(pp, base)[0]
    centers = rng.uniform(-12, 12, (6, 6))
    pick = rng.integers(0, 6, n)
    steps = centers[pick] + rng.normal(0, 1.2, (n, 6))
    c = np.repeat(base[None, :], n, axis=0)
    c[:, 0] += steps[:, 0] / TC
    c[:, 1] += steps[:, 1] * r[0]
    c[:, 2] += steps[:, 2] * r[0]
    c[:, 3] += steps[:, 3] * r[1] * 0.05
    c[:, 4] += steps[:, 4] * r[2] * 0.05
    c[:, 5] += steps[:, 5] * r[3] * 0.05
    return c


def test_clusters_equal_single_linkage():
    from scipy.cluster.hierarchy import fcluster, linkage
    from scipy.spatial.distance import squareform
    pp = PP.PostParams()
    rng = np.random.default_rng(11)
    for n in (2, 17, 150):
        c = _cloud(rng, n, pp)
        w = np.sqrt(14.0)
        lab = PP.clusters(pp, c, w)
        D = np.sqrt(PP.distance_matrix2(pp, c, c))
        assert np.min(np.abs(D - w)) > 1e-9          # no pair sits on the window
        z = linkage(squareform(D, checks=False), method="single")
        ref = fcluster(z, t=w, criterion="distance")
        # same partition; labels are the smallest member index
        for i in range(n):
            same = np.nonzero(ref == ref[i])[0]
            assert lab[i] == same.min()
            assert np.array_equal(np.nonzero(lab == lab[i])[0], same)


def test_clusters_chain_and_gap():
    """Templates 3.5 bins apart in f chain into one cluster over 31.5 bins; 3.8 bins splits."""
    pp = PP.PostParams()
    a = _row(200.0, 1.0, 20 * DAY, 2e6)
    for step, n_clusters in ((3.5, 1), (3.8, 10)):
        c = np.repeat(a[None, :], 10, axis=0)
        c[:, 0] += np.arange(10) * step / TC
        lab = PP.clusters(pp, c[::-1], np.sqrt(14.0))
        assert len(np.unique(lab)) == n_clusters


def test_coincidences_of_shifted_lists():
    """List b = list a moved by 2 f bins: every i pairs with its own copy at d = 2, and with
    equal significances the centroid is the midpoint; entries far apart do not pair."""
    pp = PP.PostParams()
    a = np.stack([_row(200.0 + 40 * i / TC, 1.0, 20 * DAY, 2e6) for i in range(5)])
    b = a.copy(); b[:, 0] += 2 / TC
    s = np.arange(1, 6, dtype=np.float64)
    pairs, cen, sig = PP.coincidences(pp, a, s, b, s, 3.0)
    assert np.array_equal(pairs, np.stack([np.arange(5), np.arange(5)], axis=1))
    assert np.allclose(cen, 0.5 * (a + b), rtol=1e-15, atol=0)
    assert np.array_equal(sig, 2 * s)
    pairs, _, _ = PP.coincidences(pp, a, s, b, s, 1.9)
    assert pairs.shape[0] == 0
    # unequal significances pull the centroid towards the stronger member
    pairs, cen, _ = PP.coincidences(pp, a[:1], [3.0], b[:1], [1.0], 3.0)
    assert abs((cen[0, 0] - a[0, 0]) * TC - 0.5) < 1e-9


def test_centroids_weights_cut_and_best_cluster():
    pp = PP.PostParams()
    a = _row(200.0, 1.0, 20 * DAY, 2e6)
    c = np.repeat(a[None, :], 6, axis=0)
    c[:, 0] += np.array([0, 1, 2, 30, 31, 33]) / TC       # clusters {0,1,2} and {3,4,5}
    s = np.array([1.0, 4.0, 1.0, 2.0, 2.0, 2.5])
    lab = PP.clusters(pp, c, np.sqrt(14.0))
    assert list(lab) == [0, 0, 0, 3, 3, 3]
    out, best = PP.centroids(pp, c, s, lab)
    top, keep, wsum, cen = out[0]
    assert top == 1 and wsum == 6.0
    assert abs((cen[0] - a[0]) * TC - 1.0) < 1e-9                     # symmetric about member 1
    assert best == 3 and out[3][2] == 6.5
    # scaling every significance leaves centroids alone
    out2, _ = PP.centroids(pp, c, 7 * s, lab)
    assert np.allclose(out2[3][3], out[3][3], rtol=1e-15, atol=0)
    # the option-B cut drops members farther than the cut from the top member (member 5 is
    # 2 bins from member 4... the top of {3,4,5} is 5: members 3 (3 bins) and 4 (2 bins))
    out3, best3 = PP.centroids(pp, c, s, lab, cut=2.5)
    assert list(out3[3][1]) == [4, 5] and out3[3][2] == 4.5
    assert best3 == 0
