"""GPU post-processing (Sec. V.E) against the oracle: rows, significances, coincidences,
clusters and centroids, called through the C ABI.

Clusters and coincidence pairs are integer results and must match exactly: both sides decide
"d < window" in FP64 under the same operation order, and the inputs keep every pair at least
1e-9 (relative) away from the window.  Centroids and summed significances are FP64 sums whose
order differs (device atomics), compared to 1e-12 relative.
"""
import sys

import numpy as np
import pytest

import bsh_synth as S
import oracle as O
from oracle import post as PP

pytestmark = pytest.mark.gpu

TC = 900.0
DAY = 86400.0


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _cloud(rng, n, pp, n_centers=6, spread=1.2, f0=200.05):
    """Candidate rows scattered around a few centres, in units of the resolutions."""
    base = np.array([f0, 0.2, 0.1, 1.5, 2 * np.pi / (20 * DAY), 3e6])
    r = PP.resolutions(pp, base)[0]
    centers = rng.uniform(-12, 12, (n_centers, 6)) * np.array([1, 1, 1, 1, 1, 1]) * (n_centers / 6) ** 0.5
    pick = rng.integers(0, n_centers, n)
    steps = centers[pick] + rng.normal(0, spread, (n, 6))
    c = np.repeat(base[None, :], n, axis=0)
    c[:, 0] += steps[:, 0] / TC
    c[:, 1] += steps[:, 1] * r[0]
    c[:, 2] += steps[:, 2] * r[0]
    c[:, 3] += steps[:, 3] * r[1] * 0.05
    c[:, 4] += steps[:, 4] * r[2] * 0.05
    c[:, 5] += steps[:, 5] * r[3] * 0.05
    return c


def _margin_ok(pp, c, w):
    d2 = PP.distance_matrix2(pp, c, c)
    return np.min(np.abs(d2 - w * w)) > 1e-9 * w * w


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1904_04873_amd import bsh
    return torch, bsh


def _pp_ctypes(bsh, pp):
    return bsh.post_params(t_coh=pp.t_coh, t_obs=pp.t_obs, m_a=pp.m_a, m_omega=pp.m_omega, m_t=pp.m_t,
                           pixel_factor=pp.pixel_factor, v_over_c=pp.v_over_c)


def test_post_rows_exact(env):
    torch, bsh = env
    _say("post rows")
    rng = np.random.default_rng(1)
    sky = S.fibonacci_sphere(16)
    n = 1000
    cs = rng.integers(0, 16, n).astype(np.int32)
    cand = np.stack([rng.integers(90000, 90090, n).astype(np.float64) + rng.uniform(-.5, .5, n),
                     rng.uniform(0.01, 3, n), rng.uniform(15, 45, n) * DAY, rng.uniform(0, 1e7, n)], axis=1)
    rows = bsh.bsh_post_rows(torch.tensor(sky, device="cuda"), torch.tensor(cs, device="cuda"),
                             torch.tensor(cand, device="cuda"), TC).cpu().numpy()
    want = np.stack([cand[:, 0] / TC, sky[cs, 0], sky[cs, 1], cand[:, 1], O.TWO_PI / cand[:, 2], cand[:, 3]],
                    axis=1)
    assert np.array_equal(rows, want)


@pytest.mark.parametrize("kind", [0, 1])
def test_significance_matches_oracle(env, kind):
    torch, bsh = env
    _say(f"significance kind {kind}")
    rng = np.random.default_rng(2)
    w = S.lognormal_weights(rng, 4000)
    score = rng.uniform(800, 1600, 3001).astype(np.float32)
    got = bsh.bsh_significance(torch.tensor(score, device="cuda"), torch.tensor(w, device="cuda"), kind,
                               1.6).cpu().numpy()
    want = O.significance_h(score, w, 1.6) if kind == 0 else O.significance_p(score, w)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 17, 255, 256, 257, 3001])
def test_clusters_match_oracle(env, n):
    torch, bsh = env
    _say(f"clusters n={n}")
    pp = PP.PostParams()
    rng = np.random.default_rng(100 + n)
    c = _cloud(rng, n, pp, n_centers=max(2, n // 40))
    w = np.sqrt(14.0)
    assert _margin_ok(pp, c, w)
    got = bsh.bsh_cluster(_pp_ctypes(bsh, pp), torch.tensor(c, device="cuda"), w).cpu().numpy()
    want = PP.clusters(pp, c, w)
    assert np.array_equal(got.astype(np.int64), want)


def test_clusters_on_grid_frequencies_with_ties(env):
    """Stage-1 lists carry on-grid frequencies (bin centres), so many rows share f exactly across
    row and column tiles: 3000 rows on 12 frequency bins (ties in the frequency-window search's key
    and in its tie-break by position), plus rows whose only difference from a partner is |Delta f|
    just inside or just outside the window's frequency half-width window / Tc (2e-7 relative)."""
    torch, bsh = env
    _say("clusters on-grid f")
    pp = PP.PostParams()
    rng = np.random.default_rng(31)
    n = 3000
    base = np.array([200.0, 0.2, 0.1, 1.5, 2 * np.pi / (20 * DAY), 3e6])
    r = PP.resolutions(pp, base)[0]
    c = np.repeat(base[None, :], n, axis=0)
    c[:, 0] = 200.0 + rng.integers(0, 12, n) / TC
    c[:, 1] += rng.normal(0, 4, n) * r[0]
    c[:, 2] += rng.normal(0, 4, n) * r[0]
    c[:, 3] += rng.normal(0, 4, n) * r[1]
    c[:, 4] += rng.normal(0, 4, n) * r[2]
    c[:, 5] += rng.normal(0, 4, n) * r[3]
    w = np.sqrt(14.0)
    far = base.copy()
    far[3] += 1000 * r[1]                       # away from the cloud in a_p
    pairs = []
    for q, rel in enumerate((1 - 2e-7, 1 + 2e-7, 1 - 2e-7, 1 + 2e-7)):
        a = far.copy()
        a[5] += 1000 * q * r[3]                 # each pair on its own, apart in t_asc
        b = a.copy()
        b[0] += w / TC * rel
        pairs += [a, b]
    c = np.concatenate([c, np.array(pairs)])
    perm = rng.permutation(c.shape[0])
    c = c[perm]
    assert _margin_ok(pp, c, w)
    got = bsh.bsh_cluster(_pp_ctypes(bsh, pp), torch.tensor(c, device="cuda"), w).cpu().numpy()
    want = PP.clusters(pp, c, w)
    assert np.array_equal(got.astype(np.int64), want)
    # the inside pairs joined, the outside pairs did not
    pos = np.argsort(perm)
    for q, joined in enumerate((True, False, True, False)):
        ia, ib = pos[n + 2 * q], pos[n + 2 * q + 1]
        assert (want[ia] == want[ib]) == joined
    assert len(np.unique(np.round((c[:n, 0] - 200.0) * TC))) == 12


def test_cluster_chain_spans_tiles(env):
    """A chain of 2000 templates 3.5 bins apart, shuffled, is one cluster across 8 row tiles;
    cutting one link splits it in two."""
    torch, bsh = env
    _say("cluster chain")
    pp = PP.PostParams()
    n = 2000
    base = np.array([200.0, 0.0, 0.0, 1.0, 2 * np.pi / (20 * DAY), 2e6])
    c = np.repeat(base[None, :], n, axis=0)
    steps = np.full(n, 3.5)
    steps[0] = 0
    steps[1234] = 3.9
    c[:, 0] += np.cumsum(steps) / TC
    perm = np.random.default_rng(4).permutation(n)
    c = c[perm]
    got = bsh.bsh_cluster(_pp_ctypes(bsh, pp), torch.tensor(c, device="cuda"), np.sqrt(14.0)).cpu().numpy()
    want = PP.clusters(pp, c, np.sqrt(14.0))
    assert np.array_equal(got.astype(np.int64), want)
    assert len(np.unique(got)) == 2


def test_clusters_at_top_list_size_on_samples(env):
    """10^5 templates (a per-band top-list of the full all-sky slice): every sampled template's
    neighbours share its label, labels are roots, and sampled clusters are connected."""
    torch, bsh = env
    _say("clusters n=1e5 sampled")
    pp = PP.PostParams()
    rng = np.random.default_rng(7)
    n = 100_000
    c = _cloud(rng, n, pp, n_centers=4000, spread=1.0)
    w = np.sqrt(14.0)
    lab = bsh.bsh_cluster(_pp_ctypes(bsh, pp), torch.tensor(c, device="cuda"), w).cpu().numpy().astype(np.int64)
    assert np.all(lab <= np.arange(n)) and np.all(lab[lab] == lab)
    res = PP.resolutions(pp, c)
    for i in rng.integers(0, n, 300):
        d2 = PP.distance2(pp, c[i][None, :], c, res[i][None, :], res)
        near = np.nonzero(d2 < w * w)[0]
        assert np.all(lab[near] == lab[i]), i
    for r in rng.choice(np.unique(lab), 50, replace=False):
        mem = np.nonzero(lab == r)[0]
        assert mem.min() == r
        assert np.array_equal(PP.clusters(pp, c[mem], w), np.zeros(mem.size, np.int64)), r


def test_coincidences_match_oracle(env):
    torch, bsh = env
    _say("coincidences")
    pp = PP.PostParams()
    rng = np.random.default_rng(9)
    a = _cloud(rng, 700, pp, n_centers=30)
    b = _cloud(np.random.default_rng(10), 513, pp, n_centers=30)
    sa = rng.uniform(1, 9, a.shape[0])
    sb = rng.uniform(1, 9, b.shape[0])
    win = 3.0
    d2 = PP.distance_matrix2(pp, a, b)
    assert np.min(np.abs(d2 - win * win)) > 1e-9 * win * win
    pairs_o, rows_o, sig_o = PP.coincidences(pp, a, sa, b, sb, win)
    m = pairs_o.shape[0]
    assert m > 50
    T = lambda x: torch.tensor(x, device="cuda")
    for cap in (m + 10, m // 3):
        n_p, pairs, rows, sig = bsh.bsh_coincidences(_pp_ctypes(bsh, pp), T(a), T(sa), T(b), T(sb), win, cap)
        k = min(m, cap)
        assert int(n_p.item()) == m
        assert np.array_equal(pairs[:k].cpu().numpy(), pairs_o[:k])
        assert np.allclose(rows[:k].cpu().numpy(), rows_o[:k], rtol=1e-14, atol=0)
        assert np.array_equal(sig[:k].cpu().numpy(), sig_o[:k])
    n_p, _, _, _ = bsh.bsh_coincidences(_pp_ctypes(bsh, pp), T(a), T(sa), T(b[:0]), T(sb[:0]), win, 4)
    assert int(n_p.item()) == 0


@pytest.mark.parametrize("cut", [0.0, 2.5])
def test_centroids_match_oracle(env, cut):
    torch, bsh = env
    _say(f"centroids cut={cut}")
    pp = PP.PostParams()
    rng = np.random.default_rng(12)
    n = 1500
    c = _cloud(rng, n, pp, n_centers=40)
    s = rng.uniform(0.5, 12, n)
    s[rng.integers(0, n, 20)] = 12.0          # exact ties for the top member
    w = np.sqrt(14.0)
    lab = PP.clusters(pp, c, w)
    if cut > 0:
        d2 = PP.distance_matrix2(pp, c, c)
        assert np.min(np.abs(d2 - cut * cut)) > 1e-9 * cut * cut
    T = lambda x: torch.tensor(x, device="cuda")
    st = bsh.Status("cuda")
    cen, weight, top, best = bsh.bsh_cluster_centroids(_pp_ctypes(bsh, pp), T(c), T(s),
                                                       T(lab.astype(np.int32)), cut=cut, status=st)
    torch.cuda.synchronize()
    assert st.value() == 0
    out, best_o = PP.centroids(pp, c, s, lab, cut=cut if cut > 0 else None)
    cen, weight, top = cen.cpu().numpy(), weight.cpu().numpy(), top.cpu().numpy()
    roots = np.unique(lab)
    non = np.setdiff1d(np.arange(n), roots)
    assert np.all(top[non] == -1) and np.all(weight[non] == 0)
    for r in roots:
        t_o, keep, w_o, c_o = out[int(r)]
        assert top[r] == t_o
        assert abs(weight[r] - w_o) <= 1e-12 * w_o
        assert np.allclose(cen[r], c_o, rtol=1e-12, atol=1e-12 * np.abs(c_o).max())
    b = int(best.item())
    assert abs(weight[b] - out[best_o][2]) <= 1e-12 * out[best_o][2]


def test_centroids_flag_bad_significance(env):
    torch, bsh = env
    _say("centroids status")
    pp = PP.PostParams()
    c = _cloud(np.random.default_rng(13), 50, pp)
    lab = PP.clusters(pp, c, np.sqrt(14.0)).astype(np.int32)
    s = np.ones(50)
    s[7] = -1.0
    T = lambda x: torch.tensor(x, device="cuda")
    st = bsh.Status("cuda")
    bsh.bsh_cluster_centroids(_pp_ctypes(bsh, pp), T(c), T(s), T(lab), status=st)
    torch.cuda.synchronize()
    assert st.value() & 4
    st.reset()
    bad = np.arange(50, dtype=np.int32)             # every row its own cluster, except that
    bad[5] = 4
    bad[3] = 5                                      # row 3 names row 5, which is not a root
    bsh.bsh_cluster_centroids(_pp_ctypes(bsh, pp), T(c), T(np.ones(50)), T(bad), status=st)
    torch.cuda.synchronize()
    assert st.value() & 4
