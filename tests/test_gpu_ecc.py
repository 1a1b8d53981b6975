"""GPU parity of the low-eccentricity (ELL1) track of eq:frequencyevo in both stages, through the
C ABI: the stage-1 count of a grid with an eccentricity pair, its batched form mixed with
circular grids, the stage-2 statistic and counts on the same track, and the adjoint in all six
parameters.  Acceptance as in test_gpu_parity: counts exact up to oracle-flagged near-ties,
weighted sums and powers to 1e-5 relative, gradients to 1e-5 of the sum of absolute terms; with
zero eccentricity every result equals the circular kernels' bit for bit."""
import math
import sys

import numpy as np
import pytest

import bsh_synth as S
import oracle as O

pytestmark = pytest.mark.gpu

REL = 1e-5


@pytest.fixture(scope="module")
def B():
    import torch  # noqa: F401
    from paper_1904_04873_amd import bsh
    return bsh


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _np(t):
    return t.detach().cpu().numpy()


def _check_counts(cnt_g, ws_g, cnt_o, nw_o, nt_o, ntw_o):
    if cnt_g is not None:
        diff = np.abs(cnt_g.astype(np.int64) - cnt_o.astype(np.int64))
        assert np.all(diff <= nt_o), f"count mismatch outside near-ties at {np.nonzero(diff > nt_o)[0][:10]}"
    err = np.abs(ws_g.astype(np.float64) - nw_o)
    assert np.all(err <= REL * np.abs(nw_o) + ntw_o + 1e-30), f"max rel err {np.max(err / np.maximum(nw_o, 1e-30))}"


def _ecc_pair(e, om):
    return e * math.cos(om), e * math.sin(om)


def _count(B, ds, g, variant, with_count):
    import torch
    st = B.Status(torch.device("cuda"))
    ws, cnt = B.bsh_hough_count(ds, g, with_count=with_count, variant=variant, status=st)
    torch.cuda.synchronize()
    st.raise_if_set("bsh_hough_count (ELL1)")
    return _np(ws), (_np(cnt).view(np.uint32) if cnt is not None else None)


@pytest.mark.parametrize("e", [0.002, 0.03])
def test_ecc_count_matches_oracle_map(B, e):
    """400 gapped segments, 8 a_p x 4 P x 64 t_asc (8 tiles per pixel), 2 pixels: every template of
    the ELL1 map against the oracle, with counts and with the table variant."""
    _say(f"ELL1 count e={e}")
    w = S.config2(n_per_det=200)
    seg = w.segments[0]
    spec = S.GridSpec(k0=180000, n_f0=90, ap_lo=0.3, ap_hi=3.0, n_ap=8, per_lo=15 * S.DAY,
                      per_hi=45 * S.DAY, n_per=4, tasc_fixed=64)
    sky = S.fibonacci_sphere(2)
    ec, es = _ecc_pair(e, 2.3)
    ds = B.DeviceSegments.from_host(seg)
    g = B.DeviceGrid.build(spec, seg.t_span_mid(), sky, ecc=(ec, es))
    o = O.grid_tables(spec, seg.t_span_mid())
    cnt_o, nw_o, nt_o, ntw_o = O.hough_count_ecc(seg, sky, spec.k0, spec.n_f0, *o, ec, es)
    ws, cnt = _count(B, ds, g, 1, True)
    _check_counts(cnt, ws, cnt_o, nw_o, nt_o, ntw_o)
    ws_t, _ = _count(B, ds, g, 2, False)
    _check_counts(None, ws_t, cnt_o, nw_o, nt_o, ntw_o)
    # counts from the table variant (unit weights): the select variant's, bit for bit
    ws_tc, cnt_t = _count(B, ds, g, 2, True)
    assert np.array_equal(cnt_t, cnt) and np.array_equal(ws_tc, ws_t)
    # the eccentric terms move bins: the circular map differs
    ws_c, _ = _count(B, ds, g.with_ecc(0.0, 0.0), 2, False)
    assert not np.array_equal(ws_c, ws_t)


def test_ecc_count_ragged_per_sky_weights_every_tile_shape(B):
    """Uneven t_asc per cell, 3 pixels with their own weights, n_f0 = 37: the ELL1 map against the
    oracle, and bitwise the same at every tile shape."""
    import torch
    _say("ELL1 count ragged, tile shapes")
    rng = np.random.default_rng(7)
    base = S.tiny_segments(n_seg=300, k0=150000, n_f0=37, margin=19, seed=22, span_days=200)
    spec = S.GridSpec(k0=150000, n_f0=37, ap_lo=0.05, ap_hi=3.25, n_ap=5, per_lo=15 * S.DAY,
                      per_hi=45 * S.DAY, n_per=3)
    sky = S.fibonacci_sphere(3)
    wps = np.exp(0.3 * rng.standard_normal((3, 300))).astype(np.float32)
    ec, es = _ecc_pair(0.01, 4.0)
    ds = B.DeviceSegments.from_host(base, weight=wps)
    g = B.DeviceGrid.build(spec, base.t_span_mid(), sky, ecc=(ec, es))
    o = O.grid_tables(spec, base.t_span_mid())
    seg_o = S.Segments(t_mid=base.t_mid, v_over_c=base.v_over_c, weight=wps, power=base.power,
                       k_lo=base.k_lo, n_bins=base.n_bins)
    cnt_o, nw_o, nt_o, ntw_o = O.hough_count_ecc(seg_o, sky, spec.k0, spec.n_f0, *o, ec, es, weight_per_sky=True)
    ref = None
    for lanes in (64, 256, 512):
        for chunk in (128, 512):
            ws, _ = B.bsh_hough_count(ds, g, variant=2, lanes=lanes, chunk=chunk)
            torch.cuda.synchronize()
            ws = _np(ws)
            if ref is None:
                ref = ws
                _check_counts(None, ws, cnt_o, nw_o, nt_o, ntw_o)
            assert np.array_equal(ws, ref), (lanes, chunk)


def test_ecc_stage2_counts_agree_with_stage1_on_grid(B):
    """Stage 2 on the ELL1 track at every grid template of the tiny band selects the stage-1 bins:
    its counts and weighted counts equal the stage-1 map exactly; its power matches the oracle."""
    import torch
    _say("ELL1 stage 1 vs stage 2 bins")
    w = S.config1()
    seg, spec = w.segments[0], w.grids[0]
    ec, es = _ecc_pair(0.02, 0.7)
    ds = B.DeviceSegments.from_host(seg)
    g = B.DeviceGrid.build(spec, seg.t_span_mid(), w.sky, ecc=(ec, es))
    ws, cnt = _count(B, ds, g, 1, True)
    idx = torch.arange(g.n_templates, device="cuda", dtype=torch.int64)
    cs, cp = B.bsh_decode_templates(g, idx)
    ce = B.with_ecc_columns(cp, ec, es)
    P, c2, w2 = B.bsh_power_stat_ecc(ds, g.sky, cs, ce, mode=0, with_counts=True)
    torch.cuda.synchronize()
    assert np.array_equal(_np(c2).view(np.uint32), cnt)
    assert np.array_equal(_np(w2), ws)
    P_o, nt_o = O.power_stat_ecc(seg, w.sky, _np(cs), _np(ce), mode=0)
    tol = REL * np.abs(P_o) + nt_o * float(seg.weight.max()) * float(seg.power.max())
    assert np.all(np.abs(_np(P).astype(np.float64) - P_o) <= tol)


def test_ecc_stage2_zero_eccentricity_is_circular_with_counts(B):
    import torch
    _say("ELL1 stage 2 at e = 0")
    w = S.config2(n_per_det=500)
    seg = w.segments[0]
    ds = B.DeviceSegments.from_host(seg)
    sky = torch.from_numpy(w.sky).cuda()
    rng = np.random.default_rng(3)
    cand = np.stack([180000 + rng.uniform(0, 89, 700), rng.uniform(0.01, 3, 700),
                     rng.uniform(15, 45, 700) * S.DAY, rng.uniform(0, 3e6, 700)], axis=1)
    cs = torch.zeros(700, dtype=torch.int32, device="cuda")
    cp = torch.from_numpy(cand).cuda()
    a = B.bsh_power_stat(ds, sky, cs, cp, mode=0, with_counts=True)
    b = B.bsh_power_stat_ecc(ds, sky, cs, B.with_ecc_columns(cp, 0.0, 0.0), mode=0, with_counts=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_ecc_adjoint_matches_oracle(B):
    """bsh_power_stat_grad_ecc on 2000 eccentric candidates x 4000 segments: all six columns against
    the FP64 oracle, P_lin from the same pass against the oracle; at e = 0 the first four columns
    are the circular adjoint's bit for bit."""
    import torch
    _say("ELL1 adjoint")
    w = S.config2()
    seg = w.segments[0]
    ds = B.DeviceSegments.from_host(seg)
    sky = torch.from_numpy(w.sky).cuda()
    rng = np.random.default_rng(11)
    n = 2000
    cand = np.stack([180000 + rng.uniform(0, 89, n), rng.uniform(0.3, 3, n),
                     rng.uniform(15, 45, n) * S.DAY, rng.uniform(0, 3e6, n)], axis=1)
    e = 10 ** rng.uniform(-4, -1.5, n)
    om = rng.uniform(0, 2 * math.pi, n)
    ce = np.concatenate([cand, np.stack([e * np.cos(om), e * np.sin(om)], axis=1)], axis=1)
    gp = rng.standard_normal(n)
    cs = np.zeros(n, np.int32)
    st = B.Status(torch.device("cuda"))
    P, g = B.bsh_power_stat_grad_ecc(ds, sky, torch.from_numpy(cs).cuda(), torch.from_numpy(ce).cuda(),
                                     grad_P=torch.from_numpy(gp).cuda(), status=st)
    torch.cuda.synchronize()
    st.raise_if_set("bsh_power_stat_grad_ecc")
    g_o, a_o = O.power_grad_ecc(seg, w.sky, cs, ce, grad_p=gp, with_abs=True)
    assert np.all(np.abs(_np(g) - g_o) <= REL * a_o + 1e-300)
    P_o, _ = O.power_stat_ecc(seg, w.sky, cs, ce, mode=1)
    assert np.all(np.abs(_np(P).astype(np.float64) - P_o) <= REL * np.abs(P_o))
    z = np.concatenate([cand, np.zeros((n, 2))], axis=1)
    _, g0 = B.bsh_power_stat_grad_ecc(ds, sky, torch.from_numpy(cs).cuda(), torch.from_numpy(z).cuda(),
                                      grad_P=torch.from_numpy(gp).cuda())
    gc = B.bsh_power_stat_grad(ds, sky, torch.from_numpy(cs).cuda(), torch.from_numpy(cand).cuda(),
                               grad_P=torch.from_numpy(gp).cuda())
    torch.cuda.synchronize()
    assert torch.equal(g0[:, :4].contiguous(), gc)


def test_eccentricity_search_in_one_batched_plan(B):
    """A search over (e cos w, e sin w): one batched plan over the same segments with a circular
    grid and three eccentric grids (the circular item then runs through the ELL1 kernel with zero
    eccentric terms).  Each item's map equals its own bsh_hough_count map bit for bit; the band's
    best template belongs to the grid of an injected eccentric signal, at the injection's
    template, and the oracle agrees with the listed scores."""
    import torch
    _say("ELL1 search plan")
    seg = S.tiny_segments(n_seg=600, k0=180000, n_f0=90, margin=24, seed=31, span_days=120)
    spec = S.GridSpec(k0=180000, n_f0=90, ap_lo=1.5, ap_hi=3.0, n_ap=4, per_lo=15 * S.DAY,
                      per_hi=25 * S.DAY, n_per=3, tasc_fixed=16)
    a_p, per, off, ta = O.grid_tables(spec, seg.t_span_mid())
    pairs = [(0.0, 0.0), _ecc_pair(0.01, 1.0), _ecc_pair(0.03, 2.0), _ecc_pair(0.03, 5.0)]
    # inject on grid 2's track of one template: rho = 2 + noise there
    b_true, i_true = 101, 45
    cell = np.searchsorted(off, b_true, side="right") - 1
    row = np.array([[180000 + i_true, a_p[cell // spec.n_per], per[cell % spec.n_per], ta[b_true], *pairs[2]]])
    _, k = O.track_ecc(seg, S.fixed_pixel(), [0], row)
    seg.power[np.arange(seg.n_seg), k[0] - seg.k_lo] += 4.0
    ds = B.DeviceSegments.from_host(seg)
    g0 = B.DeviceGrid.build(spec, seg.t_span_mid(), S.fixed_pixel())
    grids = [g0.with_ecc(*p) for p in pairs]
    items = [(ds, q, 0, 1, 0) for q in range(len(grids))]
    plan = B.Plan(items, grids, 1, k_item=50, k_band=50, use_graph=False)
    plan.run()
    torch.cuda.synchronize()
    plan.status.raise_if_set("ELL1 plan")
    for q, g in enumerate(grids):
        ws, _ = _count(B, ds, g, 2, False)
        assert np.array_equal(_np(plan.item_map(q)), ws), q
    top = int(_np(plan.band_index[0])[0])
    assert top >> 40 == 2
    assert (top & ((1 << 40) - 1)) == b_true * 90 + i_true
    cnt_o, nw_o, nt_o, ntw_o = O.hough_count_ecc(seg, S.fixed_pixel(), spec.k0, spec.n_f0, a_p, per, off, ta,
                                                 *pairs[2])
    _check_counts(None, _np(plan.item_map(2)), cnt_o, nw_o, nt_o, ntw_o)
