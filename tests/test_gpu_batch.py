"""The batched plan: one persistent launch over uneven work items, replayed from a HIP graph.

Integer-exact and FP32-bitwise claims: the per-lane accumulation order does not depend on the
launch form or the tile shape, so batched, plain and single-item maps are bitwise identical.
"""
import sys

import numpy as np
import pytest

import bsh_synth as S
import oracle as O

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


ITEMS = [0, 1, 2, 256, 257, 1023]   # band 0 patches 0-2, band 1 patches 0-1, band 3 patch 255


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1904_04873_amd import bsh
    w = S.config3(build_items=ITEMS)
    dsegs, grids, items, hosts = [], [], [], []
    bands = sorted({w.item_grid[i] for i in ITEMS})
    for q, it in enumerate(ITEMS):
        seg = w.segments[it]
        band = w.item_grid[it]
        g = bsh.DeviceGrid.build(w.grids[band], seg.t_span_mid(), w.sky)
        ds = bsh.DeviceSegments.from_host(seg)
        p_lo, _ = w.item_sky[it]
        items.append((ds, q, p_lo, 1, bands.index(band)))
        dsegs.append(ds)
        grids.append(g)
        hosts.append((seg, w.grids[band]))
    torch.cuda.synchronize()
    return w, bsh, items, grids, hosts, len(bands)


def _np(t):
    return t.detach().cpu().numpy()


def test_batched_equals_plain_and_single_item(setup):
    import torch
    w, bsh, items, grids, hosts, n_bands = setup
    _say("batched vs plain vs single")
    plan = bsh.Plan(items, grids, n_bands, k_item=500, k_band=300, use_graph=False, persistent=False)
    assert not plan.persistent
    plan.run()
    torch.cuda.synchronize()
    plan.status.raise_if_set("batched")
    m_b = plan.maps.clone()
    li_b = (plan.item_score.clone(), plan.item_index.clone())
    lb_b = (plan.band_score.clone(), plan.band_index.clone())
    plan.maps.fill_(-1.0)
    plan.run_plain()
    torch.cuda.synchronize()
    plan.status.raise_if_set("plain")
    assert torch.equal(plan.maps, m_b)
    assert torch.equal(plan.item_score, li_b[0]) and torch.equal(plan.item_index, li_b[1])
    assert torch.equal(plan.band_score, lb_b[0]) and torch.equal(plan.band_index, lb_b[1])
    # each item's map equals a standalone bsh_hough_count of that item (its pixel only)
    for q, (ds, gi, lo, ns, band) in enumerate(items):
        g = grids[gi]
        g1 = bsh.DeviceGrid.from_tables(_np(g.sky)[lo:lo + 1], g.k0, g.n_f0, g.a_p, g.period, g.tasc_off,
                                        _np(g.t_asc_dev))
        ws, _ = bsh.bsh_hough_count(ds, g1)
        torch.cuda.synchronize()
        assert torch.equal(ws, plan.item_map(q)), f"item {q}"
    plan.close()
    # the persistent launch form (blocks pulling units from a queue counter) gives the same maps
    # and lists, also with fewer blocks than CUs, and so does the library's choice of form
    for blocks, form in ((0, True), (7, True), (0, None)):
        pp = bsh.Plan(items, grids, n_bands, k_item=500, k_band=300, use_graph=False, persistent=form, blocks=blocks)
        assert form is None or pp.persistent == form
        pp.run()
        torch.cuda.synchronize()
        pp.status.raise_if_set("persistent")
        assert torch.equal(pp.maps, m_b)
        assert torch.equal(pp.item_index, li_b[1]) and torch.equal(pp.band_index, lb_b[1])
        assert torch.equal(pp.band_score, lb_b[0])
        pp.close()


def test_proven_plan_equals_checked_plan(setup):
    """Every item's window proven on the host: the plan takes the table kernel's proven form
    (no per-track range tests); with one item's bound unknown it takes the checked form, and
    maps and lists agree bit for bit."""
    import torch
    w, bsh, items, grids, hosts, n_bands = setup
    _say("proven vs checked plan")
    pp = bsh.Plan(items, grids, n_bands, k_item=500, k_band=300, use_graph=False)
    assert pp.proven
    pp.run()
    torch.cuda.synchronize()
    pp.status.raise_if_set("proven")
    ds0 = items[0][0]
    v_max = ds0.v_max
    ds0.v_max = 0.0
    try:
        pc = bsh.Plan(items, grids, n_bands, k_item=500, k_band=300, use_graph=False)
    finally:
        ds0.v_max = v_max
    assert not pc.proven
    pc.run()
    torch.cuda.synchronize()
    pc.status.raise_if_set("checked")
    assert torch.equal(pp.maps, pc.maps)
    assert torch.equal(pp.item_index, pc.item_index) and torch.equal(pp.band_index, pc.band_index)
    assert torch.equal(pp.band_score, pc.band_score)
    pp.close()
    pc.close()


def test_lists_are_exact_topk_of_maps(setup):
    import torch
    w, bsh, items, grids, hosts, n_bands = setup
    _say("plan lists vs sort")
    plan = bsh.Plan(items, grids, n_bands, k_item=700, k_band=900, use_graph=True)
    plan.run()
    torch.cuda.synchronize()
    allsc, allix = [], []
    for q in range(len(items)):
        m = plan.item_map(q)
        order = torch.sort(m, descending=True, stable=True).indices[:700]
        assert torch.equal(plan.item_index[q], order | (q << 40))
        assert torch.equal(plan.item_score[q], m[order])
    for b in range(n_bands):
        qs = [q for q, it in enumerate(items) if it[4] == b]
        sc = torch.cat([plan.item_score[q] for q in qs]).cpu().numpy()
        ix = torch.cat([plan.item_index[q] for q in qs]).cpu().numpy()
        rv, ri = O.topk(sc, 900, ix)
        k = min(900, sc.size)
        assert np.array_equal(_np(plan.band_index[b])[:k], ri)
        assert np.array_equal(_np(plan.band_score[b])[:k], rv)
    plan.close()


def test_item_maps_match_oracle_on_samples(setup):
    import torch
    w, bsh, items, grids, hosts, n_bands = setup
    _say("plan maps vs oracle samples")
    plan = bsh.Plan(items, grids, n_bands, use_graph=False)
    plan.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for q, (ds, gi, lo, ns, band) in enumerate(items):
        seg, spec = hosts[q]
        g = grids[gi]
        m = _np(plan.item_map(q))
        idx = rng.integers(0, m.size, 400)
        s, b, i, ia, ip = O.decode_index(idx, g.n_bin, spec.n_f0, g.tasc_off, spec.n_per)
        o = O.grid_tables(spec, seg.t_span_mid())
        cand = np.stack([(spec.k0 + i).astype(np.float64), o[0][ia], o[1][ip], o[3][b]], axis=1)
        _, c_o, nw_o, nt_o = O.power_stat(seg, w.sky[lo:lo + 1], s.astype(np.int32), cand, mode=0)
        err = np.abs(m[idx].astype(np.float64) - nw_o)
        assert np.all(err <= 1e-5 * nw_o + nt_o * float(seg.weight.max())), f"item {q}"
    plan.close()


def test_graph_replays_match_eager(setup):
    import torch
    w, bsh, items, grids, hosts, n_bands = setup
    _say("graph replays")
    eager = bsh.Plan(items, grids, n_bands, k_item=200, k_band=100, use_graph=False)
    eager.run()
    torch.cuda.synchronize()
    ref = (eager.maps.clone(), eager.band_index.clone(), eager.band_score.clone())
    eager.close()
    graph = bsh.Plan(items, grids, n_bands, k_item=200, k_band=100, use_graph=True)
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        graph.maps.fill_(0.0)
        graph.band_index.fill_(-7)
        junk = (junk * 1.0001).sin()          # unrelated eager work between replays
        graph.run()
        torch.cuda.synchronize()
        assert torch.equal(graph.maps, ref[0]), f"replay {rep}"
        assert torch.equal(graph.band_index, ref[1]) and torch.equal(graph.band_score, ref[2])
    graph.close()


def test_every_tile_shape_gives_identical_maps(setup):
    import torch
    w, bsh, items, grids, hosts, n_bands = setup
    _say("tile shapes")
    ds, gi, lo, ns, band = items[3]
    g = grids[gi]
    g1 = bsh.DeviceGrid.from_tables(_np(g.sky)[lo:lo + 1], g.k0, g.n_f0, g.a_p, g.period, g.tasc_off,
                                    _np(g.t_asc_dev))
    ref, rc = bsh.bsh_hough_count(ds, g1, with_count=True, variant=1)      # select, with counts
    ref_t, rc_t = bsh.bsh_hough_count(ds, g1, with_count=True)            # table, counts with unit weights
    torch.cuda.synchronize()
    assert torch.equal(rc, rc_t)
    for lanes in (64, 128, 256, 512):
        for chunk in (128, 256, 512):
            ws, c = bsh.bsh_hough_count(ds, g1, with_count=True, lanes=lanes, chunk=chunk, variant=1)
            wt, ct = bsh.bsh_hough_count(ds, g1, with_count=True, lanes=lanes, chunk=chunk)
            torch.cuda.synchronize()
            assert torch.equal(ws, ref) and torch.equal(c, rc), (lanes, chunk)
            assert torch.equal(wt, ref_t) and torch.equal(ct, rc), (lanes, chunk)
    for variant, want in ((1, ref), (2, ref_t)):
        one = [(ds, 0, lo, ns, 0)]          # the item's grid is the only grid of this plan
        plan = bsh.Plan(one, [g], 1, lanes=64, chunk=512, use_graph=False, lpt=False, variant=variant)
        plan.run()
        torch.cuda.synchronize()
        assert torch.equal(plan.item_map(0), want), variant
        plan.close()


def test_passes_give_the_lists_of_one_pass(setup):
    """A map buffer smaller than all maps together runs the items in passes through it; the item
    and band lists are those of the plan with room for every map, bit for bit (graph and eager,
    batched and plain)."""
    import torch
    w, bsh, items, grids, hosts, n_bands = setup
    _say("plan passes vs one pass")
    ref = bsh.Plan(items, grids, n_bands, k_item=600, k_band=800, use_graph=True)
    assert ref.passes == 1
    ref.run()
    torch.cuda.synchronize()
    want = [t.clone() for t in (ref.item_score, ref.item_index, ref.band_score, ref.band_index)]
    largest = max(int(ref.offsets[q + 1] - ref.offsets[q]) for q in range(len(items)))
    ref.close()
    for buf, graph in ((largest, True), (largest + 1, False), (2 * largest, True)):
        plan = bsh.Plan(items, grids, n_bands, k_item=600, k_band=800, use_graph=graph, map_floats=buf)
        assert plan.passes > 1
        for rep in range(2):
            for t in (plan.item_score, plan.item_index, plan.band_score, plan.band_index):
                t.fill_(-3)
            plan.run() if rep == 0 else plan.run_plain()
            torch.cuda.synchronize()
            plan.status.raise_if_set("passes")
            got = (plan.item_score, plan.item_index, plan.band_score, plan.band_index)
            for a, b in zip(got, want):
                assert torch.equal(a, b), (buf, graph, rep)
        plan.close()


def test_plan_rejects_a_buffer_below_the_largest_item(setup):
    import torch
    w, bsh, items, grids, hosts, n_bands = setup
    from paper_1904_04873_amd._native import BshError
    sizes = [ns * grids[gi].n_bin * grids[gi].n_f0 for (_, gi, _, ns, _) in items]
    with pytest.raises(BshError):
        bsh.Plan(items, grids, n_bands, k_item=10, k_band=10, map_floats=max(sizes) - 1)
    with pytest.raises(BshError):          # passes need item lists
        bsh.Plan(items, grids, n_bands, map_floats=max(sizes))
    torch.cuda.synchronize()


@pytest.mark.timeout(600)
def test_two_whole_items_against_the_oracle_map(setup):
    """Two whole work items of the batching workload, map for map against the oracle: the
    smallest band's patch 0 (49 650 binary templates) and the widest band's patch 255 (145 824,
    t_asc up to 256 per cell): counts exact outside near-ties, weighted counts within 1e-5."""
    import torch
    w, bsh, items, grids, hosts, n_bands = setup
    _say("two whole items vs the oracle")
    plan = bsh.Plan(items, grids, n_bands, use_graph=False, variant=1)
    plan.run()
    torch.cuda.synchronize()
    plan.status.raise_if_set("plan")
    tab = bsh.Plan(items, grids, n_bands, use_graph=False)
    tab.run()
    torch.cuda.synchronize()
    for q in (0, len(items) - 1):
        ds, gi, lo, ns, band = items[q]
        seg, spec = hosts[q]
        g = grids[gi]
        o = O.grid_tables(spec, seg.t_span_mid())
        assert np.array_equal(g.tasc_off, o[2])
        _say(f"oracle: item {ITEMS[q]} ({g.n_bin} binary templates, {seg.n_seg} segments)")
        cnt_o, nw_o, nt_o, ntw_o = O.hough_count(seg, w.sky[lo:lo + 1], spec.k0, spec.n_f0, *o)
        wmax = float(seg.weight.max())
        for m in (_np(plan.item_map(q)), _np(tab.item_map(q))):
            err = np.abs(m.astype(np.float64) - nw_o)
            assert np.all(err <= 1e-5 * nw_o + ntw_o + 1e-30), f"item {ITEMS[q]}: max rel {np.max(err / np.maximum(nw_o, 1e-30))}"
        # unweighted counts, standalone on the item's pixel: the table variant's (unit weights) and
        # the select variant's, the same bit for bit
        g1 = bsh.DeviceGrid.from_tables(_np(g.sky)[lo:lo + 1], g.k0, g.n_f0, g.a_p, g.period, g.tasc_off,
                                        _np(g.t_asc_dev))
        _, c = bsh.bsh_hough_count(ds, g1, with_count=True)
        _, c_s = bsh.bsh_hough_count(ds, g1, with_count=True, variant=1)
        torch.cuda.synchronize()
        assert torch.equal(c, c_s)
        c = _np(c).view(np.uint32).astype(np.int64)
        assert np.all(np.abs(c - cnt_o.astype(np.int64)) <= nt_o), f"item {ITEMS[q]} counts"
        _say(f"item {ITEMS[q]}: near-tie templates {int((nt_o > 0).sum())}")
    plan.close()
    tab.close()
