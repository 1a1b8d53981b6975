"""The all-sky slice at its full size: 2 x 4000 segments over 240 d, band 300.0-300.1 Hz, a_p 128 x
P 64 x uneven t_asc = 581 531 binary templates (52.3 M templates) per sky pixel, all 2000 pixels
(1.05e11 templates, 8.4e14 template x segments) through one batched plan whose map buffer holds 64
pixels (13.4 GB instead of the 418 GB of every map), with per-pixel and per-band top-10^5; then
stage 2 and 20 Adam steps of the interpolated power on the 10^5 winners.

Against the oracle: every listed entry is recomputed (stage-1 weighted count of that template);
the list is in (score desc, index asc) order; the 10^5 best entries that just missed the list
score at most the list's k-th score; no template of a 10^6 random sample scores above the k-th
entry without being listed; the winners' stage-2 power matches on a sample.
"""
import sys

import numpy as np
import pytest

import bsh_synth as S
import oracle as O

pytestmark = pytest.mark.gpu

REL = 1e-5
K = 100_000
PASS_PIXELS = 64


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.timeout(900)
def test_allsky_slice_full_pipeline():
    import torch
    from paper_1904_04873_amd import bsh
    from paper_1904_04873_amd.refine import refine
    w = S.config5()
    seg, spec = w.segments[0], w.grids[0]
    n_pix = len(w.sky)
    t_mid = seg.t_span_mid()
    ds = bsh.DeviceSegments.from_host(seg)
    g = bsh.DeviceGrid.build(spec, t_mid, w.sky)
    a_p, per, off, t_asc = O.grid_tables(spec, t_mid)
    assert np.array_equal(g.tasc_off, off) and int(off[-1]) == 581531 and n_pix == 2000
    n_f0 = spec.n_f0
    per_pixel = int(off[-1]) * n_f0
    items = [(ds, 0, p, 1, 0) for p in range(n_pix)]
    plan = bsh.Plan(items, [g], 1, k_item=K, k_band=K, use_graph=False, map_floats=PASS_PIXELS * per_pixel)
    assert plan.passes == (n_pix + PASS_PIXELS - 1) // PASS_PIXELS
    _say(f"all-sky slice: {n_pix} pixels in {plan.passes} passes, top-1e5")
    plan.run()
    torch.cuda.synchronize()
    plan.status.raise_if_set("all-sky plan")
    score = _np(plan.band_score[0])
    index = _np(plan.band_index[0])

    # (score desc, index asc) order
    assert np.all(index >= 0)
    assert np.all((score[:-1] > score[1:]) | ((score[:-1] == score[1:]) & (index[:-1] < index[1:])))
    wmax = float(seg.weight.max())

    def oracle_scores(pix, pos):
        s, b, i, ia, ip = O.decode_index(pos, int(off[-1]), n_f0, off, spec.n_per)
        assert np.all(s == 0)
        cand = np.stack([(spec.k0 + i).astype(np.float64), a_p[ia], per[ip], t_asc[b]], axis=1)
        _, _, nw, nt = O.power_stat(seg, w.sky, np.asarray(pix, np.int32), cand, mode=0)
        return nw, nt

    item = index >> 40
    pos = index & ((1 << 40) - 1)
    _say("oracle on the 1e5 listed templates")
    nw, nt = oracle_scores(item, pos)
    assert np.all(np.abs(score.astype(np.float64) - nw) <= REL * nw + nt * wmax)
    kth = float(score[-1])

    # the next 1e5 entries of the pixels' lists (the best templates that missed the cut)
    flat_s = plan.item_score.reshape(-1)
    flat_i = plan.item_index.reshape(-1)
    s2, i2 = bsh.bsh_topk(flat_s, 2 * K, index=flat_i)
    torch.cuda.synchronize()
    assert np.array_equal(_np(i2)[:K], index)
    run_s, run_i = _np(s2)[K:], _np(i2)[K:]
    _say("oracle on the 1e5 runners-up")
    nw_r, nt_r = oracle_scores(run_i >> 40, run_i & ((1 << 40) - 1))
    assert np.all(np.abs(run_s.astype(np.float64) - nw_r) <= REL * nw_r + nt_r * wmax)
    assert np.all(nw_r - nt_r * wmax <= kth * (1 + REL))

    # completeness on a 10^6 random sample of all 2000 maps
    _say("oracle on a 1e6-template sample")
    rng = np.random.default_rng(5)
    q_pix = rng.integers(0, n_pix, 1_000_000)
    q_pos = rng.integers(0, per_pixel, 1_000_000)
    nw_q, nt_q = oracle_scores(q_pix, q_pos)
    listed = set(index.tolist())
    above = np.nonzero(nw_q - nt_q * wmax > kth * (1 + REL))[0]
    _say(f"sampled templates above the k-th score: {above.size}")
    for j in above:
        assert ((int(q_pix[j]) << 40) | int(q_pos[j])) in listed, j

    # stage 2 on the winners, then 20 Adam steps of the interpolated power
    gidx = torch.from_numpy(item * per_pixel + pos).cuda()
    plan.close()
    cs, cp = bsh.bsh_decode_templates(g, gidx)
    st = bsh.Status(torch.device("cuda"))
    P = bsh.bsh_power_stat(ds, g.sky, cs, cp, mode=0, status=st)
    v2, pos2 = bsh.bsh_topk(P, w.topk_stage2)
    torch.cuda.synchronize()
    st.raise_if_set("stage 2")
    assert np.array_equal(_np(cs), item.astype(np.int32))
    samp = rng.choice(K, 3000, replace=False)
    P_o, _, _, nt_p = O.power_stat(seg, w.sky, _np(cs)[samp], _np(cp)[samp], mode=0)
    assert np.all(np.abs(_np(P)[samp].astype(np.float64) - P_o) <= REL * P_o + nt_p * float(seg.power.max()) * wmax)
    steps = torch.tensor([1.0, (spec.ap_hi - spec.ap_lo) / (spec.n_ap - 1),
                          (spec.per_hi - spec.per_lo) / (spec.n_per - 1), 0.0], dtype=torch.float64,
                         device="cuda").repeat(K, 1)
    steps[:, 3] = cp[:, 2] / 64.0
    theta, hist = refine(cp.contiguous(), steps, ds, g.sky, cs, n_iter=20, lr=0.05, status=st)
    torch.cuda.synchronize()
    st.raise_if_set("refinement")
    h = _np(hist)
    assert np.all(np.isfinite(h))
    assert np.median(h[-1] - h[0]) > 0, "refinement did not raise the typical candidate's power"
