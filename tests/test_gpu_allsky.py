"""The all-sky slice at its real per-pixel size: 2 x 4000 segments over 240 d, band 300.0-300.1 Hz,
a_p 128 x P 64 x uneven t_asc = 581 531 binary templates (52.3 M templates) per sky pixel, on 8 of
its 2000 pixels through the batched plan with a per-band top-10^5.

Every listed entry is recomputed by the oracle (stage-1 weighted count of that template), the list
is in (score desc, index asc) order, and no template of a random sample scores above the k-th
entry without being listed.
"""
import sys

import numpy as np
import pytest

import bsh_synth as S
import oracle as O

pytestmark = pytest.mark.gpu

REL = 1e-5
PIXELS = [0, 250, 500, 777, 1000, 1333, 1700, 1999]
K = 100_000


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def test_allsky_slice_toplist_against_oracle():
    import torch
    from paper_1904_04873_amd import bsh
    _say("all-sky slice, 8 pixels, top-1e5")
    w = S.config5()
    seg, spec = w.segments[0], w.grids[0]
    t_mid = seg.t_span_mid()
    ds = bsh.DeviceSegments.from_host(seg)
    g = bsh.DeviceGrid.build(spec, t_mid, w.sky)
    a_p, per, off, t_asc = O.grid_tables(spec, t_mid)
    assert np.array_equal(g.tasc_off, off) and int(off[-1]) == 581531
    items = [(ds, 0, p, 1, 0) for p in PIXELS]
    plan = bsh.Plan(items, [g], 1, k_item=K, k_band=K, use_graph=False)
    plan.run()
    torch.cuda.synchronize()
    plan.status.raise_if_set("all-sky plan")
    score = plan.band_score[0].cpu().numpy()
    index = plan.band_index[0].cpu().numpy()
    plan.close()

    # (score desc, index asc) order
    assert np.all(index >= 0)
    assert np.all((score[:-1] > score[1:]) | ((score[:-1] == score[1:]) & (index[:-1] < index[1:])))

    n_f0 = spec.n_f0
    item = index >> 40
    pos = index & ((1 << 40) - 1)
    s, b, i, ia, ip = O.decode_index(pos, int(off[-1]), n_f0, off, spec.n_per)
    assert np.all(s == 0) and np.all(item < len(PIXELS))
    cand = np.stack([(spec.k0 + i).astype(np.float64), a_p[ia], per[ip], t_asc[b]], axis=1)
    cs = np.asarray(PIXELS, np.int32)[item]
    _say("oracle on 1e5 listed templates")
    _, _, nw, nt = O.power_stat(seg, w.sky, cs, cand, mode=0)
    wmax = float(seg.weight.max())
    assert np.all(np.abs(score.astype(np.float64) - nw) <= REL * nw + nt * wmax)

    # completeness on a random sample of the 8 maps
    _say("oracle on a 2e4-template sample")
    rng = np.random.default_rng(5)
    n_map = int(off[-1]) * n_f0
    q_item = rng.integers(0, len(PIXELS), 20000)
    q_pos = rng.integers(0, n_map, 20000)
    s2, b2, i2, ia2, ip2 = O.decode_index(q_pos, int(off[-1]), n_f0, off, spec.n_per)
    cand2 = np.stack([(spec.k0 + i2).astype(np.float64), a_p[ia2], per[ip2], t_asc[b2]], axis=1)
    _, _, nw2, nt2 = O.power_stat(seg, w.sky, np.asarray(PIXELS, np.int32)[q_item], cand2, mode=0)
    kth = float(score[-1])
    listed = set(((q << 40) | p) for q, p in zip(item.tolist(), pos.tolist()))
    above = np.nonzero(nw2 - nt2 * wmax > kth * (1 + REL))[0]
    for j in above:
        assert ((int(q_item[j]) << 40) | int(q_pos[j])) in listed, j
