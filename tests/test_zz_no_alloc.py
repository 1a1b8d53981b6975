"""The allocation-free top-k (bsh_topk_noalloc: workspace in a static per-GPU device array)
against bsh_topk with a caller-given workspace: identical lists, bit for bit, on two calls in a
row (the second smaller, so it runs over the first call's leftovers in the shared array), with
implicit and explicit indices, ties, and the largest k the array holds."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _largest_k():
    from paper_1904_04873_amd import _native as N
    L = N.load()
    cap = int(L.bsh_topk_noalloc_max_bytes())
    lo, hi = 1, 1 << 24
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if int(L.bsh_topk_workspace(mid, mid)) <= cap:
            lo = mid
        else:
            hi = mid
    return lo


def _pair(score, k, index=None):
    import torch
    from paper_1904_04873_amd import bsh
    ref_s, ref_i = bsh.bsh_topk(score, k, index=index)
    # outputs pre-filled with garbage: every slot must be written
    out_s = torch.full((k,), 7.0, dtype=torch.float32, device=score.device)
    out_i = torch.full((k,), 12345, dtype=torch.int64, device=score.device)
    got_s, got_i = bsh.bsh_topk_noalloc(score, k, index=index, out_score=out_s, out_index=out_i)
    torch.cuda.synchronize()
    assert got_s.data_ptr() == out_s.data_ptr() and got_i.data_ptr() == out_i.data_ptr()
    rs, ri = ref_s.cpu().numpy(), ref_i.cpu().numpy()
    gs, gi = got_s.cpu().numpy(), got_i.cpu().numpy()
    assert np.array_equal(rs.view(np.uint32), gs.view(np.uint32))
    assert np.array_equal(ri, gi)
    return gs, gi


def test_noalloc_topk_equals_workspace_topk_on_two_calls():
    import torch
    from paper_1904_04873_amd import bsh
    from paper_1904_04873_amd import _native as N
    dev = torch.device("cuda")
    g = torch.Generator(device="cpu").manual_seed(11)
    k_max = _largest_k()
    _say(f"largest k of the static workspace: {k_max}")
    assert k_max >= 200_000

    # call 1: long list, k in the bucketed ordering, many exact ties
    n1, k1 = 3_000_000, 150_000
    s1 = torch.randint(0, 5000, (n1,), generator=g).to(torch.float32).to(dev)
    _say(f"call 1: n={n1}, k={k1}")
    v1, i1 = _pair(s1, k1)
    assert np.all(np.diff(v1) <= 0)

    # call 2: smaller input and k, continuous scores; reuses the array the first call left
    n2, k2 = 50_001, 777
    s2 = torch.rand(n2, generator=g).to(dev)
    _say(f"call 2: n={n2}, k={k2}")
    v2, i2 = _pair(s2, k2)
    ref = np.argsort(-s2.cpu().numpy(), kind="stable")[:k2]
    assert np.array_equal(i2, ref)

    # explicit indices (merging lists), the one-block path, and the largest k
    idx = (torch.randperm(n2, generator=g).to(torch.int64) * 3 + (5 << 40)).to(dev)
    _say("explicit indices")
    _pair(s2, 1000, index=idx)
    _say("short list (one-block path)")
    _pair(s2[:300].contiguous(), 50)
    _say(f"k = {k_max}")
    s3 = torch.randn(k_max + 12345, generator=g).to(dev)
    _pair(s3, k_max)
    # k above the array's capacity is refused without a launch
    with pytest.raises(N.BshError) as e:
        bsh.bsh_topk_noalloc(s3, k_max + 1)
    assert e.value.code == N.BSH_ENOMEM
    # fewer entries than k: the tail is (-inf, -1), as bsh_topk writes it
    _say("n < k")
    _pair(s2[:10].contiguous(), 25)
