"""Host-side checks of the C ABI: the library loads, exports every declared symbol, enumerates
the template bank exactly like the oracle, and rejects bad arguments before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

import bsh_synth as S
import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1904_04873_amd import _native
    try:
        return _native.load()
    except ImportError as e:
        pytest.fail(f"libbsh.so must be built before the tests run: {e}")


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(bsh_\w+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = _lib()
    names = _declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    from paper_1904_04873_amd import _native
    assert sorted(_native.SIGNATURES) == names


def test_version():
    assert _lib().bsh_version() == 10000


@pytest.mark.parametrize("cfg", ["cfg1", "cfg2", "cfg3", "cfg5"])
def test_grid_build_equals_oracle_bitwise(cfg):
    from paper_1904_04873_amd import bsh
    grids = {"cfg1": lambda: S.config1().grids, "cfg2": lambda: S.config2(n_per_det=5).grids,
             "cfg3": lambda: S.config3(build_items=[]).grids,
             "cfg5": lambda: S.config5(n_pixels=1, n_per_det=5).grids}[cfg]()
    for g in grids:
        t_mid = 1.0e6 + 0.37
        a = bsh.bsh_grid_build(g, t_mid)
        b = O.grid_tables(g, t_mid)
        for x, y in zip(a, b):
            assert x.dtype == y.dtype and np.array_equal(x, y)


def test_grid_build_rejects_small_capacity():
    from paper_1904_04873_amd import _native as N
    L = _lib()
    g = S.config1().grids[0]
    cs = N.GridSpec(k0=g.k0, n_f0=g.n_f0, t_coh=900.0, ap_lo=g.ap_lo, ap_hi=g.ap_hi, n_ap=g.n_ap,
                    per_lo=g.per_lo, per_hi=g.per_hi, n_per=g.n_per, tasc_fixed=8, tasc_rule_m=60.0,
                    tasc_min=4, tasc_max=256)
    a = np.zeros(8); p = np.zeros(8); off = np.zeros(65, np.int64); t = np.zeros(10)
    nb = ctypes.c_int64(0)
    rc = L.bsh_grid_build(ctypes.byref(cs), 0.0, a.ctypes.data, p.ctypes.data, off.ctypes.data,
                          t.ctypes.data, 10, ctypes.byref(nb))
    assert rc == N.BSH_ENOMEM
    assert b"capacity" in L.bsh_last_error()


def _structs(n_bins=114, k_lo=90000 - 12, v_max=0.0, n_f0=90, n_per=8):
    from paper_1904_04873_amd import _native as N
    g = S.config1().grids[0]
    a_p, per, off, t_asc = O.grid_tables(g, 5e6)
    fake = 0x1000   # never dereferenced: every case below fails on the host
    seg = N.Segments(n_seg=64, t_coh=900.0, t_mid=fake, v_over_c=fake, weight=fake, weight_per_sky=0,
                     n_bins=n_bins, k_lo=k_lo, peak_bits=fake, power=fake, v_max_host=v_max)
    keep = (a_p, per, off)
    grid = N.Grid(n_sky=1, sky=fake, k0=90000, n_f0=n_f0, n_ap=8, n_per=n_per, a_p=fake, period=fake,
                  tasc_off=fake, t_asc=fake, a_p_host=a_p.ctypes.data, period_host=per.ctypes.data,
                  tasc_off_host=off.ctypes.data)
    return seg, grid, keep


def test_hough_count_rejects_bad_arguments_on_host():
    from paper_1904_04873_amd import _native as N
    L = _lib()
    seg, grid, keep = _structs()
    fake = ctypes.c_void_p(0x2000)
    assert L.bsh_hough_count(None, ctypes.byref(grid), fake, fake, None, None) == N.BSH_EINVAL
    assert L.bsh_hough_count(ctypes.byref(seg), None, fake, fake, None, None) == N.BSH_EINVAL
    assert L.bsh_hough_count(ctypes.byref(seg), ctypes.byref(grid), None, None, None, None) == N.BSH_EINVAL
    seg2, grid2, keep2 = _structs(n_bins=0)
    assert L.bsh_hough_count(ctypes.byref(seg2), ctypes.byref(grid2), fake, fake, None, None) == N.BSH_EINVAL
    seg3, grid3, keep3 = _structs(n_f0=91)
    assert L.bsh_hough_count(ctypes.byref(seg3), ctypes.byref(grid3), fake, fake, None, None) == N.BSH_EINVAL
    seg4, grid4, keep4 = _structs(n_per=300)
    assert L.bsh_hough_count(ctypes.byref(seg4), ctypes.byref(grid4), fake, fake, None, None) == N.BSH_EINVAL
    # an eccentricity pair must be finite with e < 0.5
    for ec, es in ((0.4, 0.31), (float("nan"), 0.0), (0.0, float("inf"))):
        seg5, grid5, keep5 = _structs()
        grid5.ecc_c, grid5.ecc_s = ec, es
        assert L.bsh_hough_count(ctypes.byref(seg5), ctypes.byref(grid5), fake, fake, None, None) == N.BSH_EINVAL
        assert b"eccentricity" in L.bsh_last_error()
    seg.t_coh = float("nan")
    assert L.bsh_hough_count(ctypes.byref(seg), ctypes.byref(grid), fake, fake, None, None) == N.BSH_EINVAL
    assert b"t_coh" in L.bsh_last_error()


def test_hough_count_host_window_check():
    """With |v|max known the host refuses a staged row narrower than the tracks' bound."""
    from paper_1904_04873_amd import _native as N
    L = _lib()
    fake = ctypes.c_void_p(0x2000)
    seg, grid, keep = _structs(n_bins=100, k_lo=90000 - 5, v_max=1.015e-4)
    assert L.bsh_hough_count(ctypes.byref(seg), ctypes.byref(grid), fake, fake, None, None) == N.BSH_ERANGE
    assert b"does not cover" in L.bsh_last_error()
    # the bound widens by (1 + e) for the ELL1 track's orbit term: a row that covers the circular
    # tracks with one bin to spare no longer covers eccentric ones
    g = S.config1().grids[0]
    apw = max(g.ap_hi * 2 * np.pi / g.per_lo, g.ap_lo * 2 * np.pi / g.per_lo)
    f_hi = 90000 + 90
    m = int(np.ceil(f_hi * (1.015e-4 + apw + 1.015e-4 * apw)))
    seg, grid, keep = _structs(n_bins=90 + 2 * m + 3, k_lo=90000 - m - 1, v_max=1.015e-4)
    spec = N.TopkSpec(k=10, sky_per_pass=0)
    # bsh_hough_count_topk checks the window before the workspace size: ENOMEM means it passed
    assert L.bsh_hough_count_topk(ctypes.byref(seg), ctypes.byref(grid), ctypes.byref(spec), fake, fake, fake, 0,
                                  None, None) == N.BSH_ENOMEM
    grid.ecc_c = 0.45
    assert L.bsh_hough_count_topk(ctypes.byref(seg), ctypes.byref(grid), ctypes.byref(spec), fake, fake, fake, 0,
                                  None, None) == N.BSH_ERANGE


def test_other_entry_points_reject_bad_arguments():
    from paper_1904_04873_amd import _native as N
    L = _lib()
    seg, grid, keep = _structs()
    fake = ctypes.c_void_p(0x2000)
    assert L.bsh_power_stat(ctypes.byref(seg), fake, 1, fake, fake, 10, 2, fake, None, None, None, None) == N.BSH_EINVAL
    assert L.bsh_power_stat(ctypes.byref(seg), fake, 1, fake, fake, 10, 1, fake, fake, None, None, None) == N.BSH_EINVAL
    assert L.bsh_power_stat(ctypes.byref(seg), fake, 0, fake, fake, 10, 0, fake, None, None, None, None) == N.BSH_EINVAL
    assert L.bsh_power_stat_grad(ctypes.byref(seg), fake, 1, fake, fake, -1, None, fake, None, None) == N.BSH_EINVAL
    assert L.bsh_power_stat_value_and_grad(ctypes.byref(seg), fake, 1, fake, fake, 5, None, None, fake, None,
                                           None) == N.BSH_EINVAL
    assert L.bsh_power_stat_value_and_grad(ctypes.byref(seg), fake, 1, fake, fake, 5, None, fake, None, None,
                                           None) == N.BSH_EINVAL
    assert L.bsh_power_stat_value_and_grad(ctypes.byref(seg), fake, 0, fake, fake, 5, None, fake, fake, None,
                                           None) == N.BSH_EINVAL
    assert L.bsh_track_bins(ctypes.byref(seg), None, 1, fake, fake, 3, fake, None, None) == N.BSH_EINVAL
    assert L.bsh_peakgram(fake, 10, 0, 1.6, fake, None) == N.BSH_EINVAL
    assert L.bsh_peakgram(fake, 10, 5, float("nan"), fake, None) == N.BSH_EINVAL
    assert L.bsh_topk(fake, None, 100, 10, fake, fake, fake, 16, None) == N.BSH_ENOMEM
    assert L.bsh_topk(fake, None, -1, 10, fake, fake, fake, 1 << 20, None) == N.BSH_EINVAL
    assert L.bsh_decode_templates(None, fake, 3, fake, fake, None) == N.BSH_EINVAL
    assert L.bsh_power_stat_ecc(ctypes.byref(seg), fake, 1, fake, fake, 10, 1, fake, fake, None, None, None) == N.BSH_EINVAL
    assert L.bsh_power_stat_ecc(ctypes.byref(seg), fake, 1, fake, fake, 10, 0, None, None, None, None, None) == N.BSH_EINVAL
    assert L.bsh_power_stat_grad_ecc(ctypes.byref(seg), fake, 1, fake, fake, -1, None, None, fake, None,
                                     None) == N.BSH_EINVAL
    assert L.bsh_power_stat_grad_ecc(ctypes.byref(seg), fake, 1, fake, fake, 5, None, fake, None, None,
                                     None) == N.BSH_EINVAL
    # the allocation-free top-k refuses a k its static workspace cannot hold, before any launch
    assert L.bsh_topk_noalloc_max_bytes() == 8 << 20
    assert L.bsh_topk_noalloc(fake, None, 1000, 1 << 30, fake, fake, None) == N.BSH_ENOMEM
    assert L.bsh_topk_noalloc(fake, None, -1, 10, fake, fake, None) == N.BSH_EINVAL
    assert L.bsh_topk_noalloc(fake, None, 100, 10, None, fake, None) == N.BSH_EINVAL
    assert L.bsh_topk_noalloc(None, None, 0, 0, None, None, None) == N.BSH_OK
    # empty work is a successful no-op without touching any pointer
    assert L.bsh_topk(None, None, 0, 0, None, None, None, 0, None) == N.BSH_OK
    assert L.bsh_power_stat(ctypes.byref(seg), fake, 1, fake, fake, 0, 0, fake, None, None, None, None) == N.BSH_OK


def test_count_topk_rejects_bad_arguments_on_host():
    """The bounded stage-1 top-k checks its spec and workspace before any launch; its workspace
    is one pass's map plus O(k)."""
    from paper_1904_04873_amd import _native as N
    L = _lib()
    seg, grid, keep = _structs()
    fake = ctypes.c_void_p(0x2000)
    spec = N.TopkSpec(k=100, sky_per_pass=0)
    need = L.bsh_hough_count_topk_workspace(ctypes.byref(grid), ctypes.byref(spec))
    assert need > 0
    big = N.TopkSpec(k=100000, sky_per_pass=0)
    assert L.bsh_hough_count_topk_workspace(ctypes.byref(grid), ctypes.byref(big)) > need
    bad = N.TopkSpec(k=0, sky_per_pass=0)
    assert L.bsh_hough_count_topk_workspace(ctypes.byref(grid), ctypes.byref(bad)) == 0
    args = (fake, fake, fake, need, None, None)
    assert L.bsh_hough_count_topk(ctypes.byref(seg), ctypes.byref(grid), None, *args) == N.BSH_EINVAL
    assert L.bsh_hough_count_topk(ctypes.byref(seg), ctypes.byref(grid), ctypes.byref(bad), *args) == N.BSH_EINVAL
    neg = N.TopkSpec(k=10, sky_per_pass=-1)
    assert L.bsh_hough_count_topk(ctypes.byref(seg), ctypes.byref(grid), ctypes.byref(neg), *args) == N.BSH_EINVAL
    assert L.bsh_hough_count_topk(ctypes.byref(seg), ctypes.byref(grid), ctypes.byref(spec), fake, None, fake, need,
                                  None, None) == N.BSH_EINVAL
    assert L.bsh_hough_count_topk(ctypes.byref(seg), ctypes.byref(grid), ctypes.byref(spec), fake, fake, fake,
                                  need - 1, None, None) == N.BSH_ENOMEM
    assert L.bsh_hough_count_topk(ctypes.byref(seg), ctypes.byref(grid), ctypes.byref(spec), fake, fake, None, need,
                                  None, None) == N.BSH_EINVAL


def test_topk_workspace_is_order_k():
    """The tie resolution re-reads the scores, so the workspace does not grow with n."""
    L = _lib()
    a = L.bsh_topk_workspace(1000, 10)
    b = L.bsh_topk_workspace(10**9, 10)
    c = L.bsh_topk_workspace(1000, 5000)
    assert a == b and c > a and c >= 12 * 5000
    assert L.bsh_topk_segmented_workspace(100, 10) > L.bsh_topk_segmented_workspace(1, 10)
    # the candidate pass's room for several lists: 32768 scores and indices per segment up to
    # k = 4096, 8 k (rounded up to 1024) beyond; none for a single list
    for k, cap in ((2048, 32768), (2049, 32768), (100000, 800768)):
        extra = L.bsh_topk_segmented_candidate_workspace(100, k) - L.bsh_topk_segmented_workspace(100, k)
        assert 100 * cap * 12 <= extra < 100 * cap * 12 + 4096, k
    assert L.bsh_topk_segmented_candidate_workspace(1, 10) == L.bsh_topk_segmented_workspace(1, 10)
    assert L.bsh_topk_segmented_candidate_workspace(0, 10) == 0


def test_plan_rejects_bad_items_on_host():
    from paper_1904_04873_amd import _native as N
    L = _lib()
    seg, grid, keep = _structs()
    fake = ctypes.c_void_p(0x2000)
    items = (N.Item * 2)()
    items[0] = N.Item(seg=seg, grid=0, sky_lo=0, n_sky=1, band=1)
    items[1] = N.Item(seg=seg, grid=0, sky_lo=0, n_sky=1, band=0)     # bands out of order
    grids = (N.Grid * 1)(grid)
    h = ctypes.c_void_p()
    opts = N.PlanOpts()
    assert L.bsh_plan_create(items, 2, grids, 1, 2, ctypes.byref(opts), fake, 10**9, None, None, None,
                             None, None, ctypes.byref(h)) == N.BSH_EINVAL
    assert b"ordered by band" in L.bsh_last_error()
    items[1] = N.Item(seg=seg, grid=3, sky_lo=0, n_sky=1, band=1)     # grid index out of range
    assert L.bsh_plan_create(items, 2, grids, 1, 2, ctypes.byref(opts), fake, 10**9, None, None, None,
                             None, None, ctypes.byref(h)) == N.BSH_EINVAL
    items[1] = N.Item(seg=seg, grid=0, sky_lo=1, n_sky=1, band=1)     # pixel outside the grid's sky
    assert L.bsh_plan_create(items, 2, grids, 1, 2, ctypes.byref(opts), fake, 10**9, None, None, None,
                             None, None, ctypes.byref(h)) == N.BSH_EINVAL
    items[1] = N.Item(seg=seg, grid=0, sky_lo=0, n_sky=1, band=1)
    assert L.bsh_items_map_floats(items, 2, grids, 1) == 2 * 46080
    assert L.bsh_plan_create(items, 2, grids, 1, 2, ctypes.byref(opts), fake, 1000, None, None, None,
                             None, None, ctypes.byref(h)) == N.BSH_ENOMEM
    bad = N.PlanOpts(lanes=96)
    assert L.bsh_plan_create(items, 2, grids, 1, 2, ctypes.byref(bad), fake, 10**9, None, None, None,
                             None, None, ctypes.byref(h)) == N.BSH_EINVAL
    assert L.bsh_plan_destroy(None) == N.BSH_OK
    assert L.bsh_plan_units(None) == -1
    assert L.bsh_plan_persistent(None) == -1
    assert L.bsh_plan_proven(None) == -1


def test_post_processing_entry_points_reject_bad_arguments():
    from paper_1904_04873_amd import _native as N
    L = _lib()
    fake = ctypes.c_void_p(0x2000)
    pp = N.PostParams(t_coh=900.0, t_obs=1e7, m_a=0.4, m_omega=0.4, m_t=0.4, pixel_factor=1.0, v_over_c=1e-4)
    bad = N.PostParams(t_coh=900.0, t_obs=1e7, m_a=0.0, m_omega=0.4, m_t=0.4, pixel_factor=1.0, v_over_c=1e-4)
    assert L.bsh_cluster(ctypes.byref(bad), fake, 10, 3.0, fake, None) == N.BSH_EINVAL
    assert L.bsh_cluster(None, fake, 10, 3.0, fake, None) == N.BSH_EINVAL
    assert L.bsh_cluster(ctypes.byref(pp), fake, 10, float("nan"), fake, None) == N.BSH_EINVAL
    assert L.bsh_cluster(ctypes.byref(pp), None, 10, 3.0, fake, None) == N.BSH_EINVAL
    assert L.bsh_cluster(ctypes.byref(pp), fake, 1 << 31, 3.0, fake, None) == N.BSH_EINVAL
    assert L.bsh_cluster(ctypes.byref(pp), None, 0, 3.0, None, None) == N.BSH_OK
    assert L.bsh_coincidences_workspace(100) >= 8 * 201
    assert L.bsh_coincidences(ctypes.byref(pp), fake, fake, 100, fake, fake, 50, 3.0, 10, fake, fake, fake,
                              fake, fake, 16, None) == N.BSH_ENOMEM
    assert L.bsh_coincidences(ctypes.byref(pp), fake, fake, 100, fake, fake, 50, 3.0, 10, None, fake, fake,
                              fake, fake, 1 << 20, None) == N.BSH_EINVAL
    assert L.bsh_coincidences(ctypes.byref(pp), fake, fake, 100, fake, fake, 50, -1.0, 10, fake, fake, fake,
                              fake, fake, 1 << 20, None) == N.BSH_EINVAL
    assert L.bsh_cluster_centroids(ctypes.byref(pp), fake, fake, fake, 100, 0.0, fake, fake, fake, fake,
                                   None, fake, 8, None) == N.BSH_ENOMEM
    assert L.bsh_cluster_centroids(ctypes.byref(pp), fake, fake, fake, 100, float("nan"), fake, fake, fake,
                                   fake, None, fake, 1 << 20, None) == N.BSH_EINVAL
    assert L.bsh_significance(fake, 10, fake, 10, 2, 1.6, fake, None) == N.BSH_EINVAL
    assert L.bsh_significance(fake, 10, fake, 0, 1, 1.6, fake, None) == N.BSH_EINVAL
    assert L.bsh_post_rows(fake, fake, fake, 10, 0.0, fake, None) == N.BSH_EINVAL
