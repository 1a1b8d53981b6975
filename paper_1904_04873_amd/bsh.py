"""Torch-facing binding of libbsh (same names as include/bsh.h).

PyTorch only provides device memory and the current HIP stream; every step of
the search runs in the library's HIP kernels.  All calls are asynchronous on
``torch.cuda.current_stream()``; outputs are returned as new tensors unless an
``out=`` tensor is given.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _native as N
from ._native import BshError, check

__all__ = [
    "BshError", "DeviceSegments", "DeviceGrid", "Status", "TopK", "Plan", "bsh_version",
    "bsh_grid_build", "bsh_normalize", "bsh_peakgram", "bsh_hough_count", "bsh_hough_count_topk",
    "bsh_topk", "bsh_topk_noalloc",
    "bsh_decode_templates", "bsh_power_stat", "bsh_power_stat_ecc", "bsh_power_stat_grad",
    "bsh_power_stat_grad_ecc", "with_ecc_columns",
    "bsh_power_stat_value_and_grad",
    "bsh_track_bins", "post_params", "bsh_post_rows", "bsh_significance", "bsh_coincidences",
    "bsh_cluster", "bsh_cluster_centroids",
]


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dev(a, dtype, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)


class Status:
    """A device int32 the kernels OR error bits into; read it after a synchronisation."""

    def __init__(self, device):
        self.t = torch.zeros(1, dtype=torch.int32, device=device)

    def ptr(self) -> int:
        return self.t.data_ptr()

    def reset(self) -> None:
        self.t.zero_()

    def value(self) -> int:
        return int(self.t.item())

    def raise_if_set(self, where: str = "kernel") -> None:
        v = self.value()
        if v:
            what = []
            if v & N.STATUS_RANGE:
                what.append("a track left the staged row")
            if v & N.STATUS_MODEL:
                what.append("a track drifted more than one bin across the f0 band")
            if v & N.STATUS_INPUT:
                what.append("an input is out of range (a candidate's sky pixel, a significance or a "
                            "cluster label)")
            raise BshError(N.BSH_ERANGE, where, "; ".join(what))


@dataclasses.dataclass
class DeviceSegments:
    """One work item's per-segment tables on the device plus the C struct that points at them."""
    t_mid: torch.Tensor
    v_over_c: torch.Tensor
    weight: torch.Tensor
    k_lo: int
    n_bins: int
    t_coh: float
    peak_bits: Optional[torch.Tensor] = None
    power: Optional[torch.Tensor] = None
    weight_per_sky: bool = False
    v_max: float = 0.0

    @classmethod
    def from_host(cls, seg, device="cuda", with_power: bool = True, rho_th: float = 1.6,
                  weight=None) -> "DeviceSegments":
        """Upload a host segment set (fields t_mid, v_over_c, weight, power, k_lo, n_bins, t_coh)
        and build its peakgram on the device with bsh_peakgram."""
        w = seg.weight if weight is None else weight
        power = _dev(seg.power, torch.float32, device)
        ds = cls(t_mid=_dev(seg.t_mid, torch.float64, device),
                 v_over_c=_dev(seg.v_over_c, torch.float64, device),
                 weight=_dev(w, torch.float32, device), k_lo=int(seg.k_lo), n_bins=int(seg.n_bins),
                 t_coh=float(seg.t_coh), power=power if with_power else None,
                 weight_per_sky=bool(np.ndim(w) == 2),
                 v_max=float(np.linalg.norm(np.asarray(seg.v_over_c), axis=1).max()) if seg.n_seg else 0.0)
        ds.peak_bits = bsh_peakgram(power, rho_th)
        return ds

    @property
    def n_seg(self) -> int:
        return int(self.t_mid.numel())

    def struct(self) -> N.Segments:
        return N.Segments(n_seg=self.n_seg, t_coh=self.t_coh, t_mid=_ptr(self.t_mid),
                          v_over_c=_ptr(self.v_over_c), weight=_ptr(self.weight),
                          weight_per_sky=int(self.weight_per_sky), n_bins=self.n_bins, k_lo=self.k_lo,
                          peak_bits=_ptr(self.peak_bits), power=_ptr(self.power),
                          v_max_host=float(self.v_max))


@dataclasses.dataclass
class DeviceGrid:
    """One band's template grid: device tables, host copies of the small ones, and the C struct."""
    sky: torch.Tensor
    k0: int
    n_f0: int
    a_p: np.ndarray
    period: np.ndarray
    tasc_off: np.ndarray
    t_asc_dev: torch.Tensor
    a_p_dev: torch.Tensor
    period_dev: torch.Tensor
    tasc_off_dev: torch.Tensor
    ecc_c: float = 0.0      # (e cos w, e sin w) of every template: the ELL1 track; 0, 0 = circular
    ecc_s: float = 0.0

    @classmethod
    def build(cls, spec, t_mid: float, sky, device="cuda", ecc=(0.0, 0.0)) -> "DeviceGrid":
        """Enumerate the grid with bsh_grid_build (host) and upload its tables."""
        a_p, per, off, t_asc = bsh_grid_build(spec, t_mid)
        return cls.from_tables(sky, spec.k0, spec.n_f0, a_p, per, off, t_asc, device, ecc=ecc)

    @classmethod
    def from_tables(cls, sky, k0, n_f0, a_p, per, off, t_asc, device="cuda", ecc=(0.0, 0.0)) -> "DeviceGrid":
        a_p = np.ascontiguousarray(a_p, np.float64)
        per = np.ascontiguousarray(per, np.float64)
        off = np.ascontiguousarray(off, np.int64)
        return cls(sky=_dev(sky, torch.float64, device), k0=int(k0), n_f0=int(n_f0), a_p=a_p, period=per,
                   tasc_off=off, t_asc_dev=_dev(t_asc, torch.float64, device),
                   a_p_dev=_dev(a_p, torch.float64, device), period_dev=_dev(per, torch.float64, device),
                   tasc_off_dev=_dev(off, torch.int64, device), ecc_c=float(ecc[0]), ecc_s=float(ecc[1]))

    def with_ecc(self, ecc_c: float, ecc_s: float) -> "DeviceGrid":
        """The same template tables (shared, not copied) with another eccentricity pair."""
        return dataclasses.replace(self, ecc_c=float(ecc_c), ecc_s=float(ecc_s))

    @property
    def n_sky(self) -> int:
        return int(self.sky.shape[0])

    @property
    def n_bin(self) -> int:
        return int(self.tasc_off[-1])

    @property
    def n_templates(self) -> int:
        return self.n_sky * self.n_bin * self.n_f0

    def struct(self) -> N.Grid:
        return N.Grid(n_sky=self.n_sky, sky=_ptr(self.sky), k0=self.k0, n_f0=self.n_f0,
                      n_ap=int(self.a_p.size), n_per=int(self.period.size), a_p=_ptr(self.a_p_dev),
                      period=_ptr(self.period_dev), tasc_off=_ptr(self.tasc_off_dev),
                      t_asc=_ptr(self.t_asc_dev),
                      a_p_host=self.a_p.ctypes.data, period_host=self.period.ctypes.data,
                      tasc_off_host=self.tasc_off.ctypes.data, ecc_c=self.ecc_c, ecc_s=self.ecc_s)


# ---------------------------------------------------------------- entry points

def bsh_version() -> int:
    return int(N.load().bsh_version())


def bsh_grid_build(spec, t_mid: float):
    """Template bank of one band (host): (a_p, period, tasc_off, t_asc) NumPy arrays.

    ``spec`` has the fields of bsh_grid_spec (e.g. a bsh_synth.GridSpec)."""
    L = N.load()
    cs = N.GridSpec(k0=int(spec.k0), n_f0=int(spec.n_f0), t_coh=float(spec.t_coh),
                    ap_lo=float(spec.ap_lo), ap_hi=float(spec.ap_hi), n_ap=int(spec.n_ap),
                    per_lo=float(spec.per_lo), per_hi=float(spec.per_hi), n_per=int(spec.n_per),
                    tasc_fixed=int(spec.tasc_fixed), tasc_rule_m=float(spec.tasc_rule_m),
                    tasc_min=int(spec.tasc_min), tasc_max=int(spec.tasc_max))
    a_p = np.zeros(spec.n_ap, np.float64)
    per = np.zeros(spec.n_per, np.float64)
    off = np.zeros(spec.n_ap * spec.n_per + 1, np.int64)
    n_bin = ctypes.c_int64(0)
    check(L.bsh_grid_build(ctypes.byref(cs), float(t_mid), a_p.ctypes.data, per.ctypes.data,
                           off.ctypes.data, None, 0, ctypes.byref(n_bin)), "bsh_grid_build")
    t_asc = np.zeros(max(1, n_bin.value), np.float64)
    check(L.bsh_grid_build(ctypes.byref(cs), float(t_mid), a_p.ctypes.data, per.ctypes.data,
                           off.ctypes.data, t_asc.ctypes.data, t_asc.size, ctypes.byref(n_bin)),
          "bsh_grid_build")
    return a_p, per, off, t_asc[:n_bin.value]


def bsh_normalize(raw: torch.Tensor, window: int = 101, out: Optional[torch.Tensor] = None):
    """Normalized power [n_seg, n_raw - window + 1] from raw SFT powers by a running median."""
    assert raw.is_cuda and raw.dtype == torch.float32 and raw.dim() == 2
    raw = raw.contiguous()
    n_seg, n_raw = raw.shape
    if out is None:
        out = torch.empty((n_seg, n_raw - window + 1), dtype=torch.float32, device=raw.device)
    check(N.load().bsh_normalize(_ptr(raw), n_seg, n_raw, int(window), _ptr(out), _stream()), "bsh_normalize")
    return out


def bsh_peakgram(power: torch.Tensor, rho_th: float = 1.6, out: Optional[torch.Tensor] = None):
    """Bit-packed peakgram [n_seg, ceil(n_bins/32)] int32 (bit patterns of uint32 words)."""
    assert power.is_cuda and power.dtype == torch.float32 and power.dim() == 2
    power = power.contiguous()
    n_seg, n_bins = power.shape
    nw = (n_bins + 31) // 32
    if out is None:
        out = torch.empty((n_seg, nw), dtype=torch.int32, device=power.device)
    check(N.load().bsh_peakgram(_ptr(power), n_seg, n_bins, float(rho_th), _ptr(out), _stream()),
          "bsh_peakgram")
    return out


def bsh_hough_count(seg: DeviceSegments, grid: DeviceGrid, with_count: bool = False,
                    status: Optional[Status] = None, wsum_out=None, count_out=None,
                    lanes: int = 0, chunk: int = 0, variant: int = 0):
    """Stage-1 map: (wsum float32 [n_templates], count int32 [n_templates] or None).

    lanes / chunk select the tile shape and variant the accumulation (bsh_hough_count_ex:
    0 auto, 1 select-and-add, 2 subset-sum tables); 0 keeps the defaults."""
    dev = seg.t_mid.device
    if wsum_out is None:
        wsum_out = torch.empty(grid.n_templates, dtype=torch.float32, device=dev)
    if with_count and count_out is None:
        count_out = torch.empty(grid.n_templates, dtype=torch.int32, device=dev)
    s_c, g_c = seg.struct(), grid.struct()
    if lanes or chunk or variant:
        check(N.load().bsh_hough_count_ex(ctypes.byref(s_c), ctypes.byref(g_c), int(lanes or 256),
                                          int(chunk or 256), int(variant), _ptr(count_out), _ptr(wsum_out),
                                          status.ptr() if status else None, _stream()),
              "bsh_hough_count_ex")
    else:
        check(N.load().bsh_hough_count(ctypes.byref(s_c), ctypes.byref(g_c), _ptr(count_out),
                                       _ptr(wsum_out), status.ptr() if status else None, _stream()),
              "bsh_hough_count")
    return wsum_out, (count_out if with_count else None)


def count_window_proven(seg: DeviceSegments, grid: DeviceGrid) -> bool:
    """Whether the table count of (seg, grid) takes the kernel form for host-proven windows."""
    s_c, g_c = seg.struct(), grid.struct()
    rc = int(N.load().bsh_count_window_proven(ctypes.byref(s_c), ctypes.byref(g_c)))
    if rc < 0:
        check(rc, "bsh_count_window_proven")
    return rc == 1


class CountTopK:
    """Reusable workspace for bsh_hough_count_topk (stage 1 with its top-k and bounded memory)."""

    def __init__(self, grid: "DeviceGrid", k: int, sky_per_pass: int = 0, device="cuda"):
        self.k, self.sky_per_pass = int(k), int(sky_per_pass)
        self.spec = N.TopkSpec(k=self.k, sky_per_pass=self.sky_per_pass)
        g_c = grid.struct()
        nbytes = int(N.load().bsh_hough_count_topk_workspace(ctypes.byref(g_c), ctypes.byref(self.spec)))
        if nbytes == 0:
            raise BshError(N.BSH_EINVAL, "bsh_hough_count_topk_workspace", "bad grid or k")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)

    def __call__(self, seg: "DeviceSegments", grid: "DeviceGrid", status: Optional["Status"] = None,
                 out_score=None, out_index=None):
        dev = seg.t_mid.device
        if out_score is None:
            out_score = torch.empty(self.k, dtype=torch.float32, device=dev)
        if out_index is None:
            out_index = torch.empty(self.k, dtype=torch.int64, device=dev)
        s_c, g_c = seg.struct(), grid.struct()
        check(N.load().bsh_hough_count_topk(ctypes.byref(s_c), ctypes.byref(g_c), ctypes.byref(self.spec),
                                            _ptr(out_score), _ptr(out_index), _ptr(self.ws), self.ws.numel(),
                                            status.ptr() if status else None, _stream()),
              "bsh_hough_count_topk")
        return out_score, out_index


def bsh_hough_count_topk(seg: "DeviceSegments", grid: "DeviceGrid", k: int, sky_per_pass: int = 0,
                         status: Optional["Status"] = None):
    """Stage-1 top-k of the grid without its full map: (scores float32 [k], indices int64 [k])."""
    return CountTopK(grid, k, sky_per_pass, seg.t_mid.device)(seg, grid, status)


class TopK:
    """Reusable workspace for bsh_topk."""

    def __init__(self, n: int, k: int, device="cuda"):
        self.n, self.k = int(n), int(k)
        nbytes = int(N.load().bsh_topk_workspace(self.n, self.k))
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)

    def __call__(self, score: torch.Tensor, index: Optional[torch.Tensor] = None,
                 out_score=None, out_index=None):
        n = int(score.numel())
        if n > self.n:
            raise ValueError("more entries than the workspace was sized for")
        dev = score.device
        if out_score is None:
            out_score = torch.empty(self.k, dtype=torch.float32, device=dev)
        if out_index is None:
            out_index = torch.empty(self.k, dtype=torch.int64, device=dev)
        check(N.load().bsh_topk(_ptr(score), _ptr(index), n, self.k, _ptr(out_score), _ptr(out_index),
                                _ptr(self.ws), self.ws.numel(), _stream()), "bsh_topk")
        return out_score, out_index


def bsh_topk(score: torch.Tensor, k: int, index: Optional[torch.Tensor] = None):
    """Exact top-k under (score desc, index asc): (scores float32 [k], indices int64 [k])."""
    assert score.dtype == torch.float32 and score.is_contiguous()
    if index is not None:
        assert index.dtype == torch.int64 and index.numel() == score.numel()
    return TopK(score.numel(), k, score.device)(score, index)


def bsh_topk_segmented(score: torch.Tensor, offsets: np.ndarray, k: int, index: Optional[torch.Tensor] = None,
                       index_shift: int = 0, candidates: bool = True):
    """Independent top-k lists of the segments score[offsets[g] .. offsets[g+1]):
    (scores float32 [n_segs, k], indices int64 [n_segs, k]).  candidates: give the workspace
    that lets long segments take the candidate pass (the same lists)."""
    assert score.dtype == torch.float32 and score.is_contiguous()
    if index is not None:
        assert index.dtype == torch.int64 and index.is_contiguous() and index.numel() == score.numel()
    dev = score.device
    off_h = np.ascontiguousarray(offsets, dtype=np.int64)
    n_segs = off_h.size - 1
    off_d = torch.from_numpy(off_h).to(dev)
    L = N.load()
    wsb = int((L.bsh_topk_segmented_candidate_workspace if candidates else L.bsh_topk_segmented_workspace)(
        n_segs, int(k)))
    ws = torch.empty(max(1, wsb), dtype=torch.uint8, device=dev)
    out_s = torch.empty((n_segs, k), dtype=torch.float32, device=dev)
    out_i = torch.empty((n_segs, k), dtype=torch.int64, device=dev)
    check(L.bsh_topk_segmented(_ptr(score), _ptr(index), _ptr(off_d), off_h.ctypes.data_as(ctypes.c_void_p),
                               n_segs, int(k), int(index_shift), _ptr(out_s), _ptr(out_i), _ptr(ws), wsb,
                               _stream()), "bsh_topk_segmented")
    return out_s, out_i


def bsh_topk_noalloc(score: torch.Tensor, k: int, index: Optional[torch.Tensor] = None,
                     out_score: Optional[torch.Tensor] = None, out_index: Optional[torch.Tensor] = None):
    """bsh_topk through the library's static per-GPU workspace (the library allocates nothing;
    pass out_score / out_index to allocate nothing here either)."""
    assert score.dtype == torch.float32 and score.is_contiguous()
    if index is not None:
        assert index.dtype == torch.int64 and index.is_contiguous() and index.numel() == score.numel()
    dev = score.device
    if out_score is None:
        out_score = torch.empty(k, dtype=torch.float32, device=dev)
    if out_index is None:
        out_index = torch.empty(k, dtype=torch.int64, device=dev)
    assert out_score.numel() >= k and out_index.numel() >= k
    check(N.load().bsh_topk_noalloc(_ptr(score), _ptr(index), int(score.numel()), int(k), _ptr(out_score),
                                    _ptr(out_index), _stream()), "bsh_topk_noalloc")
    return out_score, out_index


def bsh_topk_noalloc_max_bytes() -> int:
    return int(N.load().bsh_topk_noalloc_max_bytes())


def bsh_decode_templates(grid: DeviceGrid, index: torch.Tensor):
    """Stage-1 template indices -> (cand_sky int32 [n], cand_params float64 [n, 4])."""
    n = int(index.numel())
    dev = index.device
    cs = torch.empty(n, dtype=torch.int32, device=dev)
    cp = torch.empty((n, 4), dtype=torch.float64, device=dev)
    g_c = grid.struct()
    check(N.load().bsh_decode_templates(ctypes.byref(g_c), _ptr(index.contiguous()), n, _ptr(cs),
                                        _ptr(cp), _stream()), "bsh_decode_templates")
    return cs, cp


def bsh_power_stat(seg: DeviceSegments, sky: torch.Tensor, cand_sky: torch.Tensor,
                   cand_params: torch.Tensor, mode: int = 0, with_power: bool = True,
                   with_counts: bool = False, status: Optional[Status] = None, out=None):
    """Stage-2 statistic: P float32 [n] (or None), and (count int32, wsum float32) if with_counts."""
    n = int(cand_sky.numel())
    dev = cand_sky.device
    P = (out if out is not None else torch.empty(n, dtype=torch.float32, device=dev)) if with_power else None
    cnt = torch.empty(n, dtype=torch.int32, device=dev) if with_counts else None
    ws = torch.empty(n, dtype=torch.float32, device=dev) if with_counts else None
    s_c = seg.struct()
    check(N.load().bsh_power_stat(ctypes.byref(s_c), _ptr(sky), int(sky.shape[0]), _ptr(cand_sky),
                                  _ptr(cand_params), n, int(mode), _ptr(P), _ptr(cnt), _ptr(ws),
                                  status.ptr() if status else None, _stream()), "bsh_power_stat")
    return (P, cnt, ws) if with_counts else P


def with_ecc_columns(cand_params: torch.Tensor, ecc_c: float, ecc_s: float) -> torch.Tensor:
    """[n, 4] candidate rows (e.g. decoded grid templates) -> [n, 6] rows of one eccentricity pair."""
    n = int(cand_params.shape[0])
    e = torch.tensor([float(ecc_c), float(ecc_s)], dtype=torch.float64, device=cand_params.device)
    return torch.cat([cand_params.to(torch.float64), e.expand(n, 2)], dim=1).contiguous()


def bsh_power_stat_ecc(seg: DeviceSegments, sky: torch.Tensor, cand_sky: torch.Tensor,
                       cand_params: torch.Tensor, mode: int = 0, with_power: bool = True,
                       with_counts: bool = False, status: Optional[Status] = None):
    """Stage-2 statistic on the ELL1 track; cand_params [n, 6] = (F, a_p, P, t_asc, e cos w, e sin w).
    P float32 [n] (or None), and (count int32, wsum float32) if with_counts (mode 0)."""
    n = int(cand_sky.numel())
    dev = cand_sky.device
    P = torch.empty(n, dtype=torch.float32, device=dev) if with_power else None
    cnt = torch.empty(n, dtype=torch.int32, device=dev) if with_counts else None
    ws = torch.empty(n, dtype=torch.float32, device=dev) if with_counts else None
    s_c = seg.struct()
    check(N.load().bsh_power_stat_ecc(ctypes.byref(s_c), _ptr(sky), int(sky.shape[0]), _ptr(cand_sky),
                                      _ptr(cand_params.contiguous()), n, int(mode), _ptr(P), _ptr(cnt), _ptr(ws),
                                      status.ptr() if status else None, _stream()), "bsh_power_stat_ecc")
    if with_counts:
        return P, cnt, ws
    return P


def bsh_power_stat_grad_ecc(seg: DeviceSegments, sky: torch.Tensor, cand_sky: torch.Tensor,
                            cand_params: torch.Tensor, grad_P: Optional[torch.Tensor] = None,
                            with_value: bool = True, status: Optional[Status] = None):
    """(P_lin float32 [n] or None, grad_P * d P_lin / d(F, a_p, P, t_asc, e cos w, e sin w) float64
    [n, 6]) on the ELL1 track, in one pass."""
    n = int(cand_sky.numel())
    dev = cand_sky.device
    P = torch.empty(n, dtype=torch.float32, device=dev) if with_value else None
    out = torch.empty((n, 6), dtype=torch.float64, device=dev)
    gp = None if grad_P is None else grad_P.to(torch.float64).contiguous()
    s_c = seg.struct()
    check(N.load().bsh_power_stat_grad_ecc(ctypes.byref(s_c), _ptr(sky), int(sky.shape[0]), _ptr(cand_sky),
                                           _ptr(cand_params.contiguous()), n, _ptr(gp), _ptr(P), _ptr(out),
                                           status.ptr() if status else None, _stream()),
          "bsh_power_stat_grad_ecc")
    return P, out


def bsh_power_stat_grad(seg: DeviceSegments, sky: torch.Tensor, cand_sky: torch.Tensor,
                        cand_params: torch.Tensor, grad_P: Optional[torch.Tensor] = None,
                        status: Optional[Status] = None):
    """d P_lin / d(F, a_p, P, t_asc), scaled by grad_P: float64 [n, 4]."""
    n = int(cand_sky.numel())
    out = torch.empty((n, 4), dtype=torch.float64, device=cand_sky.device)
    gp = None if grad_P is None else grad_P.to(torch.float64).contiguous()
    s_c = seg.struct()
    check(N.load().bsh_power_stat_grad(ctypes.byref(s_c), _ptr(sky), int(sky.shape[0]), _ptr(cand_sky),
                                       _ptr(cand_params), n, _ptr(gp), _ptr(out),
                                       status.ptr() if status else None, _stream()),
          "bsh_power_stat_grad")
    return out


def bsh_power_stat_value_and_grad(seg: DeviceSegments, sky: torch.Tensor, cand_sky: torch.Tensor,
                                  cand_params: torch.Tensor, grad_P: Optional[torch.Tensor] = None,
                                  status: Optional[Status] = None):
    """(P_lin float32 [n], grad_P * d P_lin / d(F, a_p, P, t_asc) float64 [n, 4]) in one pass."""
    n = int(cand_sky.numel())
    P = torch.empty(n, dtype=torch.float32, device=cand_sky.device)
    out = torch.empty((n, 4), dtype=torch.float64, device=cand_sky.device)
    gp = None if grad_P is None else grad_P.to(torch.float64).contiguous()
    s_c = seg.struct()
    check(N.load().bsh_power_stat_value_and_grad(ctypes.byref(s_c), _ptr(sky), int(sky.shape[0]),
                                                 _ptr(cand_sky), _ptr(cand_params), n, _ptr(gp), _ptr(P),
                                                 _ptr(out), status.ptr() if status else None, _stream()),
          "bsh_power_stat_value_and_grad")
    return P, out


def bsh_track_bins(seg: DeviceSegments, sky: torch.Tensor, cand_sky: torch.Tensor,
                   cand_params: torch.Tensor, status: Optional[Status] = None):
    """Absolute bins of each candidate's track: int32 [n, n_seg]."""
    n = int(cand_sky.numel())
    out = torch.empty((n, seg.n_seg), dtype=torch.int32, device=cand_sky.device)
    s_c = seg.struct()
    check(N.load().bsh_track_bins(ctypes.byref(s_c), _ptr(sky), int(sky.shape[0]), _ptr(cand_sky),
                                  _ptr(cand_params), n, _ptr(out), status.ptr() if status else None,
                                  _stream()), "bsh_track_bins")
    return out


# ---------------------------------------------------------------- post-processing


def post_params(t_coh: float = 900.0, t_obs: float = 86400.0 * 120, m_a: float = 0.4,
                m_omega: float = 0.4, m_t: float = 0.4, pixel_factor: float = 1.0,
                v_over_c: float = 1.0e-4) -> N.PostParams:
    """bsh_post_params: resolutions of the post-processing distance."""
    return N.PostParams(t_coh=t_coh, t_obs=t_obs, m_a=m_a, m_omega=m_omega, m_t=m_t,
                        pixel_factor=pixel_factor, v_over_c=v_over_c)


def bsh_post_rows(sky: torch.Tensor, cand_sky: torch.Tensor, cand_params: torch.Tensor,
                  t_coh: float = 900.0):
    """Rows (f, x, y, a_p, Omega, t_asc) [n, 6] float64 of stage-2 candidates."""
    n = int(cand_sky.numel())
    out = torch.empty((n, 6), dtype=torch.float64, device=cand_sky.device)
    check(N.load().bsh_post_rows(_ptr(sky), _ptr(cand_sky), _ptr(cand_params), n, float(t_coh),
                                 _ptr(out), _stream()), "bsh_post_rows")
    return out


def bsh_significance(score: torch.Tensor, weight: torch.Tensor, kind: int, rho_th: float = 1.6):
    """s_H (kind 0) or s_P (kind 1) of float32 scores: float64 [n]."""
    n = int(score.numel())
    out = torch.empty(n, dtype=torch.float64, device=score.device)
    check(N.load().bsh_significance(_ptr(score), n, _ptr(weight), int(weight.numel()), int(kind),
                                    float(rho_th), _ptr(out), _stream()), "bsh_significance")
    return out


def bsh_coincidences(pp: N.PostParams, rows_a: torch.Tensor, sig_a: torch.Tensor,
                     rows_b: torch.Tensor, sig_b: torch.Tensor, window: float, cap: int):
    """Pairs closer than `window`: (n_pairs device int64 [1], pairs [cap, 2], rows [cap, 6],
    sig [cap]); the first min(n_pairs, cap) rows are valid."""
    L = N.load()
    dev = rows_a.device
    na, nb = int(rows_a.shape[0]), int(rows_b.shape[0])
    ws = torch.empty(max(1, int(L.bsh_coincidences_workspace(na))), dtype=torch.uint8, device=dev)
    pairs = torch.empty((cap, 2), dtype=torch.int64, device=dev)
    rows = torch.empty((cap, 6), dtype=torch.float64, device=dev)
    sig = torch.empty(cap, dtype=torch.float64, device=dev)
    n_pairs = torch.empty(1, dtype=torch.int64, device=dev)
    check(L.bsh_coincidences(ctypes.byref(pp), _ptr(rows_a), _ptr(sig_a), na, _ptr(rows_b), _ptr(sig_b), nb,
                             float(window), int(cap), _ptr(pairs), _ptr(rows), _ptr(sig), _ptr(n_pairs),
                             _ptr(ws), ws.numel(), _stream()), "bsh_coincidences")
    return n_pairs, pairs, rows, sig


def bsh_cluster(pp: N.PostParams, rows: torch.Tensor, window: float):
    """Cluster label (smallest member index) of every row: int32 [n]."""
    n = int(rows.shape[0])
    out = torch.empty(n, dtype=torch.int32, device=rows.device)
    check(N.load().bsh_cluster(ctypes.byref(pp), _ptr(rows), n, float(window), _ptr(out), _stream()),
          "bsh_cluster")
    return out


def bsh_cluster_centroids(pp: N.PostParams, rows: torch.Tensor, sig: torch.Tensor, label: torch.Tensor,
                          cut: float = 0.0, status: Optional[Status] = None):
    """(centroid [n, 6], weight [n], top [n], best [1]) per cluster root (see the C header)."""
    L = N.load()
    n = int(rows.shape[0])
    dev = rows.device
    ws = torch.empty(max(1, int(L.bsh_cluster_centroids_workspace(n))), dtype=torch.uint8, device=dev)
    cen = torch.empty((n, 6), dtype=torch.float64, device=dev)
    weight = torch.empty(n, dtype=torch.float64, device=dev)
    top = torch.empty(n, dtype=torch.int32, device=dev)
    best = torch.empty(1, dtype=torch.int32, device=dev)
    check(L.bsh_cluster_centroids(ctypes.byref(pp), _ptr(rows), _ptr(sig), _ptr(label), n, float(cut),
                                  _ptr(cen), _ptr(weight), _ptr(top), _ptr(best),
                                  status.ptr() if status else None, _ptr(ws), ws.numel(), _stream()),
          "bsh_cluster_centroids")
    return cen, weight, top, best


# ---------------------------------------------------------------- batched plan

ITEM_SHIFT = 40


class Plan:
    """A batched stage-1 run over many items (bsh_plan_create / _run / _run_plain).

    items: sequence of (DeviceSegments, grid index, sky_lo, n_sky, band), ordered by band.
    persistent: True / False for the persistent or one-block-per-unit launch form, None for the
    library's choice (the `persistent` property tells which).
    The plan keeps references to every tensor it points at."""

    def __init__(self, items, grids: Sequence[DeviceGrid], n_bands: int, k_item: int = 0,
                 k_band: int = 0, lanes: int = 0, chunk: int = 0, use_graph: bool = True,
                 lpt: bool = True, blocks: int = 0, variant: int = 0, status: Optional[Status] = None,
                 device="cuda", map_floats: Optional[int] = None, persistent: Optional[bool] = None):
        L = N.load()
        self._keep = [items, grids]
        self.n_items = len(items)
        self.n_bands, self.k_item, self.k_band = int(n_bands), int(k_item), int(k_band)
        self._segs = [it[0].struct() for it in items]
        arr_i = (N.Item * self.n_items)()
        for q, (ds, gi, lo, ns, band) in enumerate(items):
            arr_i[q] = N.Item(seg=self._segs[q], grid=int(gi), sky_lo=int(lo), n_sky=int(ns), band=int(band))
        arr_g = (N.Grid * len(grids))()
        for q, g in enumerate(grids):
            arr_g[q] = g.struct()
        self._arr_i, self._arr_g = arr_i, arr_g
        n_maps = int(L.bsh_items_map_floats(arr_i, self.n_items, arr_g, len(grids)))
        if n_maps < 0:
            raise BshError(N.BSH_EINVAL, "bsh_items_map_floats", "bad items")
        # map_floats below the total runs the items in passes through one reused buffer
        n_buf = n_maps if map_floats is None else min(int(map_floats), n_maps)
        self.maps = torch.empty(max(1, n_buf), dtype=torch.float32, device=device)
        self.item_score = torch.empty((self.n_items, max(1, self.k_item)), dtype=torch.float32, device=device)
        self.item_index = torch.empty((self.n_items, max(1, self.k_item)), dtype=torch.int64, device=device)
        self.band_score = torch.empty((self.n_bands, max(1, self.k_band)), dtype=torch.float32, device=device)
        self.band_index = torch.empty((self.n_bands, max(1, self.k_band)), dtype=torch.int64, device=device)
        self.status = status if status is not None else Status(device)
        opts = N.PlanOpts(lanes=int(lanes), chunk=int(chunk), k_item=self.k_item, k_band=self.k_band,
                          use_graph=int(bool(use_graph)), lpt=int(bool(lpt)), blocks=int(blocks),
                          variant=int(variant), persistent=-1 if persistent is None else int(bool(persistent)))
        h = ctypes.c_void_p()
        check(L.bsh_plan_create(arr_i, self.n_items, arr_g, len(grids), self.n_bands, ctypes.byref(opts),
                                _ptr(self.maps), self.maps.numel(), _ptr(self.item_score),
                                _ptr(self.item_index), _ptr(self.band_score), _ptr(self.band_index),
                                self.status.ptr(), ctypes.byref(h)),
              "bsh_plan_create")
        self.h = h
        self.offsets = np.zeros(self.n_items + 1, np.int64)
        for q, (ds, gi, lo, ns, band) in enumerate(items):
            self.offsets[q + 1] = self.offsets[q] + ns * grids[gi].n_bin * grids[gi].n_f0

    def run(self) -> None:
        check(N.load().bsh_plan_run(self.h, _stream()), "bsh_plan_run")

    def run_plain(self) -> None:
        check(N.load().bsh_plan_run_plain(self.h, _stream()), "bsh_plan_run_plain")

    def run_count(self) -> None:
        check(N.load().bsh_plan_run_count(self.h, _stream()), "bsh_plan_run_count")

    def item_map(self, q: int) -> torch.Tensor:
        if self.passes != 1:
            raise ValueError("the plan runs in passes: only the last pass's maps are kept")
        return self.maps[int(self.offsets[q]):int(self.offsets[q + 1])]

    @property
    def passes(self) -> int:
        return int(N.load().bsh_plan_passes(self.h))

    @property
    def units(self) -> int:
        return int(N.load().bsh_plan_units(self.h))

    @property
    def blocks(self) -> int:
        return int(N.load().bsh_plan_blocks(self.h))

    @property
    def persistent(self) -> bool:
        return int(N.load().bsh_plan_persistent(self.h)) == 1

    @property
    def proven(self) -> bool:
        """The count launches take the table kernel's form for proven windows."""
        return int(N.load().bsh_plan_proven(self.h)) == 1

    def close(self) -> None:
        if getattr(self, "h", None):
            torch.cuda.synchronize()
            h, self.h = self.h, None
            check(N.load().bsh_plan_destroy(h), "bsh_plan_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
