"""Seeded synthetic inputs for the semi-coherent binary Hough search.

This module only draws and lays out input data: segment time stamps, the
detector velocity table, normalized powers, segment weights, sky pixels and
the numeric ranges of each template grid.  It holds none of the search's own
arithmetic (no frequency track, no bin selection, no thresholding, no grid
enumeration), so that the CPU oracle and the GPU library can both consume the
same inputs without sharing any method code.

Conventions (stated once, used by both sides):

* Times are seconds from the start of the first coherent slot; a segment's
  time stamp is its mid-time (start + Tc/2), matching the weights being
  evaluated at SFT mid-time (Sec. IV.A of the paper).
* Normalized powers follow the Gaussian-noise law p(rho) = exp(-rho)
  (Sec. V.F, cost model), i.e. Exp(1) draws.
* Weights are log-normal and normalized to mean 1 (the commented weight
  normalization of Sec. IV.A).
* The velocity table is a closed-form stand-in for the detector ephemeris:
  an annual circular orbit of |v|/c = 1e-4 plus a sidereal rotation of
  1.5e-6 tilted by the obliquity; the paper uses real ephemerides that are
  not available here.
* An injected signal turns the power at one bin per segment into a
  non-central chi-square draw with two degrees of freedom, halved, with
  mean 1 + SNR.  The bins are supplied by the caller.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

T_COH = 900.0                    # coherent time of one SFT (s), Sec. V.A
DAY = 86400.0
YEAR = 365.25 * DAY
SIDEREAL_DAY = 86164.0905
OBLIQUITY = 0.409093             # rad
RHO_TH = 1.6                     # peak threshold, Sec. IV.A
V_ORBIT = 1.0e-4                 # |v|/c of the annual orbit
V_SPIN = 1.5e-6                  # |v|/c of the sidereal rotation
DETECTOR_PHASE = (0.0, 2.0)      # sidereal phase offset per detector (rad)
SEED_BASE = 190404873

STREAMS = ("timestamps", "powers", "weights", "injections", "candidates")


def rng_streams(config_id: int) -> dict:
    """Independent generators for one configuration, keyed by purpose."""
    ss = np.random.SeedSequence(SEED_BASE + int(config_id))
    kids = ss.spawn(len(STREAMS))
    return {name: np.random.default_rng(k) for name, k in zip(STREAMS, kids)}


# --------------------------------------------------------------------------
# detector motion and sky
# --------------------------------------------------------------------------

def velocity_over_c(t: np.ndarray, detector: int = 0) -> np.ndarray:
    """Closed-form detector velocity / c at times t (s); returns [n, 3] float64."""
    t = np.asarray(t, dtype=np.float64)
    py = 2.0 * math.pi * t / YEAR
    pd = 2.0 * math.pi * t / SIDEREAL_DAY + DETECTOR_PHASE[detector]
    out = np.empty((t.size, 3), dtype=np.float64)
    ce, se = math.cos(OBLIQUITY), math.sin(OBLIQUITY)
    rx, ry = -np.sin(pd), np.cos(pd)
    out[:, 0] = V_ORBIT * (-np.sin(py)) + V_SPIN * rx
    out[:, 1] = V_ORBIT * np.cos(py) + V_SPIN * ry * ce
    out[:, 2] = V_SPIN * ry * se
    return out


def fixed_pixel() -> np.ndarray:
    """The single sky pixel of the one-pixel workloads, [1, 3] float64."""
    a, b = 0.3, 1.0
    return np.array([[math.cos(a) * math.cos(b), math.cos(a) * math.sin(b), math.sin(a)]],
                    dtype=np.float64)


def fibonacci_sphere(n: int) -> np.ndarray:
    """n nearly uniform unit vectors, [n, 3] float64."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


# --------------------------------------------------------------------------
# segments
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Segments:
    """Host copy of one work item's per-segment inputs."""
    t_mid: np.ndarray          # [N] float64, seconds
    v_over_c: np.ndarray       # [N, 3] float64
    weight: np.ndarray         # [N] float32 (or [n_sky, N])
    power: np.ndarray          # [N, n_bins] float32 normalized power
    k_lo: int                  # absolute bin of column 0
    n_bins: int
    t_coh: float = T_COH
    detector: Optional[np.ndarray] = None   # [N] int8

    @property
    def n_seg(self) -> int:
        return int(self.t_mid.size)

    def t_span_mid(self) -> float:
        """Middle of the observation: (first start + last end) / 2."""
        if self.n_seg == 0:
            return 0.0
        first = float(self.t_mid.min()) - 0.5 * self.t_coh
        last = float(self.t_mid.max()) + 0.5 * self.t_coh
        return 0.5 * (first + last)


def even_starts(n: int, span_s: float, t_coh: float = T_COH) -> np.ndarray:
    """n segment start times evenly spaced so the last one ends at span_s."""
    if n == 1:
        return np.zeros(1)
    return np.arange(n, dtype=np.float64) * ((span_s - t_coh) / (n - 1))


def gapped_starts(rng: np.random.Generator, n_pick: int, n_slots: int,
                  t_coh: float = T_COH) -> np.ndarray:
    """Starts of n_pick distinct contiguous Tc slots drawn at random, sorted."""
    slots = np.sort(rng.choice(n_slots, size=n_pick, replace=False))
    return slots.astype(np.float64) * t_coh


def lognormal_weights(rng: np.random.Generator, n: int, sigma: float = 0.3) -> np.ndarray:
    w = np.exp(sigma * rng.standard_normal(n))
    w = w / w.mean()
    return w.astype(np.float32)


def exp1_powers(rng: np.random.Generator, n_seg: int, n_bins: int) -> np.ndarray:
    return rng.standard_exponential((n_seg, n_bins), dtype=np.float32)


def raw_sft_powers(rng: np.random.Generator, n_seg: int, n_raw: int, k_first: int,
                   level_spread: float = 0.5) -> np.ndarray:
    """Un-normalized SFT powers |x_k|^2 [n_seg, n_raw] float32: Exp(1) draws times a noise floor
    that varies smoothly with frequency and from segment to segment (a stand-in for
    (Tc/2) S_n(f) of each SFT)."""
    k = np.arange(n_raw, dtype=np.float64) + k_first
    seg_level = np.exp(level_spread * rng.standard_normal(n_seg))[:, None]
    shape = 1.0 + 0.3 * np.sin(2 * np.pi * k / 173.0) + 0.1 * np.cos(2 * np.pi * k / 31.0)
    floor = 1e-3 * seg_level * shape[None, :]
    return (floor * rng.standard_exponential((n_seg, n_raw))).astype(np.float32)


def inject(power: np.ndarray, rng: np.random.Generator, cols_list: Sequence[np.ndarray],
           snrs: Sequence[float]) -> None:
    """Add signals in place.

    Signal q occupies column cols_list[q][J] (bin - k_lo) in segment J, as
    computed by the caller from a frequency track; negative entries are
    skipped.  Signals landing on the same bin add their SNRs.  Every touched
    bin is redrawn as ((X + sqrt(2 snr))^2 + Y^2) / 2 with X, Y ~ N(0, 1):
    Exp(1) for snr = 0, mean 1 + snr.
    """
    snr_map = np.zeros(power.shape, dtype=np.float64)
    for cols, snr in zip(cols_list, snrs):
        cols = np.asarray(cols)
        rows = np.nonzero(cols >= 0)[0]
        np.add.at(snr_map, (rows, cols[rows]), float(snr))
    r, c = np.nonzero(snr_map)
    x = rng.standard_normal(r.size) + np.sqrt(2.0 * snr_map[r, c])
    y = rng.standard_normal(r.size)
    power[r, c] = (0.5 * (x * x + y * y)).astype(np.float32)


# --------------------------------------------------------------------------
# grid ranges (numbers only: enumeration belongs to the search itself)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class GridSpec:
    """Numeric ranges of one band's template grid.

    t_asc points per (a_p, P) cell are either a fixed number or follow the
    spacing rule with the constant ``tasc_rule_m`` and the clamp
    [tasc_min, tasc_max]; f_hi is the band's upper edge in Hz.
    """
    k0: int
    n_f0: int
    ap_lo: float
    ap_hi: float
    n_ap: int
    per_lo: float
    per_hi: float
    n_per: int
    tasc_fixed: int = 0
    tasc_rule_m: float = 60.0
    tasc_min: int = 4
    tasc_max: int = 256
    t_coh: float = T_COH

    @property
    def f_hi(self) -> float:
        return (self.k0 + self.n_f0) / self.t_coh


def band_window(k0: int, n_f0: int, margin: int) -> Tuple[int, int]:
    """Staged row for a band: (k_lo, n_bins) with `margin` bins on each side."""
    return k0 - margin, n_f0 + 2 * margin


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    config_id: int
    segments: List[Segments]
    sky: np.ndarray                  # [n_sky, 3]
    grids: List[GridSpec]            # one per band (items map to one grid)
    item_grid: List[int]             # grid index of each work item
    item_segments: List[int]         # segment-set index of each work item
    item_sky: List[Tuple[int, int]]  # sky pixel range [lo, hi) of each item
    topk_stage1: int = 0
    topk_stage2: int = 0
    rng: Optional[dict] = None


def _segments(t_start: np.ndarray, det: np.ndarray, weights: np.ndarray,
              rng_pow: np.random.Generator, k_lo: int, n_bins: int) -> Segments:
    t_mid = t_start + 0.5 * T_COH
    v = np.empty((t_mid.size, 3))
    for d in (0, 1):
        m = det == d
        if m.any():
            v[m] = velocity_over_c(t_mid[m], d)
    return Segments(t_mid=t_mid, v_over_c=v, weight=weights,
                    power=exp1_powers(rng_pow, t_mid.size, n_bins),
                    k_lo=k_lo, n_bins=n_bins, detector=det.astype(np.int8))


def half_shifted(seg: Segments, rng: np.random.Generator, sigma: float = 0.3) -> Segments:
    """The Tc/2-shifted companion of a gapped segment set: one segment starting half a Tc after
    each segment whose next Tc slot of the same detector is also filled (so it lies inside
    contiguous data).  Powers are fresh Exp(1) draws over the same row (the correlation between
    overlapping segments is not modelled) and weights fresh log-normal draws of mean 1."""
    det = seg.detector if seg.detector is not None else np.zeros(seg.n_seg, np.int8)
    start = seg.t_mid - 0.5 * seg.t_coh
    keep = []
    for d in np.unique(det):
        idx = np.nonzero(det == d)[0]
        idx = idx[np.argsort(start[idx], kind="stable")]
        nxt = np.isclose(np.diff(start[idx]), seg.t_coh, rtol=0, atol=1e-6)
        keep.append(idx[:-1][nxt])
    keep = np.sort(np.concatenate(keep)) if keep else np.zeros(0, np.int64)
    t_mid = seg.t_mid[keep] + 0.5 * seg.t_coh
    d = det[keep]
    v = np.empty((t_mid.size, 3))
    for dd in np.unique(d):
        m = d == dd
        v[m] = velocity_over_c(t_mid[m], int(dd))
    return Segments(t_mid=t_mid, v_over_c=v, weight=lognormal_weights(rng, t_mid.size, sigma),
                    power=exp1_powers(rng, t_mid.size, seg.n_bins), k_lo=seg.k_lo, n_bins=seg.n_bins,
                    t_coh=seg.t_coh, detector=d.astype(np.int8))


def concat_segments(a: Segments, b: Segments) -> Segments:
    """One table holding the segments of a followed by those of b (same row window)."""
    assert a.k_lo == b.k_lo and a.n_bins == b.n_bins and a.t_coh == b.t_coh
    det = None
    if a.detector is not None and b.detector is not None:
        det = np.concatenate([a.detector, b.detector])
    return Segments(t_mid=np.concatenate([a.t_mid, b.t_mid]),
                    v_over_c=np.concatenate([a.v_over_c, b.v_over_c]),
                    weight=np.concatenate([a.weight, b.weight]),
                    power=np.concatenate([a.power, b.power]), k_lo=a.k_lo, n_bins=a.n_bins,
                    t_coh=a.t_coh, detector=det)


def two_detector_starts(rng: np.random.Generator, n_per_det: Sequence[int],
                        n_slots: int) -> Tuple[np.ndarray, np.ndarray]:
    starts, det = [], []
    for d, n in enumerate(n_per_det):
        s = gapped_starts(rng, n, n_slots)
        starts.append(s)
        det.append(np.full(s.size, d, dtype=np.int8))
    return np.concatenate(starts), np.concatenate(det)


def config1() -> Workload:
    """64 evenly spaced segments over 120 d, one pixel, 100.0-100.1 Hz, 8x8x8 binary grid."""
    rng = rng_streams(1)
    k0, nf = 90000, 90
    k_lo, n_bins = band_window(k0, nf, 12)
    t0 = even_starts(64, 120 * DAY)
    seg = _segments(t0, np.zeros(64, np.int8), np.ones(64, np.float32),
                    rng["powers"], k_lo, n_bins)
    g = GridSpec(k0=k0, n_f0=nf, ap_lo=0.01, ap_hi=3.0, n_ap=8,
                 per_lo=15 * DAY, per_hi=45 * DAY, n_per=8, tasc_fixed=8)
    return Workload("cfg1_plain_tiny", 1, [seg], fixed_pixel(), [g], [0], [0], [(0, 1)],
                    topk_stage1=100, rng=rng)


def config2(n_per_det: int = 2000) -> Workload:
    """2 x 2000 gapped segments over ~29.8 d, one pixel, 200.0-200.1 Hz, 64x32x64 grid."""
    rng = rng_streams(2)
    k0, nf = 180000, 90
    k_lo, n_bins = band_window(k0, nf, 22)
    t0, det = two_detector_starts(rng["timestamps"], (n_per_det, n_per_det), 2858)
    w = lognormal_weights(rng["weights"], t0.size)
    seg = _segments(t0, det, w, rng["powers"], k_lo, n_bins)
    g = GridSpec(k0=k0, n_f0=nf, ap_lo=0.01, ap_hi=3.0, n_ap=64,
                 per_lo=15 * DAY, per_hi=45 * DAY, n_per=32, tasc_fixed=64)
    return Workload("cfg2_band_200Hz", 2, [seg], fixed_pixel(), [g], [0], [0], [(0, 1)],
                    topk_stage1=10000, topk_stage2=100, rng=rng)


CFG3_BANDS = (100.0, 166.6, 233.2, 299.8)
CFG3_MARGINS = (12, 19, 26, 33)


def config3(n_patches: int = 256, bands: Sequence[float] = CFG3_BANDS,
            build_items: Optional[Sequence[int]] = None) -> Workload:
    """256 one-pixel patches x 4 bands; per-item gapped segment sets of 1500-3000 per detector
    (each detector fills 70 % of ceil(max count / 0.7) contiguous Tc slots).

    Items are ordered band-major (item = band * n_patches + patch).  With
    ``build_items`` only those items get segment data (the others are left
    as None) so a small sample can be drawn without materializing all.
    """
    rng = rng_streams(3)
    sky = fibonacci_sphere(n_patches)
    grids, items_g, items_sky = [], [], []
    for bi, f_lo in enumerate(bands):
        k0 = int(round(f_lo * T_COH))
        grids.append(GridSpec(k0=k0, n_f0=90, ap_lo=0.003, ap_hi=3.25, n_ap=64,
                              per_lo=15 * DAY, per_hi=45 * DAY, n_per=32))
    n_items = len(bands) * n_patches
    counts = rng["timestamps"].integers(1500, 3001, size=(n_items, 2))
    seeds = rng["powers"].integers(0, 2**63 - 1, size=n_items)
    segs: List[Optional[Segments]] = []
    want = set(range(n_items)) if build_items is None else set(build_items)
    for it in range(n_items):
        bi, p = divmod(it, n_patches)
        items_g.append(bi)
        items_sky.append((p, p + 1))
        if it not in want:
            segs.append(None)
            continue
        r = np.random.default_rng(seeds[it])
        # the 70 % duty factor of config 2, with enough Tc slots for the larger detector
        n_slots = int(math.ceil(max(int(c) for c in counts[it]) / 0.7))
        t0, det = two_detector_starts(r, tuple(int(c) for c in counts[it]), n_slots)
        w = lognormal_weights(r, t0.size)
        k_lo, n_bins = band_window(grids[bi].k0, 90, CFG3_MARGINS[bi])
        segs.append(_segments(t0, det, w, r, k_lo, n_bins))
    return Workload("cfg3_batched_256x4", 3, segs, sky, grids, items_g,
                    list(range(n_items)), items_sky, topk_stage1=1000, rng=rng)


def config4() -> Workload:
    """Config-2 data layout for the differentiable stage 2 (candidates drawn by the caller)."""
    w = config2()
    w.name, w.config_id, w.rng = "cfg4_refine", 4, rng_streams(4)
    seg = w.segments[0]
    r = w.rng
    t0, det = two_detector_starts(r["timestamps"], (2000, 2000), 2858)
    wt = lognormal_weights(r["weights"], t0.size)
    w.segments = [_segments(t0, det, wt, r["powers"], seg.k_lo, seg.n_bins)]
    w.topk_stage1, w.topk_stage2 = 0, 0
    return w


def config5(n_pixels: int = 2000, n_per_det: int = 4000) -> Workload:
    """2 x 4000 segments over 240 d, 2000 pixels, 300.0-300.1 Hz, 128 x 64 x rule-t_asc grid."""
    rng = rng_streams(5)
    k0, nf = 270000, 90
    k_lo, n_bins = band_window(k0, nf, 33)
    t0, det = two_detector_starts(rng["timestamps"], (n_per_det, n_per_det), 23040)
    w = lognormal_weights(rng["weights"], t0.size)
    seg = _segments(t0, det, w, rng["powers"], k_lo, n_bins)
    g = GridSpec(k0=k0, n_f0=nf, ap_lo=0.003, ap_hi=3.25, n_ap=128,
                 per_lo=15 * DAY, per_hi=45 * DAY, n_per=64)
    sky = fibonacci_sphere(n_pixels)
    return Workload("cfg5_allsky_slice", 5, [seg], sky, [g], [0] * n_pixels, [0] * n_pixels,
                    [(p, p + 1) for p in range(n_pixels)], topk_stage1=100000,
                    topk_stage2=5000, rng=rng)


def tiny_segments(n_seg: int = 4, k0: int = 1000, n_f0: int = 3, margin: int = 4,
                  seed: int = 7, span_days: float = 30.0) -> Segments:
    """A very small segment set for brute-force checks."""
    rng = np.random.default_rng(seed)
    t0 = np.sort(rng.uniform(0, span_days * DAY - T_COH, n_seg))
    k_lo, n_bins = band_window(k0, n_f0, margin)
    return Segments(t_mid=t0 + 0.5 * T_COH, v_over_c=velocity_over_c(t0 + 0.5 * T_COH),
                    weight=lognormal_weights(rng, n_seg),
                    power=exp1_powers(rng, n_seg, n_bins), k_lo=k_lo, n_bins=n_bins)
