"""ctypes declarations of libbsh.so (include/bsh.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BSH_LIBRARY", os.path.join(HERE, "libbsh.so"))

BSH_OK = 0
BSH_EINVAL = -1
BSH_ERANGE = -2
BSH_EHIP = -3
BSH_ENOMEM = -4
STATUS_RANGE = 1
STATUS_MODEL = 2
STATUS_INPUT = 4
MAX_PER = 256
MAX_F0 = 90
MAX_WORDS = 16
VARIANT_AUTO = 0
VARIANT_SELECT = 1
VARIANT_TABLE = 2

_c_i32 = ctypes.c_int32
_c_i64 = ctypes.c_int64
_c_f64 = ctypes.c_double
_vp = ctypes.c_void_p


class Segments(ctypes.Structure):
    _fields_ = [
        ("n_seg", _c_i64),
        ("t_coh", _c_f64),
        ("t_mid", _vp),
        ("v_over_c", _vp),
        ("weight", _vp),
        ("weight_per_sky", _c_i32),
        ("n_bins", _c_i32),
        ("k_lo", _c_i64),
        ("peak_bits", _vp),
        ("power", _vp),
        ("v_max_host", _c_f64),
    ]


class Grid(ctypes.Structure):
    _fields_ = [
        ("n_sky", _c_i32),
        ("sky", _vp),
        ("k0", _c_i64),
        ("n_f0", _c_i32),
        ("n_ap", _c_i32),
        ("n_per", _c_i32),
        ("a_p", _vp),
        ("period", _vp),
        ("tasc_off", _vp),
        ("t_asc", _vp),
        ("a_p_host", _vp),
        ("period_host", _vp),
        ("tasc_off_host", _vp),
        ("ecc_c", _c_f64),
        ("ecc_s", _c_f64),
    ]


class GridSpec(ctypes.Structure):
    _fields_ = [
        ("k0", _c_i64),
        ("n_f0", _c_i32),
        ("t_coh", _c_f64),
        ("ap_lo", _c_f64),
        ("ap_hi", _c_f64),
        ("n_ap", _c_i32),
        ("per_lo", _c_f64),
        ("per_hi", _c_f64),
        ("n_per", _c_i32),
        ("tasc_fixed", _c_i32),
        ("tasc_rule_m", _c_f64),
        ("tasc_min", _c_i32),
        ("tasc_max", _c_i32),
    ]


class Item(ctypes.Structure):
    _fields_ = [
        ("seg", Segments),
        ("grid", _c_i32),
        ("sky_lo", _c_i32),
        ("n_sky", _c_i32),
        ("band", _c_i32),
    ]


class PlanOpts(ctypes.Structure):
    _fields_ = [
        ("lanes", _c_i32),
        ("chunk", _c_i32),
        ("k_item", _c_i32),
        ("k_band", _c_i32),
        ("use_graph", _c_i32),
        ("lpt", _c_i32),
        ("blocks", _c_i32),
        ("variant", _c_i32),
        ("persistent", _c_i32),
    ]


class TopkSpec(ctypes.Structure):
    _fields_ = [
        ("k", _c_i32),
        ("sky_per_pass", _c_i32),
    ]


class PostParams(ctypes.Structure):
    """bsh_post_params: resolutions of the post-processing distance (eq:postdist)."""
    _fields_ = [
        ("t_coh", _c_f64),
        ("t_obs", _c_f64),
        ("m_a", _c_f64),
        ("m_omega", _c_f64),
        ("m_t", _c_f64),
        ("pixel_factor", _c_f64),
        ("v_over_c", _c_f64),
    ]


# name -> (restype, argtypes); the complete exported surface of include/bsh.h
SIGNATURES = {
    "bsh_version": (ctypes.c_int, []),
    "bsh_last_error": (ctypes.c_char_p, []),
    "bsh_grid_build": (ctypes.c_int, [ctypes.POINTER(GridSpec), _c_f64, _vp, _vp, _vp, _vp, _c_i64,
                                      ctypes.POINTER(_c_i64)]),
    "bsh_normalize": (ctypes.c_int, [_vp, _c_i64, _c_i32, _c_i32, _vp, _vp]),
    "bsh_peakgram": (ctypes.c_int, [_vp, _c_i64, _c_i32, _c_f64, _vp, _vp]),
    "bsh_hough_count": (ctypes.c_int, [ctypes.POINTER(Segments), ctypes.POINTER(Grid), _vp, _vp, _vp,
                                       _vp]),
    "bsh_hough_count_ex": (ctypes.c_int, [ctypes.POINTER(Segments), ctypes.POINTER(Grid), _c_i32, _c_i32,
                                          _c_i32, _vp, _vp, _vp, _vp]),
    "bsh_hough_count_topk_workspace": (ctypes.c_size_t, [ctypes.POINTER(Grid), ctypes.POINTER(TopkSpec)]),
    "bsh_hough_count_topk": (ctypes.c_int, [ctypes.POINTER(Segments), ctypes.POINTER(Grid),
                                            ctypes.POINTER(TopkSpec), _vp, _vp, _vp, ctypes.c_size_t, _vp,
                                            _vp]),
    "bsh_items_map_floats": (_c_i64, [ctypes.POINTER(Item), _c_i32, ctypes.POINTER(Grid), _c_i32]),
    "bsh_plan_create": (ctypes.c_int, [ctypes.POINTER(Item), _c_i32, ctypes.POINTER(Grid), _c_i32, _c_i32,
                                       ctypes.POINTER(PlanOpts), _vp, _c_i64, _vp, _vp, _vp, _vp, _vp,
                                       ctypes.POINTER(_vp)]),
    "bsh_plan_run": (ctypes.c_int, [_vp, _vp]),
    "bsh_plan_run_plain": (ctypes.c_int, [_vp, _vp]),
    "bsh_plan_run_count": (ctypes.c_int, [_vp, _vp]),
    "bsh_plan_units": (_c_i64, [_vp]),
    "bsh_plan_blocks": (_c_i32, [_vp]),
    "bsh_plan_persistent": (_c_i32, [_vp]),
    "bsh_plan_proven": (_c_i32, [_vp]),
    "bsh_count_window_proven": (_c_i32, [_vp, _vp]),
    "bsh_plan_passes": (_c_i32, [_vp]),
    "bsh_plan_destroy": (ctypes.c_int, [_vp]),
    "bsh_topk_workspace": (ctypes.c_size_t, [_c_i64, _c_i32]),
    "bsh_topk": (ctypes.c_int, [_vp, _vp, _c_i64, _c_i32, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "bsh_topk_noalloc_max_bytes": (ctypes.c_size_t, []),
    "bsh_topk_noalloc": (ctypes.c_int, [_vp, _vp, _c_i64, _c_i32, _vp, _vp, _vp]),
    "bsh_topk_segmented_workspace": (ctypes.c_size_t, [_c_i32, _c_i32]),
    "bsh_topk_segmented_candidate_workspace": (ctypes.c_size_t, [_c_i32, _c_i32]),
    "bsh_topk_segmented": (ctypes.c_int, [_vp, _vp, _vp, _vp, _c_i32, _c_i32, _c_i32, _vp, _vp, _vp,
                                          ctypes.c_size_t, _vp]),
    "bsh_decode_templates": (ctypes.c_int, [ctypes.POINTER(Grid), _vp, _c_i64, _vp, _vp, _vp]),
    "bsh_power_stat": (ctypes.c_int, [ctypes.POINTER(Segments), _vp, _c_i32, _vp, _vp, _c_i64, _c_i32,
                                      _vp, _vp, _vp, _vp, _vp]),
    "bsh_power_stat_ecc": (ctypes.c_int, [ctypes.POINTER(Segments), _vp, _c_i32, _vp, _vp, _c_i64, _c_i32,
                                          _vp, _vp, _vp, _vp, _vp]),
    "bsh_power_stat_grad_ecc": (ctypes.c_int, [ctypes.POINTER(Segments), _vp, _c_i32, _vp, _vp, _c_i64, _vp,
                                               _vp, _vp, _vp, _vp]),
    "bsh_power_stat_grad": (ctypes.c_int, [ctypes.POINTER(Segments), _vp, _c_i32, _vp, _vp, _c_i64,
                                           _vp, _vp, _vp, _vp]),
    "bsh_power_stat_value_and_grad": (ctypes.c_int, [ctypes.POINTER(Segments), _vp, _c_i32, _vp, _vp,
                                                     _c_i64, _vp, _vp, _vp, _vp, _vp]),
    "bsh_post_rows": (ctypes.c_int, [_vp, _vp, _vp, _c_i64, _c_f64, _vp, _vp]),
    "bsh_significance": (ctypes.c_int, [_vp, _c_i64, _vp, _c_i64, _c_i32, _c_f64, _vp, _vp]),
    "bsh_coincidences_workspace": (ctypes.c_size_t, [_c_i64]),
    "bsh_coincidences": (ctypes.c_int, [ctypes.POINTER(PostParams), _vp, _vp, _c_i64, _vp, _vp, _c_i64,
                                        _c_f64, _c_i64, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "bsh_cluster": (ctypes.c_int, [ctypes.POINTER(PostParams), _vp, _c_i64, _c_f64, _vp, _vp]),
    "bsh_cluster_centroids_workspace": (ctypes.c_size_t, [_c_i64]),
    "bsh_cluster_centroids": (ctypes.c_int, [ctypes.POINTER(PostParams), _vp, _vp, _vp, _c_i64, _c_f64,
                                             _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "bsh_track_bins": (ctypes.c_int, [ctypes.POINTER(Segments), _vp, _c_i32, _vp, _vp, _c_i64, _vp,
                                      _vp, _vp]),
}

_lib = None


class BshError(RuntimeError):
    def __init__(self, code: int, where: str, text: str):
        super().__init__(f"{where} failed with code {code}: {text}")
        self.code = code


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libbsh.so.  There is no fallback: a missing library is an error."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run paper_1904_04873_amd.build.build() first")
        L = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int, where: str) -> None:
    if rc != BSH_OK:
        text = load().bsh_last_error()
        raise BshError(rc, where, text.decode() if text else "")
