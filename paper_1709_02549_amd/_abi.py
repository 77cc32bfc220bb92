"""ctypes mirror of include/uwb.h (structs, enums, prototypes) and the library loader.

torch is imported before the library is opened so both share one HIP runtime
(the library's libamdhip64 dependency resolves to the copy torch already loaded).
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede loading libuwb.so)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libuwb.so")

UWB_OK, UWB_EINVAL, UWB_ERANGE, UWB_ENOMEM, UWB_EHIP, UWB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
UWB_DAS, UWB_DMAS, UWB_MVDR = 0, 1, 2
MVDR_LOADING = 3.0        # UWB_MVDR_LOADING
MVDR_MAX_WINDOW = 11      # UWB_MVDR_MAX_WINDOW
UWB_MAX_WINDOW = 31
UWB_MAX_SAMPLES = 65536
UWB_MAX_LEVELS = 16
METRICS = {"mean": 0, "var": 1, "eq5": 2, "max": 3, "max_over_mean": 4, "eq5_clamped": 5}
TERMS = {"fixed": 0, "wb": 1}
WALKS = {"per_level": 0, "paper": 1}

c_i32, c_i64, c_f32, c_f64, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.c_void_p


class UwbScan(ctypes.Structure):
    _fields_ = [("n_ant", c_i32), ("n_samp", c_i32), ("ant_pos", c_vp), ("traces", c_vp),
                ("dt", c_f64), ("t0", c_f64), ("v", c_f64)]


class UwbScanBatch(ctypes.Structure):
    _fields_ = [("n_scans", c_i32), ("n_ant", c_i32), ("n_samp", c_i32), ("ant_pos", c_vp), ("traces", c_vp),
                ("params", c_vp), ("v_min", c_f64), ("dt_min", c_f64)]


class UwbGrid(ctypes.Structure):
    _fields_ = [("origin", c_f64 * 3), ("pitch", c_f64 * 3), ("dims", c_i32 * 3)]


class UwbPeak(ctypes.Structure):
    _fields_ = [("index", c_i64), ("value", c_f64), ("value32", c_f32), ("candidates", c_i32)]


class UwbSegmentTree(ctypes.Structure):
    _fields_ = [("beamformer", c_i32), ("walk", c_i32), ("coarse", c_i32), ("decimation", c_i32),
                ("min_tumour", c_f64), ("max_depth", c_i32), ("metric", c_i32), ("term", c_i32),
                ("frame_level", c_f64), ("frame_final", c_f64)]


class UwbSegmentResult(ctypes.Structure):
    _fields_ = [("n_levels", c_i32), ("term_level", c_i32), ("decimation", c_i32), ("n_samples_level0", c_i32),
                ("child", c_i32 * UWB_MAX_LEVELS), ("box", (c_i32 * 6) * (UWB_MAX_LEVELS + 1)),
                ("score", (c_f64 * 8) * UWB_MAX_LEVELS), ("wb", (c_f64 * 2) * (UWB_MAX_LEVELS + 1)),
                ("n_wb", c_i32), ("roi", c_i32 * 6), ("argmax", c_i64), ("peak", c_f64),
                ("voxels_evaluated", c_i64), ("learned_mask", c_i32), ("guard_hits", c_i32)]


class UwbBatchItem(ctypes.Structure):
    _fields_ = [("scan", UwbScan), ("grid", UwbGrid), ("img", c_vp)]


class UwbBatchConfig(ctypes.Structure):
    _fields_ = [("vpl", c_i32), ("wgs_per_cu", c_i32), ("lds_kb", c_i32), ("order", c_i32)]


class UwbGenRecipe(ctypes.Structure):
    _fields_ = [("n_ant", c_i32), ("n_samp", c_i32), ("n_clutter", c_i32), ("v", c_f64), ("dt", c_f64),
                ("t0", c_f64), ("radius", c_f64), ("snr_db", c_f64), ("pulse_f0", c_f64), ("pulse_sigma", c_f64),
                ("pulse_peak", c_f64), ("salt", ctypes.c_uint64)]


# name -> (restype, argtypes)
PROTOTYPES = {
    "uwb_das": (c_i32, [ctypes.POINTER(UwbScan), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp]),
    "uwb_dmas": (c_i32, [ctypes.POINTER(UwbScan), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp]),
    "uwb_das_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp]),
    "uwb_dmas_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp]),
    "uwb_mvdr": (c_i32, [ctypes.POINTER(UwbScan), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp]),
    "uwb_mvdr_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp]),
    "uwb_mvdr_multistatic": (c_i32, [ctypes.POINTER(UwbScan), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp]),
    "uwb_mvdr_multistatic_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_vp,
                                           c_vp]),
    "uwb_das_dmas": (c_i32, [ctypes.POINTER(UwbScan), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp, c_vp]),
    "uwb_das_dmas_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp, c_vp]),
    "uwb_das_dmas_multistatic_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_vp,
                                               c_vp, c_vp]),
    "uwb_das_multistatic": (c_i32, [ctypes.POINTER(UwbScan), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp]),
    "uwb_dmas_multistatic": (c_i32, [ctypes.POINTER(UwbScan), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp]),
    "uwb_das_multistatic_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp]),
    "uwb_dmas_multistatic_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_vp,
                                           c_vp]),
    "uwb_argmax_multistatic": (c_i32, [ctypes.POINTER(UwbScan), ctypes.POINTER(UwbGrid), c_i32, c_i32, c_vp, c_vp,
                                       c_vp, ctypes.c_size_t, c_vp]),
    "uwb_argmax_multistatic_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_i32,
                                             c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "uwb_segment_refine_multistatic": (c_i32, [ctypes.POINTER(UwbScan), ctypes.POINTER(UwbGrid), c_i32,
                                               ctypes.POINTER(UwbSegmentTree), c_vp, c_vp, c_i64, c_vp,
                                               ctypes.c_size_t, c_vp]),
    "uwb_segment_refine_multistatic_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32,
                                                     ctypes.POINTER(UwbSegmentTree), c_vp, c_vp, c_i64, c_vp,
                                                     ctypes.c_size_t, c_vp]),
    "uwb_argmax_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(UwbGrid), c_i32]),
    "uwb_argmax": (c_i32, [ctypes.POINTER(UwbScan), ctypes.POINTER(UwbGrid), c_i32, c_i32, c_vp, c_vp, c_vp,
                           ctypes.c_size_t, c_vp]),
    "uwb_argmax_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_i32, c_vp, c_vp,
                                 c_vp, ctypes.c_size_t, c_vp]),
    "uwb_image_tiles": (c_i64, [ctypes.POINTER(UwbGrid)]),
    "uwb_das_dmas_batch_tilemax": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp,
                                           c_vp, c_vp, c_vp]),
    "uwb_argmax_tilemax_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(UwbGrid), c_i32]),
    "uwb_argmax_batch_tilemax": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_i32, c_vp,
                                         c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "uwb_argmax_batch_noalloc": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_i32,
                                         c_vp, c_vp, c_vp]),
    "uwb_segment_roi_capacity": (c_i64, [ctypes.POINTER(UwbGrid), ctypes.POINTER(UwbSegmentTree)]),
    "uwb_segment_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(UwbGrid), ctypes.POINTER(UwbSegmentTree),
                                                      c_i32]),
    "uwb_segment_refine": (c_i32, [ctypes.POINTER(UwbScan), ctypes.POINTER(UwbGrid), c_i32,
                                   ctypes.POINTER(UwbSegmentTree), c_vp, c_vp, c_i64, c_vp, ctypes.c_size_t, c_vp]),
    "uwb_segment_refine_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32,
                                         ctypes.POINTER(UwbSegmentTree), c_vp, c_vp, c_i64, c_vp, ctypes.c_size_t,
                                         c_vp]),
    "uwb_segment_composite_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32,
                                            ctypes.POINTER(UwbSegmentTree), c_vp, c_vp, c_i64, c_vp,
                                            ctypes.c_size_t, c_vp, c_vp]),
    "uwb_tumour_check_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(UwbGrid), ctypes.POINTER(UwbSegmentTree),
                                                           c_i32, c_i32, c_i32]),
    "uwb_tumour_check_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32,
                                       ctypes.POINTER(UwbSegmentTree), c_i32, c_i32, c_vp, c_vp, c_vp,
                                       ctypes.c_size_t, c_vp]),
    "uwb_batch_plan_create": (c_i32, [ctypes.POINTER(c_vp), ctypes.POINTER(UwbBatchItem), c_i32, c_i32, c_i32,
                                      ctypes.POINTER(UwbBatchConfig)]),
    "uwb_batch_run": (c_i32, [c_vp, c_vp]),
    "uwb_batch_autotune": (c_i32, [c_vp, c_i32, c_vp, ctypes.POINTER(UwbBatchConfig)]),
    "uwb_batch_get_config": (c_i32, [c_vp, ctypes.POINTER(UwbBatchConfig)]),
    "uwb_batch_set_config": (c_i32, [c_vp, ctypes.POINTER(UwbBatchConfig)]),
    "uwb_batch_timestamps": (c_i32, [c_vp, ctypes.POINTER(c_i64), c_vp]),
    "uwb_batch_plan_destroy": (c_i32, [c_vp]),
    "uwb_cnn_param_count": (c_i32, []),
    "uwb_cnn_create": (c_i32, [ctypes.POINTER(c_vp), c_i32, c_vp]),
    "uwb_cnn_destroy": (c_i32, [c_vp]),
    "uwb_cnn_forward": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp]),
    "uwb_cnn_gradients": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "uwb_cnn_train_step": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_f32, c_vp, c_vp]),
    "uwb_cnn_get_state": (c_i32, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(c_i64), c_vp]),
    "uwb_cnn_set_state": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64, c_vp]),
    "uwb_cnn_weights_bf16": (c_vp, [c_vp]),
    "uwb_learned_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(UwbGrid), ctypes.POINTER(UwbSegmentTree),
                                                      c_i32]),
    "uwb_learned_refine_batch": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32,
                                         ctypes.POINTER(UwbSegmentTree), c_vp, c_f32, c_vp, c_vp, c_i64, c_vp,
                                         ctypes.c_size_t, c_vp]),
    "uwb_cnn_input_levels": (c_i32, [ctypes.POINTER(UwbGrid)]),
    "uwb_cnn_training_inputs": (c_i32, [ctypes.POINTER(UwbScanBatch), ctypes.POINTER(UwbGrid), c_i32, c_vp, c_vp,
                                        c_vp, c_vp]),
    "uwb_generate_disc_scans": (c_i32, [ctypes.POINTER(UwbGenRecipe), c_vp, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "uwb_auto_decimation": (c_i32, [c_f64, c_f64]),
    "uwb_probe_lds_read": (c_i32, [c_i32, c_i32, c_i32, ctypes.POINTER(c_f64), ctypes.POINTER(c_f64), c_vp]),
    "uwb_status_string": (ctypes.c_char_p, [c_i32]),
    "uwb_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """The loaded libuwb.so; raises if the HIP library has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -m paper_1709_02549_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


class UwbError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().uwb_status_string(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def check(status: int, where: str) -> None:
    if status != UWB_OK:
        raise UwbError(status, where)
