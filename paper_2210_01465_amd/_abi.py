"""ctypes declarations of the C ABI in include/fl.h.

Loading needs a built ``libfl.so`` (``python -m paper_2210_01465_amd.build``);
there is no fallback.  torch is imported first so that the library binds to
the HIP runtime torch already loaded.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (load torch's HIP runtime before libfl.so)

# FL_LIBRARY selects another build of the engine (for example one compiled
# with different -D options); by default the in-tree libfl.so is used.
LIB_PATH = os.environ.get("FL_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                        "libfl.so")

FL_OK, FL_EINVAL, FL_ENOMEM, FL_EHIP, FL_ENOCONV, FL_EOVERFLOW, FL_EBUSY, FL_ENOTIMPL = (
    0, -1, -2, -3, -4, -5, -6, -7)
STATUS_NAMES = {0: "FL_OK", -1: "FL_EINVAL", -2: "FL_ENOMEM", -3: "FL_EHIP", -4: "FL_ENOCONV",
                -5: "FL_EOVERFLOW", -6: "FL_EBUSY", -7: "FL_ENOTIMPL"}
FL_NB_HAMMING, FL_NB_ADJACENT = 0, 1
FL_STEP_SEPARATE = 1


class fl_space(ctypes.Structure):
    _fields_ = [("n_params", ctypes.c_int32), ("radix", ctypes.POINTER(ctypes.c_int32))]


class fl_params(ctypes.Structure):
    _fields_ = [("damping", ctypes.c_double), ("p", ctypes.c_double), ("tol_l1", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("row_mapping", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class fl_summary(ctypes.Structure):
    _fields_ = [("n_raw", ctypes.c_int64), ("n_valid", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("n_minima", ctypes.c_int64), ("iterations", ctypes.c_int32),
                ("row_mapping", ctypes.c_int32), ("n_slots", ctypes.c_int32),
                ("mask_words", ctypes.c_int32), ("status", ctypes.c_int32),
                ("n_plateau", ctypes.c_int32), ("residual_l1", ctypes.c_double),
                ("f_opt", ctypes.c_double), ("score", ctypes.c_double),
                ("mass_minima", ctypes.c_double), ("mass_near", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class fl_timing(ctypes.Structure):
    _fields_ = [("build_ms", ctypes.c_double), ("pagerank_ms", ctypes.c_double),
                ("iterate_ms", ctypes.c_double), ("score_ms", ctypes.c_double),
                ("iterations", ctypes.c_int32),
                ("launches", ctypes.c_int32), ("sweep_ms", ctypes.c_double),
                ("sweeps_timed", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes); the list of exported entry points of include/fl.h
_P = ctypes.c_void_p
PROTOTYPES = {
    "fl_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P]),
    "fl_destroy": (ctypes.c_int, [_P]),
    "fl_last_error": (ctypes.c_char_p, [_P]),
    "fl_plan_create": (ctypes.c_int, [_P, ctypes.POINTER(fl_space), _P, ctypes.c_int,
                                      ctypes.POINTER(_P), ctypes.POINTER(fl_summary)]),
    "fl_execute": (ctypes.c_int, [_P, _P, ctypes.POINTER(fl_params), _P, _P,
                                  ctypes.POINTER(fl_summary)]),
    "fl_execute_exact": (ctypes.c_int, [_P, _P, ctypes.POINTER(fl_params), _P, _P,
                                  ctypes.POINTER(fl_summary)]),
    "fl_plan_export": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "fl_plan_timing": (ctypes.c_int, [_P, _P, ctypes.POINTER(fl_timing)]),
    "fl_profile": (ctypes.c_int, [_P, ctypes.c_int32]),
    "fl_score_curve": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]),
    "fl_naive_metric": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "fl_plan_destroy": (ctypes.c_int, [_P, _P]),
    "fl_analyze": (ctypes.c_int, [_P, ctypes.POINTER(fl_space), _P, ctypes.c_int,
                                  ctypes.POINTER(fl_params), _P, _P, _P,
                                  ctypes.POINTER(fl_summary)]),
    "fl_analyze_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(fl_space), _P, ctypes.c_int,
                                          ctypes.POINTER(fl_params), _P, _P, _P,
                                          ctypes.POINTER(fl_summary)]),
    "fl_tune": (ctypes.c_int, [_P, _P, ctypes.POINTER(fl_params), ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "fl_bucket_map": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int64)]),
    "fl_batch_create": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "fl_batch_destroy": (ctypes.c_int, [_P, _P]),
    "fl_batch_add": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(fl_params), _P, _P, ctypes.c_int64]),
    "fl_batch_step": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "fl_batch_collect": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(fl_summary), ctypes.POINTER(ctypes.c_int32)]),
    "fl_batch_timing": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64)]),
    "fl_batch_set_graphs": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "fl_batch_set_small": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "fl_analyze_batch": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(fl_space), _P, _P,
                                        ctypes.POINTER(fl_params), _P, _P, ctypes.POINTER(fl_summary)]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2210_01465_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
