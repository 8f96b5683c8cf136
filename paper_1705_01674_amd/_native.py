"""ctypes binding of the C ABI in ``include/sgwls.h`` (argument marshalling only).

Loads the in-tree ``libsgwls.so``.  There is no fallback: if the library is
missing or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsgwls.so")

STATUS = {0: "SGWLS_OK", 1: "SGWLS_E_ARG", 2: "SGWLS_E_SHAPE", 3: "SGWLS_E_WORKSPACE",
          4: "SGWLS_E_UNSUPPORTED", 5: "SGWLS_E_HIP"}

# Every symbol include/sgwls.h declares.
EXPORTS = ["sgwls_status_str", "sgwls_version", "sgwls_validate", "sgwls_workspace_bytes",
           "sgwls_pass", "sgwls_pass_stages", "sgwls_filter", "sgwls_backward",
           "sgwls_pass_backward", "sgwls_backward_workspace_bytes",
           "sgwls_batched_workspace_bytes", "sgwls_filter_batched", "sgwls_variant_count",
           "sgwls_tune_pin", "sgwls_tune_query", "sgwls_tune_clear", "sgwls_tune_size",
           "sgwls_autotune", "sgwls_tune_save", "sgwls_tune_load",
           "sgwls_batched_variant_count", "sgwls_filter_batched_variant",
           "sgwls_autotune_batched", "sgwls_batched_graph_count", "sgwls_batched_graph_clear",
           "sgwls_interpolate_workspace_bytes", "sgwls_interpolate",
           "sgwls_wls2d_workspace_bytes", "sgwls_wls2d", "sgwls_resolve_precision",
           "sgwls_filter_noalloc", "sgwls_filter_status", "sgwls_workspace_bytes_nchw",
           "sgwls_filter_nchw",
           "sgwls_backward_workspace_bytes_nchw", "sgwls_backward_nchw",
           "sgwls_separator_bytes_nchw", "sgwls_filter_nchw_seps", "sgwls_backward_nchw_seps"]


class SgwlsParams(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_float), ("r", ctypes.c_int), ("iters", ctypes.c_int),
                ("stride", ctypes.c_int), ("kind", ctypes.c_int),
                ("sigma_s", ctypes.c_float), ("sigma_r", ctypes.c_float),
                ("alpha_s", ctypes.c_float), ("alpha_r", ctypes.c_float),
                ("eps", ctypes.c_float), ("prec", ctypes.c_int)]


class SgwlsImage(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p), ("g", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("C", ctypes.c_int), ("M", ctypes.c_int), ("N", ctypes.c_int)]


class SgwlsError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"SG-WLS HIP library not built: {LIB_PATH} is missing "
                          "(run paper_1705_01674_amd/build.py or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i, P = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(SgwlsParams)
    lib.sgwls_status_str.restype = ctypes.c_char_p
    lib.sgwls_status_str.argtypes = [i]
    lib.sgwls_version.restype = i
    lib.sgwls_validate.restype = i
    lib.sgwls_validate.argtypes = [i, i, i, P]
    lib.sgwls_workspace_bytes.restype = sz
    lib.sgwls_workspace_bytes.argtypes = [i, i, i, P, i]
    lib.sgwls_resolve_precision.restype = i
    lib.sgwls_resolve_precision.argtypes = [P, i]
    lib.sgwls_workspace_bytes_nchw.restype = sz
    lib.sgwls_workspace_bytes_nchw.argtypes = [i, i, i, i, P, i]
    lib.sgwls_filter_nchw.restype = i
    lib.sgwls_filter_nchw.argtypes = [vp, vp, vp, i, i, i, i, P, vp, vp, vp, sz, vp]
    lib.sgwls_backward_workspace_bytes_nchw.restype = sz
    lib.sgwls_backward_workspace_bytes_nchw.argtypes = [i, i, i, i, P]
    lib.sgwls_backward_nchw.restype = i
    lib.sgwls_backward_nchw.argtypes = [vp, vp, vp, vp, vp, vp, i, i, i, i, P, vp, vp, sz, vp]
    lib.sgwls_separator_bytes_nchw.restype = sz
    lib.sgwls_separator_bytes_nchw.argtypes = [i, i, i, i, P]
    lib.sgwls_filter_nchw_seps.restype = i
    lib.sgwls_filter_nchw_seps.argtypes = [vp, vp, vp, i, i, i, i, P, vp, vp, vp, sz, vp, sz, vp]
    lib.sgwls_backward_nchw_seps.restype = i
    lib.sgwls_backward_nchw_seps.argtypes = [vp, vp, vp, vp, sz, vp, vp, vp, vp, i, i, i, i, P,
                                             vp, vp, sz, vp]
    lib.sgwls_filter_noalloc.restype = i
    lib.sgwls_filter_noalloc.argtypes = [vp, vp, vp, i, i, i, P, vp, vp, vp]
    lib.sgwls_filter_status.restype = i
    lib.sgwls_filter_status.argtypes = [vp, vp]
    lib.sgwls_pass.restype = i
    lib.sgwls_pass.argtypes = [i, vp, vp, vp, i, i, i, P, vp, vp, sz, vp]
    lib.sgwls_pass_stages.restype = i
    lib.sgwls_pass_stages.argtypes = [i, i, vp, vp, vp, i, i, i, P, vp, vp, sz, vp]
    lib.sgwls_filter.restype = i
    lib.sgwls_filter.argtypes = [vp, vp, vp, i, i, i, P, vp, vp, vp, sz, vp]
    lib.sgwls_interpolate_workspace_bytes.restype = sz
    lib.sgwls_interpolate_workspace_bytes.argtypes = [i, i, i, P]
    lib.sgwls_interpolate.restype = i
    lib.sgwls_interpolate.argtypes = [vp, vp, vp, vp, i, i, i, P, vp, vp, sz, vp]
    lib.sgwls_wls2d_workspace_bytes.restype = sz
    lib.sgwls_wls2d_workspace_bytes.argtypes = [i, i, i, P]
    lib.sgwls_wls2d.restype = i
    lib.sgwls_wls2d.argtypes = [vp, vp, vp, i, i, i, P, i, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                vp, sz, vp]
    lib.sgwls_backward.restype = i
    lib.sgwls_backward.argtypes = [vp, vp, vp, vp, vp, vp, i, i, i, P, vp, vp, sz, vp]
    lib.sgwls_pass_backward.restype = i
    lib.sgwls_pass_backward.argtypes = [i, vp, vp, vp, vp, vp, vp, i, i, i, P, vp, vp, sz, vp]
    lib.sgwls_backward_workspace_bytes.restype = sz
    lib.sgwls_backward_workspace_bytes.argtypes = [i, i, i, P]
    lib.sgwls_batched_workspace_bytes.restype = sz
    lib.sgwls_batched_workspace_bytes.argtypes = [ctypes.POINTER(SgwlsImage), P, i]
    lib.sgwls_filter_batched.restype = i
    lib.sgwls_filter_batched.argtypes = [ctypes.POINTER(SgwlsImage), P, i, vp, sz, vp]
    IM = ctypes.POINTER(SgwlsImage)
    lib.sgwls_batched_variant_count.restype = i
    lib.sgwls_batched_variant_count.argtypes = [i]
    lib.sgwls_filter_batched_variant.restype = i
    lib.sgwls_filter_batched_variant.argtypes = [IM, P, i, i, vp, sz, vp]
    lib.sgwls_autotune_batched.restype = i
    lib.sgwls_autotune_batched.argtypes = [IM, P, i, vp, sz, vp, i, ctypes.POINTER(ctypes.c_int)]
    lib.sgwls_batched_graph_count.restype = i
    lib.sgwls_batched_graph_count.argtypes = []
    lib.sgwls_batched_graph_clear.restype = None
    lib.sgwls_batched_graph_clear.argtypes = []
    lib.sgwls_variant_count.restype = i
    lib.sgwls_variant_count.argtypes = [i, i, i]
    lib.sgwls_tune_pin.restype = i
    lib.sgwls_tune_pin.argtypes = [i, i, i, i, P, i]
    lib.sgwls_tune_query.restype = i
    lib.sgwls_tune_query.argtypes = [i, i, i, i, P]
    lib.sgwls_tune_clear.restype = None
    lib.sgwls_tune_clear.argtypes = []
    lib.sgwls_tune_size.restype = i
    lib.sgwls_tune_size.argtypes = []
    lib.sgwls_autotune.restype = i
    lib.sgwls_autotune.argtypes = [vp, vp, vp, i, i, i, P, vp, sz, vp, i, ctypes.POINTER(ctypes.c_int)]
    lib.sgwls_tune_save.restype = i
    lib.sgwls_tune_save.argtypes = [ctypes.c_char_p, ctypes.c_char_p]
    lib.sgwls_tune_load.restype = i
    lib.sgwls_tune_load.argtypes = [ctypes.c_char_p, ctypes.c_char_p]
    return lib


lib = _load()


def check(code: int, what: str) -> None:
    if code != 0:
        raise SgwlsError(code, what)
