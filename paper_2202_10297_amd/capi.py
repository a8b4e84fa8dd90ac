"""ctypes binding of libpvjp.so under the C-ABI names of include/pvjp.h.

Argument marshalling only: every function here forwards plain integers and
pointers to the library.  Loading fails loudly when the library is missing;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpvjp.so")

PVJP_OK, PVJP_EINVAL, PVJP_ENOMEM, PVJP_EDEVICE, PVJP_EUNSUPPORTED = 0, 1, 2, 3, 4
F32, F64 = 0, 1
ADD, MUL, MIN, MAX = 0, 1, 2, 3
FN_SQUARE, FN_EXP, FN_LOG, FN_SIN, FN_TANH = 0, 1, 2, 3, 4
GOP_LOGADDEXP, GOP_LINREC, GOP_MAT2 = 0, 1, 2
GMAP = {"gather": 0, "mul": 1, "sqdiff": 2}
LINREC_CKPT_INTERVAL = 1024
HIST_PATH_LDS, HIST_PATH_CACHE, HIST_PATH_PARTITION = 0, 1, 2
DIAG_OOB, DIAG_DUP, DIAG_NAN, DIAG_INF, DIAG_N = 0, 1, 2, 3, 4

_P = ctypes.c_void_p
_I = ctypes.c_int
_L = ctypes.c_int64
_Z = ctypes.c_size_t
_S = ctypes.c_char_p

# name -> (restype, argtypes), in header order.
SIGNATURES = {
    "pvjp_last_error": (_S, []),
    "pvjp_version": (_S, []),
    "pvjp_ws_clear": (_I, [_P, _Z, _P]),
    "pvjp_ws_check": (_I, [_P, _I, _P]),
    "pvjp_diag_indices": (_I, [_P, _L, _L, _P, _P]),
    "pvjp_diag_scatter_ws_bytes": (_Z, [_L]),
    "pvjp_diag_scatter": (_I, [_P, _L, _L, _P, _P, _Z, _P]),
    "pvjp_diag_nonfinite": (_I, [_I, _P, _L, _P, _P]),
    "pvjp_linrec_ckpt_len": (_L, [_L]),
    "pvjp_linrec_scan_ws_bytes": (_Z, [_I, _L]),
    "pvjp_linrec_scan": (_I, [_I, _P, _P, _L, _P, _P, _P, _P, _Z, _P]),
    "pvjp_linrec_scan_vjp_ws_bytes": (_Z, [_I, _L]),
    "pvjp_linrec_scan_vjp": (_I, [_I, _P, _P, _P, _P, _L, _P, _P, _P, _I, _P, _Z, _P]),
    "pvjp_linrec_scan_vjp_noalloc_max_bytes": (_Z, []),
    "pvjp_linrec_scan_vjp_noalloc": (_I, [_I, _P, _P, _P, _P, _L, _P, _P, _P, _I, _P]),
    "pvjp_reduce_ws_bytes": (_Z, [_I, _I, _L]),
    "pvjp_reduce": (_I, [_I, _I, _P, _L, _P, _P, _P, _P, _P, _Z, _P]),
    "pvjp_reduce_vjp": (_I, [_I, _I, _P, _L, _P, _P, _P, _P, _P, _I, _P]),
    "pvjp_hist_ws_bytes": (_Z, [_I, _I, _L, _L]),
    "pvjp_hist_plan_info": (_I, [_I, _I, _L, _L, _I, _P]),
    "pvjp_hist": (_I, [_I, _I, _P, _P, _L, _L, _P, _P, _P, _P, _P, _P, _Z, _P]),
    "pvjp_hist_vjp": (_I, [_I, _I, _P, _P, _L, _L, _P, _P, _P, _P, _P, _I, _P]),
    "pvjp_scatter": (_I, [_I, _P, _L, _P, _P, _L, _P, _P]),
    "pvjp_scatter_vjp": (_I, [_I, _P, _L, _P, _L, _P, _I, _P, _P, _P]),
    "pvjp_scatter_plan_bytes": (_Z, [_I, _L, _L]),
    "pvjp_scatter_planned": (_I, [_I, _P, _L, _P, _P, _L, _P, _Z, _P]),
    "pvjp_scatter_planned_vjp": (_I, [_I, _P, _L, _L, _P, _I, _P, _P, _Z, _P]),
    "pvjp_map": (_I, [_I, _I, _P, _L, _P, _P]),
    "pvjp_map_vjp": (_I, [_I, _I, _P, _P, _L, _P, _I, _P]),
    "pvjp_fig1": (_I, [_I, _P, _P, _L, _P, _P, _P]),
    "pvjp_fig1_vjp": (_I, [_I, _P, _P, _P, _P, _L, _P, _P, _I, _P]),
    "pvjp_gop_components": (_I, [_I]),
    "pvjp_reduce_generic_ws_bytes": (_Z, [_I, _I, _L]),
    "pvjp_reduce_generic_ckpt_bytes": (_Z, [_I, _I, _L]),
    "pvjp_reduce_generic": (_I, [_I, _I, _P, _L, _P, _P, _P, _Z, _P]),
    "pvjp_reduce_generic_vjp": (_I, [_I, _I, _P, _L, _P, _P, _P, _I, _P, _Z, _P]),
    "pvjp_scan_generic_ws_bytes": (_Z, [_I, _I, _L]),
    "pvjp_scan_generic_ckpt_bytes": (_Z, [_I, _I, _L]),
    "pvjp_scan_generic": (_I, [_I, _I, _P, _L, _P, _P, _P, _Z, _P]),
    "pvjp_scan_generic_vjp": (_I, [_I, _I, _P, _L, _P, _P, _P, _I, _P, _Z, _P]),
    "pvjp_scan_generic_batched_ws_bytes": (_Z, [_I, _I, _L, _L]),
    "pvjp_scan_generic_batched_ckpt_bytes": (_Z, [_I, _I, _L, _L]),
    "pvjp_scan_generic_batched": (_I, [_I, _I, _P, _L, _L, _P, _P, _P, _Z, _P]),
    "pvjp_scan_generic_batched_vjp": (_I, [_I, _I, _P, _L, _L, _P, _P, _P, _I, _P, _Z, _P]),
    "pvjp_map_jvp": (_I, [_I, _I, _P, _P, _L, _P, _P]),
    "pvjp_reduce_jvp": (_I, [_I, _I, _P, _P, _L, _P, _P, _P, _P, _P, _Z, _P]),
    "pvjp_hist_jvp_ws_bytes": (_Z, [_I, _I, _L, _L]),
    "pvjp_hist_jvp": (_I, [_I, _I, _P, _P, _L, _L, _P, _P, _P, _Z, _P]),
    "pvjp_scatter_jvp": (_I, [_I, _P, _L, _P, _P, _L, _P]),
    "pvjp_reduce_generic_jvp_ws_bytes": (_Z, [_I, _I, _L]),
    "pvjp_scan_generic_jvp_ws_bytes": (_Z, [_I, _I, _L]),
    "pvjp_reduce_generic_jvp": (_I, [_I, _I, _P, _P, _L, _P, _P, _P, _Z, _P]),
    "pvjp_scan_generic_jvp": (_I, [_I, _I, _P, _P, _L, _P, _P, _P, _Z, _P]),
    "pvjp_seg_ws_bytes": (_Z, [_L, _L, _I]),
    "pvjp_seg_prepare": (_I, [_P, _L, _I, _P, _Z, _P]),
    "pvjp_seg_linrec_scan": (_I, [_I, _P, _P, _L, _L, _I, _P, _P, _P, _P, _Z, _P]),
    "pvjp_seg_batch_vjp": (_I, [_I, _P, _P, _P, _P, _L, _L, _I, _P, _P, _P, _P, _P, _I, _I, _P, _Z, _P]),
    "pvjp_kmeans_ws_bytes": (_Z, [_L, _I, _I]),
    "pvjp_kmeans_objective": (_I, [_P, _L, _I, _P, _I, _P, _P, _P, _Z, _P]),
    "pvjp_kmeans_vjp": (_I, [_P, _L, _I, _P, _I, _P, ctypes.c_double, _P, _P, _P, _I, _P, _Z, _P]),
    "pvjp_gather_map": (_I, [_I, _I, _P, _L, _P, _P, _L, _P, _P]),
    "pvjp_sparse_kmeans_ws_bytes": (_Z, [_L, _L, _I, _L]),
    "pvjp_hist_lae_ws_bytes": (_Z, [_I, _L, _L]),
    "pvjp_hist_lae": (_I, [_I, _P, _P, _L, _L, _P, _P, _Z, _P]),
    "pvjp_hist_lae_vjp": (_I, [_I, _P, _P, _L, _L, _P, _P, _P, _I, _P]),
    "pvjp_hist_generic_ws_bytes": (_Z, [_I, _I, _L, _L]),
    "pvjp_hist_generic": (_I, [_I, _I, _P, _P, _L, _L, _P, _P, _Z, _P]),
    "pvjp_hist_generic_vjp": (_I, [_I, _I, _P, _P, _L, _L, _P, _P, _I, _P, _Z, _P]),
    "pvjp_sparse_kmeans_objective": (_I, [_P, _P, _P, _L, _L, _L, _P, _I, _P, _P, _P, _Z, _P]),
    "pvjp_sparse_kmeans_vjp": (_I, [_P, _P, _P, _L, _L, _L, _P, _I, _P, ctypes.c_double, _P, _P, _P, _I, _P, _Z,
                                    _P]),
    "pvjp_gather_map_ws_bytes": (_Z, [_I, _L, _L]),
    "pvjp_gather_map_vjp": (_I, [_I, _I, _P, _L, _P, _P, _L, _P, _P, _P, _I, _P, _Z, _P]),
    "pvjp_gmm_ws_bytes": (_Z, [_L, _I, _I]),
    "pvjp_gmm_objective": (_I, [_P, _L, _I, _I, _P, _P, _P, _P, _P, _P, _P, _P, _Z, _P]),
    "pvjp_gmm_vjp": (_I, [_P, _L, _I, _I, _P, _P, _P, _P, ctypes.c_double, _P, _P, _P, _P, _P, _P, _I, _P, _Z,
                          _P]),
}

_lib = None


class PvjpError(RuntimeError):
    def __init__(self, name, status, msg):
        super().__init__(f"{name} failed with status {status}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """Loads libpvjp.so (built in-tree by paper_2202_10297_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2202_10297_amd.build` "
                "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().pvjp_last_error().decode()


def version() -> str:
    return lib().pvjp_version().decode()


def ptr_array(ptrs):
    """A host array of device pointers (the K component arrays of an
    element); None entries become NULL."""
    return (ctypes.c_void_p * len(ptrs))(*[p or None for p in ptrs])


def call(name: str, *args):
    """Calls a status-returning entry point and raises PvjpError on failure."""
    st = getattr(lib(), name)(*args)
    if st != PVJP_OK:
        raise PvjpError(name, st, last_error())
    return st


def __getattr__(name):
    # capi.pvjp_xxx -> the raw ctypes function of the same name
    if name in SIGNATURES:
        return getattr(lib(), name)
    raise AttributeError(name)
