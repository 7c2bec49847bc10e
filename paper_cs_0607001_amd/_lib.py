"""ctypes binding of libsidwt.so (the C ABI in include/sidwt.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  If the library is missing the import of this module raises; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsidwt.so")

SIDWT_OK = 0
SIDWT_E_INVAL = -1
SIDWT_E_SIZE = -2
SIDWT_E_NOMEM = -3
SIDWT_E_DEVICE = -4
SIDWT_E_UNSUPPORTED = -5
SIDWT_E_SCRATCH = -6

FILTERS = {"legall53": 1, "cdf97": 2, "d4": 3, "legall53_int": 4}

_lib = None


class SidwtError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = lib().sidwt_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} (code {code})" if what else f"{msg} (code {code})")


def _declare(L):
    c = ctypes
    vp, i64, i32 = c.c_void_p, c.c_int64, c.c_int
    L.sidwt_plan_create.argtypes = [i32, i32, vp, i64, c.POINTER(vp)]
    L.sidwt_plan_create.restype = i32
    L.sidwt_free.argtypes = [vp]
    L.sidwt_free.restype = None
    L.sidwt_out_len.argtypes = [vp, i64]
    L.sidwt_out_len.restype = i64
    L.sidwt_set_stream.argtypes = [vp, vp]
    L.sidwt_set_stream.restype = i32
    L.sidwt_correlate.argtypes = [vp, vp, i64, vp]
    L.sidwt_correlate.restype = i32
    L.sidwt_correlate_many.argtypes = [vp, vp, i64, i64, i64, vp, i64]
    L.sidwt_correlate_many.restype = i32
    L.sidwt_correlate_on.argtypes = [vp, vp, i64, vp, vp]
    L.sidwt_correlate_on.restype = i32
    L.sidwt_correlate_many_on.argtypes = [vp, vp, i64, i64, i64, vp, i64, c.c_uint, vp]
    L.sidwt_correlate_many_on.restype = i32
    L.sidwt_lift_many.argtypes = [i32, i32, vp, i64, i64, i64, vp, vp]
    L.sidwt_lift_many.restype = i32
    L.sidwt_correlate_planes.argtypes = [vp, vp, i64, i64, i64, vp, i64, c.c_uint]
    L.sidwt_correlate_planes.restype = i32
    L.sidwt_synth_many.argtypes = [i32, i32, i32, vp, i64, i64, vp, vp]
    L.sidwt_synth_many.restype = i32
    L.sidwt_swap_workspace_bytes.argtypes = [vp, i64, i64]
    L.sidwt_swap_workspace_bytes.restype = i64
    L.sidwt_correlate_swapped.argtypes = [vp, vp, i64, i64, i64, vp, i64, vp, i64]
    L.sidwt_correlate_swapped.restype = i32
    L.sidwt_correlate_swapped_on.argtypes = [vp, vp, i64, i64, i64, vp, i64, vp, i64, vp]
    L.sidwt_correlate_swapped_on.restype = i32
    L.sidwt_correlate_swapped_noalloc.argtypes = [vp, vp, i64, i64, i64, vp, i64, vp]
    L.sidwt_correlate_swapped_noalloc.restype = i32
    L.sidwt_detect_peaks.argtypes = [vp, i64, i32, i64, i64, c.c_float, i32, vp, vp, vp, vp]
    L.sidwt_detect_peaks.restype = i32
    dp = c.POINTER(c.c_double)
    ip = c.POINTER(i32)
    L.sidwt_lifting_factorize.argtypes = [dp, i32, i32, dp, i32, i32, c.POINTER(vp)]
    L.sidwt_lifting_factorize.restype = i32
    L.sidwt_lifting_count.argtypes = [vp]
    L.sidwt_lifting_count.restype = i32
    L.sidwt_lifting_step.argtypes = [vp, i32, ip, ip, ip, dp]
    L.sidwt_lifting_step.restype = i32
    L.sidwt_lifting_scaling.argtypes = [vp, dp, ip, dp, ip]
    L.sidwt_lifting_scaling.restype = i32
    L.sidwt_lifting_free.argtypes = [vp]
    L.sidwt_lifting_free.restype = None
    L.sidwt_lift_generic.argtypes = [vp, i32, vp, i64, i64, i64, vp, vp]
    L.sidwt_lift_generic.restype = i32
    L.sidwt_correlate_batch.argtypes = [c.POINTER(vp), c.POINTER(vp), c.POINTER(i64),
                                        c.POINTER(vp), i32, vp]
    L.sidwt_correlate_batch.restype = i32
    L.sidwt_plan_phase.argtypes = [vp, i32, i32, i32, c.POINTER(c.c_int32),
                                   c.POINTER(c.c_int32), vp]
    L.sidwt_plan_phase.restype = i32
    L.sidwt_plan_info.argtypes = [vp, c.POINTER(i64), i32]
    L.sidwt_plan_info.restype = i32
    L.sidwt_strerror.argtypes = [i32]
    L.sidwt_strerror.restype = c.c_char_p
    L.sidwt_version.argtypes = []
    L.sidwt_version.restype = c.c_char_p
    pp = c.POINTER(vp)
    L.sidwt_batch_create.argtypes = [pp, c.POINTER(i64), i32, pp]
    L.sidwt_batch_create.restype = i32
    L.sidwt_batch_run.argtypes = [vp, pp, pp, vp]
    L.sidwt_batch_run.restype = i32
    L.sidwt_batch_tune.argtypes = [vp, pp, pp, vp]
    L.sidwt_batch_tune.restype = i32
    L.sidwt_batch_config.argtypes = [vp, i64, i32]
    L.sidwt_batch_config.restype = i32
    L.sidwt_batch_configure.argtypes = [vp, i64, i32, i32]
    L.sidwt_batch_configure.restype = i32
    L.sidwt_batch_info.argtypes = [vp, c.POINTER(i64), i32]
    L.sidwt_batch_info.restype = i32
    L.sidwt_batch_free.argtypes = [vp]
    L.sidwt_batch_free.restype = None
    L.sidwt_bank_create.argtypes = [i32, i32, pp, c.POINTER(i64), i32, i32, pp]
    L.sidwt_bank_create.restype = i32
    L.sidwt_bank_correlate.argtypes = [vp, pp, c.POINTER(i64), c.POINTER(i32), pp, i32, vp]
    L.sidwt_bank_correlate.restype = i32
    L.sidwt_bank_eligible.argtypes = [vp, i64]
    L.sidwt_bank_eligible.restype = i64
    L.sidwt_bank_out_len.argtypes = [vp, i64, i32]
    L.sidwt_bank_out_len.restype = i64
    L.sidwt_bank_plan.argtypes = [vp, i32]
    L.sidwt_bank_plan.restype = vp
    L.sidwt_bank_info.argtypes = [vp, c.POINTER(i64), i32]
    L.sidwt_bank_info.restype = i32
    L.sidwt_bank_free.argtypes = [vp]
    L.sidwt_bank_free.restype = None
    L.sidwt_bank_ws_create.argtypes = [vp, pp]
    L.sidwt_bank_ws_create.restype = i32
    L.sidwt_bank_ws_free.argtypes = [vp]
    L.sidwt_bank_ws_free.restype = None
    L.sidwt_bank_ws_timing.argtypes = [vp, i32]
    L.sidwt_bank_ws_timing.restype = i32
    L.sidwt_bank_ws_times.argtypes = [vp, c.POINTER(c.c_float), c.POINTER(c.c_float)]
    L.sidwt_bank_ws_times.restype = i32
    L.sidwt_bank_correlate_ws.argtypes = [vp, vp, pp, c.POINTER(i64), c.POINTER(i32), pp, i32, vp]
    L.sidwt_bank_correlate_ws.restype = i32
    L.sidwt_bank_scratch_bytes.argtypes = [vp, i64, i32]
    L.sidwt_bank_scratch_bytes.restype = i64
    return L


def lib():
    """Load libsidwt.so (HIP runtime is shared with PyTorch when torch is
    imported first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libsidwt.so not built ({LIB_PATH}); run __graft_entry__.build()")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def check(code: int, what: str = ""):
    if code != SIDWT_OK:
        raise SidwtError(code, what)
