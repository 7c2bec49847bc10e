"""MI355X-native SIDWT multiresolution correlation (Python binding).

The computation lives in libsidwt.so (hand-written HIP for gfx950, C ABI in
include/sidwt.h).  This module marshals PyTorch device tensors and streams
to that ABI; PyTorch provides memory and streams only.

Functions keep the C names without the `sidwt_` prefix:

    plan = plan_create("cdf97", J, ref)          # ref: host complex (m,) or int16 (m, 2)
    out = correlate(plan, rx)                    # rx: cuda complex64 (n,) -> (J, N)
    out = correlate_many(plan, rx)               # rx: cuda complex64 (count, n) -> (count, J, N)
    pyr = lift_many("cdf97", J, rx)              # lifting only -> (count, N)
    plan.free()
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import FILTERS, SidwtError, check, lib  # noqa: F401

__all__ = ["Plan", "plan_create", "correlate", "correlate_many", "lift_many", "out_len",
           "transform_length", "plan_phase", "SidwtError", "FILTERS", "version"]


def transform_length(n: int, J: int) -> int:
    q = 1 << J
    return q * ((n + q - 1) // q)


def _torch():
    import torch  # imported first so the HIP runtime is shared with PyTorch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """Owns a sidwt_plan (device phase pyramid of one reference)."""

    def __init__(self, filt: str, J: int, ref):
        _torch()
        self.filter = filt
        self.J = J
        if filt not in FILTERS:
            raise ValueError(f"unknown filter {filt}")
        if filt == "legall53_int":
            arr = np.ascontiguousarray(np.asarray(ref, dtype=np.int16).reshape(-1, 2))
        else:
            arr = np.ascontiguousarray(np.asarray(ref, dtype=np.complex64).reshape(-1))
        self.m = arr.shape[0]
        self._ref = arr
        h = ctypes.c_void_p()
        check(lib().sidwt_plan_create(FILTERS[filt], J, arr.ctypes.data_as(ctypes.c_void_p),
                                      self.m, ctypes.byref(h)), "sidwt_plan_create")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan already freed")
        return self._h

    @property
    def is_int(self) -> bool:
        return self.filter == "legall53_int"

    def out_len(self, n: int) -> int:
        return lib().sidwt_out_len(self.handle, n)

    def free(self):
        if getattr(self, "_h", None) is not None:
            lib().sidwt_free(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.free()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def plan_create(filt: str, J: int, ref) -> Plan:
    return Plan(filt, J, ref)


def out_len(plan: Plan, n: int) -> int:
    return plan.out_len(n)


def _check_rx(plan: Plan, rx):
    torch = _torch()
    if not rx.is_cuda:
        raise ValueError("rx must be a device tensor")
    if plan.is_int:
        if rx.dtype != torch.int16 or rx.shape[-1] != 2:
            raise ValueError("integer plans take int16 (..., n, 2) I/Q pulses")
    elif rx.dtype != torch.complex64:
        raise ValueError("float plans take complex64 pulses")
    if not rx.is_contiguous():
        raise ValueError("rx must be contiguous")


def _out_like(plan: Plan, lead, N, device):
    torch = _torch()
    if plan.is_int:
        return torch.empty(tuple(lead) + (plan.J, N, 2), dtype=torch.int64, device=device)
    return torch.empty(tuple(lead) + (plan.J, N), dtype=torch.complex64, device=device)


def correlate(plan: Plan, rx, out=None, stream=None):
    """One pulse.  rx: complex64 (n,) or int16 (n, 2); returns (J, N) complex64
    or (J, N, 2) int64."""
    _check_rx(plan, rx)
    n = rx.shape[0]
    N = transform_length(n, plan.J)
    if out is None:
        out = _out_like(plan, (), N, rx.device)
    check(lib().sidwt_set_stream(plan.handle, _stream_ptr(stream)), "sidwt_set_stream")
    check(lib().sidwt_correlate(plan.handle, ctypes.c_void_p(rx.data_ptr()), n,
                                ctypes.c_void_p(out.data_ptr())), "sidwt_correlate")
    return out


def correlate_many(plan: Plan, rx, out=None, stream=None):
    """Uniform batch in one launch.  rx: complex64 (count, n) or int16
    (count, n, 2); returns (count, J, N) or (count, J, N, 2)."""
    _check_rx(plan, rx)
    count, n = rx.shape[0], rx.shape[1]
    N = transform_length(n, plan.J)
    if out is None:
        out = _out_like(plan, (count,), N, rx.device)
    check(lib().sidwt_set_stream(plan.handle, _stream_ptr(stream)), "sidwt_set_stream")
    check(lib().sidwt_correlate_many(plan.handle, ctypes.c_void_p(rx.data_ptr()), n, count, n,
                                     ctypes.c_void_p(out.data_ptr()), plan.J * N),
          "sidwt_correlate_many")
    return out


def lift_many(filt: str, J: int, rx, pyr=None, stream=None):
    """Critical y-side lifting only.  Returns (count, N): d_1 | ... | d_J | c_J
    (complex64, or int32 pairs (count, N, 2) for the integer filter)."""
    torch = _torch()
    count, n = rx.shape[0], rx.shape[1]
    N = transform_length(n, J)
    if pyr is None:
        if filt == "legall53_int":
            pyr = torch.empty((count, N, 2), dtype=torch.int32, device=rx.device)
        else:
            pyr = torch.empty((count, N), dtype=torch.complex64, device=rx.device)
    check(lib().sidwt_lift_many(FILTERS[filt], J, ctypes.c_void_p(rx.data_ptr()), n, count, n,
                                ctypes.c_void_p(pyr.data_ptr()), _stream_ptr(stream)),
          "sidwt_lift_many")
    return pyr


def plan_phase(plan: Plan, level: int, band: int, r: int):
    """(lo, coefficients) of a stored phase (test introspection)."""
    lo = ctypes.c_int32()
    ln = ctypes.c_int32()
    check(lib().sidwt_plan_phase(plan.handle, level, band, r, ctypes.byref(lo), ctypes.byref(ln),
                                 None), "sidwt_plan_phase")
    if plan.is_int:
        buf = np.zeros((ln.value, 2), np.int32)
    else:
        buf = np.zeros(ln.value, np.complex64)
    check(lib().sidwt_plan_phase(plan.handle, level, band, r, ctypes.byref(lo), ctypes.byref(ln),
                                 buf.ctypes.data_as(ctypes.c_void_p)), "sidwt_plan_phase")
    return lo.value, buf


def version() -> str:
    return lib().sidwt_version().decode()
