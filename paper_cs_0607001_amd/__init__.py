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

__all__ = ["Plan", "plan_create", "correlate", "correlate_many", "correlate_swapped", "lift_many",
           "synth_many", "detect_peaks", "Lifting", "lift_generic", "out_len",
           "transform_length", "plan_phase", "Batch", "correlate_batch", "Bank",
           "SidwtError", "FILTERS", "version"]


def transform_length(n: int, J: int) -> int:
    q = 1 << J
    return q * ((n + q - 1) // q)


def _torch():
    import torch  # imported first so the HIP runtime is shared with PyTorch
    return torch


def _stream_ptr(stream=None):
    """The HIP stream of a call: `stream`, else torch's current stream on the
    current device (read through torch's raw accessor where it has one: the
    public one builds a Stream object per call, a few microseconds)."""
    torch = _torch()
    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream)
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return ctypes.c_void_p(raw(torch._C._cuda_getDevice()))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """Owns a sidwt_plan (device phase pyramid of one reference)."""

    @classmethod
    def borrowed(cls, handle, filt: str, J: int, m: int):
        """A view of a plan owned by someone else (freeing it is a no-op)."""
        p = cls.__new__(cls)
        p.filter, p.J, p.m, p._ref = filt, J, m, None
        p._h = ctypes.c_void_p(handle)
        p._borrowed = True
        return p

    def __init__(self, filt: str, J: int, ref):
        _torch()
        self._borrowed = False
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

    INFO_KEYS = ("filter", "J", "m", "coef_bytes", "i8_weight_digits", "i8_panel_bytes")

    def info(self) -> dict:
        v = (ctypes.c_int64 * len(self.INFO_KEYS))()
        check(lib().sidwt_plan_info(self.handle, v, len(self.INFO_KEYS)), "sidwt_plan_info")
        return dict(zip(self.INFO_KEYS, list(v)))

    def free(self):
        if getattr(self, "_h", None) is not None:
            if not getattr(self, "_borrowed", False):
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


def _check_buf(t, dtype, numel: int, what: str, device=None):
    """A caller-supplied device buffer: a contiguous device tensor of `dtype`
    holding at least `numel` elements (on `device` when given), else
    ValueError before anything is launched."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{what} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{what} holds {t.numel()} elements, needs {numel}")
    return t


def _check_pulses(rx, dtype, what="rx"):
    """A (count, n[, 2]) batch of pulses: contiguous device tensor of dtype."""
    torch = _torch()
    if not isinstance(rx, torch.Tensor) or not rx.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if rx.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {rx.dtype}")
    if not rx.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if rx.dim() < 2 or rx.shape[0] < 0 or rx.shape[1] < 1:
        raise ValueError(f"{what} must be shaped (count, n, ...)")


def _out_numel(plan: Plan, count: int, N: int) -> int:
    """Elements of torch's view of the output: complex64, or int64 with the
    (re, im) pair as the last axis."""
    return count * plan.J * N * (2 if plan.is_int else 1)


def _out_dtype(plan: Plan):
    torch = _torch()
    return torch.int64 if plan.is_int else torch.complex64


def _out_like(plan: Plan, lead, N, device):
    torch = _torch()
    if plan.is_int:
        return torch.empty(tuple(lead) + (plan.J, N, 2), dtype=torch.int64, device=device)
    return torch.empty(tuple(lead) + (plan.J, N), dtype=torch.complex64, device=device)


def correlate(plan: Plan, rx, out=None, stream=None):
    """One pulse.  rx: complex64 (n,) or int16 (n, 2); returns (J, N) complex64
    or (J, N, 2) int64."""
    _check_rx(plan, rx)
    if rx.dim() != (2 if plan.is_int else 1):
        raise ValueError("rx must be shaped (n,) (complex64) or (n, 2) (int16)")
    n = rx.shape[0]
    N = transform_length(n, plan.J)
    if out is None:
        out = _out_like(plan, (), N, rx.device)
    _check_buf(out, _out_dtype(plan), _out_numel(plan, 1, N), "out", rx.device)
    check(lib().sidwt_correlate_on(plan.handle, ctypes.c_void_p(rx.data_ptr()), n,
                                   ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
          "sidwt_correlate_on")
    return out


def correlate_many(plan: Plan, rx, out=None, stream=None, planes=None):
    """Uniform batch in one launch.  rx: complex64 (count, n) or int16
    (count, n, 2); returns (count, J, N) or (count, J, N, 2).  planes: an
    iterable of plane indices to compute (the others of out are left as they
    are); None computes all."""
    _check_rx(plan, rx)
    if rx.dim() != (3 if plan.is_int else 2):
        raise ValueError("rx must be shaped (count, n) (complex64) or (count, n, 2) (int16)")
    count, n = rx.shape[0], rx.shape[1]
    N = transform_length(n, plan.J)
    if out is None:
        out = _out_like(plan, (count,), N, rx.device)
    _check_buf(out, _out_dtype(plan), _out_numel(plan, count, N), "out", rx.device)
    mask = 0xFFFFFFFF
    if planes is not None:
        mask = 0
        for j in planes:
            if not 0 <= int(j) < plan.J:
                raise ValueError(f"plane {j} outside 0..{plan.J - 1}")
            mask |= 1 << int(j)
    check(lib().sidwt_correlate_many_on(plan.handle, ctypes.c_void_p(rx.data_ptr()), n, count, n,
                                        ctypes.c_void_p(out.data_ptr()), plan.J * N, mask,
                                        _stream_ptr(stream)), "sidwt_correlate_many_on")
    return out


def correlate_swapped(plan: Plan, rx, out=None, workspace=None, stream=None):
    """Roles exchanged: redundant y-side analysis on each received pulse,
    critical x-side on the plan's reference (plane j, lag s pairs the
    reference's level-j approximation with that of the pulse advanced by s).
    rx: complex64 (count, n); returns (count, J, N).  workspace: a device
    buffer of at least sidwt_swap_workspace_bytes (allocated if None)."""
    _check_rx(plan, rx)
    torch = _torch()
    if rx.dim() != 2:
        raise ValueError("rx must be shaped (count, n)")
    count, n = rx.shape[0], rx.shape[1]
    N = transform_length(n, plan.J)
    if out is None:
        out = _out_like(plan, (count,), N, rx.device)
    _check_buf(out, _out_dtype(plan), _out_numel(plan, count, N), "out", rx.device)
    need = lib().sidwt_swap_workspace_bytes(plan.handle, n, count)
    if need < 0:
        raise SidwtError(-1, "sidwt_swap_workspace_bytes")
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=rx.device)
    if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or \
            not workspace.is_contiguous() or workspace.device != rx.device:
        raise ValueError("workspace must be a contiguous device tensor on the pulses' device")
    check(lib().sidwt_correlate_swapped_on(plan.handle, ctypes.c_void_p(rx.data_ptr()), n, count,
                                           n, ctypes.c_void_p(out.data_ptr()), plan.J * N,
                                           ctypes.c_void_p(workspace.data_ptr()),
                                           workspace.numel() * workspace.element_size(),
                                           _stream_ptr(stream)), "sidwt_correlate_swapped_on")
    return out


def detect_peaks(planes, level_db: float = -10.0, max_peaks: int = 64, stream=None):
    """Target declaration on correlation planes (count, J, N) complex64 (as
    correlate_many returns them): per plane, the lags whose power is a local
    maximum at least level_db relative to the plane's peak.  Returns (lags
    int32 (count, J, max_peaks), db float32 (count, J, max_peaks), found
    int32 (count, J)); entries past found are unspecified."""
    torch = _torch()
    count, J, N = planes.shape
    if planes.dtype != torch.complex64 or not planes.is_contiguous():
        raise ValueError("planes must be contiguous complex64 (count, J, N)")
    import numpy as np
    rel = float(np.float32(10.0 ** (level_db / 10.0)))
    lags = torch.empty((count, J, max_peaks), dtype=torch.int32, device=planes.device)
    db = torch.empty((count, J, max_peaks), dtype=torch.float32, device=planes.device)
    found = torch.empty((count, J), dtype=torch.int32, device=planes.device)
    check(lib().sidwt_detect_peaks(ctypes.c_void_p(planes.data_ptr()), count, J, N, J * N, rel,
                                   max_peaks, ctypes.c_void_p(lags.data_ptr()),
                                   ctypes.c_void_p(db.data_ptr()),
                                   ctypes.c_void_p(found.data_ptr()), _stream_ptr(stream)),
          "sidwt_detect_peaks")
    return lags, db, found


class Lifting:
    """Lifting factorization (eq. (16)) of an analysis pair given as tap
    dicts {offset i: c_i} (out[k] = sum_i c_i u[2k + i]), computed by the
    library on the host.  steps: [(kind, first, coefs)] with kind 0 =
    predict (o += q e), 1 = update (e += q o); scaling: (ke, se, ko, so)."""

    def __init__(self, lo: dict, hi: dict):
        def arr(t):
            first = min(t)
            vals = [float(t.get(i, 0.0)) for i in range(first, max(t) + 1)]
            return first, (ctypes.c_double * len(vals))(*vals), len(vals)
        lf, la, ln = arr(lo)
        hf, ha, hn = arr(hi)
        h = ctypes.c_void_p()
        check(lib().sidwt_lifting_factorize(la, lf, ln, ha, hf, hn, ctypes.byref(h)),
              "sidwt_lifting_factorize")
        self.handle = h

    @property
    def steps(self):
        out = []
        for i in range(lib().sidwt_lifting_count(self.handle)):
            kind, first, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            coef = (ctypes.c_double * 8)()
            check(lib().sidwt_lifting_step(self.handle, i, ctypes.byref(kind), ctypes.byref(first),
                                           ctypes.byref(n), coef), "sidwt_lifting_step")
            out.append((kind.value, first.value, list(coef[:n.value])))
        return out

    @property
    def scaling(self):
        ke, ko = ctypes.c_double(), ctypes.c_double()
        se, so = ctypes.c_int32(), ctypes.c_int32()
        check(lib().sidwt_lifting_scaling(self.handle, ctypes.byref(ke), ctypes.byref(se),
                                          ctypes.byref(ko), ctypes.byref(so)),
              "sidwt_lifting_scaling")
        return ke.value, se.value, ko.value, so.value

    def free(self):
        if self.handle:
            lib().sidwt_lifting_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


def lift_generic(lifting: Lifting, J: int, rx, pyr=None, stream=None):
    """Critical lifting of complex64 pulses (count, n) with a factorized pair;
    returns (count, N): d_1 | ... | d_J | c_J, as lift_many."""
    torch = _torch()
    _check_pulses(rx, torch.complex64)
    count, n = rx.shape[0], rx.shape[1]
    N = transform_length(n, J)
    if pyr is None:
        pyr = torch.empty((count, N), dtype=torch.complex64, device=rx.device)
    _check_buf(pyr, torch.complex64, count * N, "pyr", rx.device)
    check(lib().sidwt_lift_generic(lifting.handle, J, ctypes.c_void_p(rx.data_ptr()), n, count, n,
                                   ctypes.c_void_p(pyr.data_ptr()), _stream_ptr(stream)),
          "sidwt_lift_generic")
    return pyr


def lift_many(filt: str, J: int, rx, pyr=None, stream=None):
    """Critical y-side lifting only.  Returns (count, N): d_1 | ... | d_J | c_J
    (complex64, or int32 pairs (count, N, 2) for the integer filter)."""
    torch = _torch()
    if filt not in FILTERS:
        raise ValueError(f"unknown filter {filt}")
    is_int = filt == "legall53_int"
    _check_pulses(rx, torch.int16 if is_int else torch.complex64)
    if is_int and (rx.dim() != 3 or rx.shape[2] != 2):
        raise ValueError("the integer filter takes int16 (count, n, 2) I/Q pulses")
    count, n = rx.shape[0], rx.shape[1]
    N = transform_length(n, J)
    if pyr is None:
        if is_int:
            pyr = torch.empty((count, N, 2), dtype=torch.int32, device=rx.device)
        else:
            pyr = torch.empty((count, N), dtype=torch.complex64, device=rx.device)
    if is_int:
        _check_buf(pyr, torch.int32, count * N * 2, "pyr", rx.device)
    else:
        _check_buf(pyr, torch.complex64, count * N, "pyr", rx.device)
    check(lib().sidwt_lift_many(FILTERS[filt], J, ctypes.c_void_p(rx.data_ptr()), n, count, n,
                                ctypes.c_void_p(pyr.data_ptr()), _stream_ptr(stream)),
          "sidwt_lift_many")
    return pyr


def synth_many(filt: str, J: int, pyr, to: int = 0, out=None, stream=None):
    """Coarse-to-fine formation: from pyramids as lift_many returns them
    ((count, N) complex64, or (count, N, 2) int32 for the integer filter),
    the approximations c_to, (count, N >> to) (c_0 = the zero-padded pulses)."""
    torch = _torch()
    if filt not in FILTERS:
        raise ValueError(f"unknown filter {filt}")
    is_int = filt == "legall53_int"
    _check_pulses(pyr, torch.int32 if is_int else torch.complex64, "pyr")
    if is_int and (pyr.dim() != 3 or pyr.shape[2] != 2):
        raise ValueError("the integer filter's pyramids are int32 (count, N, 2)")
    count, N = pyr.shape[0], pyr.shape[1]
    if not 0 <= to < J:
        raise ValueError(f"to = {to} outside 0..{J - 1}")
    if out is None:
        shape = (count, N >> to, 2) if is_int else (count, N >> to)
        out = torch.empty(shape, dtype=pyr.dtype, device=pyr.device)
    _check_buf(out, pyr.dtype, count * (N >> to) * (2 if is_int else 1), "out", pyr.device)
    check(lib().sidwt_synth_many(FILTERS[filt], J, to, ctypes.c_void_p(pyr.data_ptr()), N, count,
                                 ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
          "sidwt_synth_many")
    return out


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


# ---------------------------------------------------------------------------
# Uneven batches
# ---------------------------------------------------------------------------

BATCH_INFO_KEYS = ("fused_max_N", "tile_window", "items", "whole_pulse_items", "tile_items",
                   "lds_bytes", "grid", "scratch_bytes", "tuned", "tuned_us", "lift_depth",
                   "lift_passes")


def _ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr


def batch_outputs(plans, ns, device):
    """Allocate each pulse's output of a batch: (J, N) complex64, or (J, N, 2)
    int64 for integer plans."""
    return [_out_like(p, (), transform_length(n, p.J), device) for p, n in zip(plans, ns)]


def _check_batch_pulse(plan, x, o, n, i):
    """Pulse i of a batch: rx complex64 (n,) or int16 (n, 2) for an integer
    plan; out as batch_outputs allocates it."""
    torch = _torch()
    N = transform_length(n, plan.J)
    if plan.is_int:
        _check_buf(x, torch.int16, 2 * n, f"rx[{i}]")
    else:
        _check_buf(x, torch.complex64, n, f"rx[{i}]")
    if o is not None:
        _check_buf(o, _out_dtype(plan), _out_numel(plan, 1, N), f"out[{i}]", x.device)


class Batch:
    """Owns a sidwt_batch: pulses of uneven lengths with their own plans,
    one persistent launch (replayed from a HIP graph) per run; or, when every
    plan is integer, one int8 launch per group of pulses of one plan and
    length."""

    def __init__(self, plans, ns):
        _torch()
        self.plans = list(plans)
        self.ns = [int(n) for n in ns]
        if len(self.plans) != len(self.ns) or not self.plans:
            raise ValueError("plans and lengths must be non-empty and of equal length")
        h = ctypes.c_void_p()
        plan_arr = _ptr_array([p.handle.value for p in self.plans])
        n_arr = (ctypes.c_int64 * len(self.ns))(*self.ns)
        check(lib().sidwt_batch_create(plan_arr, n_arr, len(self.ns), ctypes.byref(h)),
              "sidwt_batch_create")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("batch already freed")
        return self._h

    def _arrays(self, rx, out):
        torch = _torch()
        if len(rx) != len(self.ns) or len(out) != len(self.ns):
            raise ValueError("one input and one output per pulse")
        for i, (x, o, p, n) in enumerate(zip(rx, out, self.plans, self.ns)):
            _check_batch_pulse(p, x, o, n, i)
        return _ptr_array([x.data_ptr() for x in rx]), _ptr_array([o.data_ptr() for o in out])

    def run(self, rx, out, stream=None):
        a, b = self._arrays(rx, out)
        check(lib().sidwt_batch_run(self.handle, a, b, _stream_ptr(stream)), "sidwt_batch_run")
        return out

    def bind(self, rx, out):
        """Check the pulse and output tensors once and keep their pointer
        arrays, so that run_bound() replays the batch on exactly these
        buffers without re-marshalling one pointer per pulse on every call
        (for 10^4 pulses that host work outlasts the GPU step).  The batch
        holds references to the tensors until the next bind or free."""
        a, b = self._arrays(rx, out)
        self._bound = (a, b, list(rx), list(out))

    def run_bound(self, stream=None):
        """run() on the buffers of the last bind()."""
        bound = getattr(self, "_bound", None)
        if bound is None:
            raise RuntimeError("run_bound() before bind()")
        a, b, _, out = bound
        check(lib().sidwt_batch_run(self.handle, a, b, _stream_ptr(stream)), "sidwt_batch_run")
        return out

    def tune(self, rx, out, stream=None):
        a, b = self._arrays(rx, out)
        check(lib().sidwt_batch_tune(self.handle, a, b, _stream_ptr(stream)), "sidwt_batch_tune")
        return self.info()

    def config(self, fused_max_N: int, tile_window: int, lift_depth=None):
        if lift_depth is None:
            check(lib().sidwt_batch_config(self.handle, fused_max_N, tile_window),
                  "sidwt_batch_config")
        else:
            check(lib().sidwt_batch_configure(self.handle, fused_max_N, tile_window, lift_depth),
                  "sidwt_batch_configure")

    def info(self) -> dict:
        v = (ctypes.c_int64 * len(BATCH_INFO_KEYS))()
        check(lib().sidwt_batch_info(self.handle, v, len(BATCH_INFO_KEYS)), "sidwt_batch_info")
        return dict(zip(BATCH_INFO_KEYS, list(v)))

    def free(self):
        self._bound = None
        if getattr(self, "_h", None) is not None:
            lib().sidwt_batch_free(self._h)
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


def correlate_batch(plans, rx, out=None, stream=None):
    """One-shot uneven batch (synchronises the stream before returning)."""
    torch = _torch()
    if len(plans) != len(rx) or (out is not None and len(out) != len(rx)):
        raise ValueError("one plan, input and output per pulse")
    ns = []
    for i, (p, x) in enumerate(zip(plans, rx)):
        if not isinstance(x, torch.Tensor):
            raise ValueError(f"rx[{i}] must be a torch tensor")
        ns.append(int(x.numel() // 2 if p.is_int else x.numel()))
        _check_batch_pulse(p, x, None, max(1, ns[-1]), i)
    if out is None:
        out = batch_outputs(plans, ns, rx[0].device)
    for i, (x, o, p, n) in enumerate(zip(rx, out, plans, ns)):
        _check_batch_pulse(p, x, o, n, i)
    plan_arr = _ptr_array([p.handle.value for p in plans])
    n_arr = (ctypes.c_int64 * len(ns))(*ns)
    check(lib().sidwt_correlate_batch(plan_arr, _ptr_array([x.data_ptr() for x in rx]), n_arr,
                                      _ptr_array([o.data_ptr() for o in out]), len(ns),
                                      _stream_ptr(stream)), "sidwt_correlate_batch")
    return out


# ---------------------------------------------------------------------------
# Reference banks (16-bit MFMA, hi+lo correction)
# ---------------------------------------------------------------------------

BANK_PRECISION = {"fp32": 0, "fp16": 1, "bf16": 2}
BANK_INFO_KEYS = ("references", "Jmax", "precision", "weight_bytes", "max_window")


class Bank:
    """Owns a sidwt_bank: references of ascending length, one float filter."""

    def __init__(self, filt: str, Jmax: int, refs, precision: str = "fp16"):
        _torch()
        if filt not in FILTERS or precision not in BANK_PRECISION:
            raise ValueError("unknown filter or precision")
        self.filter, self.Jmax, self.precision = filt, Jmax, precision
        self._refs = [np.ascontiguousarray(np.asarray(r, np.complex64).reshape(-1)) for r in refs]
        self.m = [len(r) for r in self._refs]
        ptrs = _ptr_array([r.ctypes.data for r in self._refs])
        ms = (ctypes.c_int64 * len(self.m))(*self.m)
        h = ctypes.c_void_p()
        check(lib().sidwt_bank_create(FILTERS[filt], Jmax, ptrs, ms, len(self.m),
                                      BANK_PRECISION[precision], ctypes.byref(h)),
              "sidwt_bank_create")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("bank already freed")
        return self._h

    def eligible(self, n: int) -> int:
        return lib().sidwt_bank_eligible(self.handle, n)

    def out_shape(self, n: int, J: int):
        return (self.eligible(n), J, transform_length(n, J))

    def plan(self, e: int) -> Plan:
        """The bank's FP32 plan of reference e (borrowed)."""
        h = lib().sidwt_bank_plan(self.handle, e)
        if not h:
            raise IndexError(e)
        return Plan.borrowed(h, self.filter, self.Jmax, self.m[e])

    def workspace(self):
        """A workspace for calls in flight on one more stream."""
        h = ctypes.c_void_p()
        check(lib().sidwt_bank_ws_create(self.handle, ctypes.byref(h)), "sidwt_bank_ws_create")
        return BankWorkspace(h)

    def scratch_bytes(self, n: int, J: int) -> int:
        return lib().sidwt_bank_scratch_bytes(self.handle, n, J)

    def correlate(self, rx, J, out=None, stream=None, workspace=None):
        """rx: list of complex64 device pulses; J: list of scale counts.
        Returns a list of (E_i, J_i, N_i) complex64 tensors."""
        torch = _torch()
        if len(J) != len(rx) or (out is not None and len(out) != len(rx)):
            raise ValueError("one scale count and one output per request")
        for i, x in enumerate(rx):
            _check_buf(x, torch.complex64, 1, f"rx[{i}]")
        ns = [int(x.numel()) for x in rx]
        if out is None:
            out = [torch.empty(self.out_shape(n, j), dtype=torch.complex64, device=x.device)
                   for x, n, j in zip(rx, ns, J)]
        for i, (o, x, n, j) in enumerate(zip(out, rx, ns, J)):
            need = lib().sidwt_bank_out_len(self.handle, n, int(j))
            if need < 0 or (o is None and need == 0):
                continue   # the library refuses bad sizes itself, before any launch
            _check_buf(o, torch.complex64, need, f"out[{i}]", x.device)
        n_arr = (ctypes.c_int64 * len(ns))(*ns)
        j_arr = (ctypes.c_int32 * len(ns))(*[int(j) for j in J])
        rx_p = _ptr_array([x.data_ptr() for x in rx])
        out_p = _ptr_array([None if o is None else o.data_ptr() for o in out])
        if workspace is None:
            check(lib().sidwt_bank_correlate(self.handle, rx_p, n_arr, j_arr, out_p, len(ns),
                                             _stream_ptr(stream)), "sidwt_bank_correlate")
        else:
            check(lib().sidwt_bank_correlate_ws(self.handle, workspace.handle, rx_p, n_arr, j_arr,
                                                out_p, len(ns), _stream_ptr(stream)),
                  "sidwt_bank_correlate_ws")
        return out

    def info(self) -> dict:
        v = (ctypes.c_int64 * len(BANK_INFO_KEYS))()
        check(lib().sidwt_bank_info(self.handle, v, len(BANK_INFO_KEYS)), "sidwt_bank_info")
        return dict(zip(BANK_INFO_KEYS, list(v)))

    def free(self):
        if getattr(self, "_h", None) is not None:
            lib().sidwt_bank_free(self._h)
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


class BankWorkspace:
    """Device buffers of one bank call in flight (one per stream)."""

    def __init__(self, handle):
        self._h = handle

    def timing(self, on: bool = True):
        """Record HIP events around the lifting and GEMM launches of calls."""
        check(lib().sidwt_bank_ws_timing(self.handle, int(bool(on))), "sidwt_bank_ws_timing")

    def times(self):
        """(lifting ms, GEMM ms) of the last timed call (waits for it)."""
        a, b = ctypes.c_float(), ctypes.c_float()
        check(lib().sidwt_bank_ws_times(self.handle, ctypes.byref(a), ctypes.byref(b)),
              "sidwt_bank_ws_times")
        return a.value, b.value

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("workspace already freed")
        return self._h

    def free(self):
        if getattr(self, "_h", None) is not None:
            lib().sidwt_bank_ws_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
