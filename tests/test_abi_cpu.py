"""CPU-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sidwt.h")
LIB = os.path.join(ROOT, "paper_cs_0607001_amd", "libsidwt.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sidwt_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.skip("libsidwt.so not built")
    from paper_cs_0607001_amd._lib import lib
    return lib()


def test_header_declares_the_core_api():
    names = declared_functions()
    for want in ("sidwt_plan_create", "sidwt_correlate", "sidwt_free", "sidwt_out_len",
                 "sidwt_set_stream", "sidwt_correlate_batch", "sidwt_strerror"):
        assert want in names


def test_library_exports_every_declared_symbol(L):
    raw = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, missing


def test_strerror_and_version(L):
    assert L.sidwt_strerror(0) == b"ok"
    assert L.sidwt_strerror(-1) == b"invalid argument"
    assert L.sidwt_strerror(-2).startswith(b"size")
    assert L.sidwt_version().startswith(b"sidwt")


def test_invalid_arguments_are_rejected_on_the_host(L):
    vp = ctypes.c_void_p
    h = vp()
    ref = (ctypes.c_float * 8)()
    # unknown filter, NULL ref, NULL out, bad J, bad m
    assert L.sidwt_plan_create(9, 3, ctypes.cast(ref, vp), 4, ctypes.byref(h)) == -1
    assert L.sidwt_plan_create(1, 3, None, 4, ctypes.byref(h)) == -1
    assert L.sidwt_plan_create(1, 3, ctypes.cast(ref, vp), 4, None) == -1
    assert L.sidwt_plan_create(1, 0, ctypes.cast(ref, vp), 4, ctypes.byref(h)) == -1
    assert L.sidwt_plan_create(1, 17, ctypes.cast(ref, vp), 4, ctypes.byref(h)) == -1
    assert L.sidwt_plan_create(1, 3, ctypes.cast(ref, vp), 0, ctypes.byref(h)) == -1
    assert L.sidwt_plan_create(1, 3, ctypes.cast(ref, vp), 1 << 20, ctypes.byref(h)) == -2
    assert h.value is None
    # NULL plan everywhere
    assert L.sidwt_correlate(None, vp(16), 8, vp(16)) == -1
    assert L.sidwt_correlate_many(None, vp(16), 8, 1, 8, vp(16), 8) == -1
    assert L.sidwt_out_len(None, 8) == -1
    assert L.sidwt_set_stream(None, None) == -1
    L.sidwt_free(None)  # no-op
    # lifting-only entry: NULL pointers, bad filter, N/2^J < 2, stride < n
    assert L.sidwt_lift_many(1, 3, None, 64, 1, 64, vp(16), None) == -1
    assert L.sidwt_lift_many(7, 3, vp(16), 64, 1, 64, vp(16), None) == -1
    assert L.sidwt_lift_many(1, 3, vp(16), 8, 1, 8, vp(16), None) == -1
    assert L.sidwt_lift_many(1, 3, vp(16), 64, 1, 32, vp(16), None) == -1
    assert L.sidwt_lift_many(1, 3, vp(16), 64, -1, 64, vp(16), None) == -1


def test_zero_pulses_is_a_no_op(L):
    # sizes are still checked; nothing is launched, so no device is needed
    assert L.sidwt_lift_many(2, 3, None, 64, 0, 64, None, None) == 0
    assert L.sidwt_lift_many(2, 3, None, 8, 0, 8, None, None) == -1   # N / 2^J < 2
    assert L.sidwt_bank_correlate(None, None, None, None, None, 0, None) == -1


def test_integer_plans_that_could_lose_exactness_are_refused(L):
    """A full-scale int16 reference at J = 16: the level-16 bound on the
    partial sums (pulse approximations doubling per level, reference
    approximations growing by 3/2, details within 2X + 1 of their input
    bound) passes 2^53, so the plan is refused on the host; a small
    reference peak keeps the same plan under it."""
    vp = ctypes.c_void_p
    m = 64
    loud = (ctypes.c_int16 * (2 * m))(*([32767, -32768] * m))
    quiet = (ctypes.c_int16 * (2 * m))(*([100, -100] * m))
    h = vp()
    assert L.sidwt_plan_create(4, 16, ctypes.cast(loud, vp), m, ctypes.byref(h)) == -2
    assert h.value is None
    rc = L.sidwt_plan_create(4, 16, ctypes.cast(quiet, vp), m, ctypes.byref(h))
    assert rc != -2      # -4 without a device
    if rc == 0:
        L.sidwt_free(h)
    rc = L.sidwt_plan_create(4, 8, ctypes.cast(loud, vp), m, ctypes.byref(h))
    assert rc != -2
    if rc == 0:
        L.sidwt_free(h)


def test_synthesis_arguments_are_checked_on_the_host(L):
    vp = ctypes.c_void_p
    assert L.sidwt_synth_many(2, 3, 3, vp(16), 64, 1, vp(16), None) == -1    # to >= J
    assert L.sidwt_synth_many(2, 3, -1, vp(16), 64, 1, vp(16), None) == -1   # to < 0
    assert L.sidwt_synth_many(2, 3, 0, vp(16), 60, 1, vp(16), None) == -1    # N % 2^J
    assert L.sidwt_synth_many(9, 3, 0, vp(16), 64, 1, vp(16), None) == -1    # filter
    assert L.sidwt_synth_many(2, 3, 0, None, 64, 0, None, None) == 0         # nothing to do
    assert L.sidwt_synth_many(2, 3, 0, vp(16), 1 << 20, 1, vp(16), None) == -5  # LDS
    # 1.5 (N >> (to+1)) complex elements in LDS: 26624 fits in 160 KB, 27648 does not
    assert L.sidwt_synth_many(2, 5, 0, None, 26624, 0, None, None) == 0
    assert L.sidwt_synth_many(2, 5, 0, None, 27648, 0, None, None) == -5
    assert L.sidwt_synth_many(2, 5, 1, None, 27648, 0, None, None) == 0


def test_plane_mask_entry_rejects_a_null_plan(L):
    vp = ctypes.c_void_p
    assert L.sidwt_correlate_planes(None, vp(16), 64, 1, 64, vp(16), 3 * 64, 1) == -1


def test_swapped_entry_points_reject_a_null_plan(L):
    vp = ctypes.c_void_p
    assert L.sidwt_swap_workspace_bytes(None, 64, 1) == -1
    assert L.sidwt_correlate_swapped(None, vp(16), 64, 1, 64, vp(16), 192, vp(16), 1 << 20) == -1
    assert L.sidwt_correlate_swapped_on(None, vp(16), 64, 1, 64, vp(16), 192, vp(16), 1 << 20,
                                        None) == -1


def test_stream_per_call_entry_points_reject_a_null_plan(L):
    vp = ctypes.c_void_p
    assert L.sidwt_correlate_on(None, vp(16), 64, vp(16), None) == -1
    assert L.sidwt_correlate_many_on(None, vp(16), 64, 1, 64, vp(16), 192, 0xFFFFFFFF, None) == -1


def test_detect_arguments_are_checked_on_the_host(L):
    vp = ctypes.c_void_p
    nan = float("nan")
    assert L.sidwt_detect_peaks(None, 0, 3, 64, 192, 0.1, 8, None, None, None, None) == 0
    assert L.sidwt_detect_peaks(vp(16), 1, 3, 64, 191, 0.1, 8, vp(16), vp(16), vp(16), None) == -1
    assert L.sidwt_detect_peaks(vp(16), 1, 3, 64, 192, nan, 8, vp(16), vp(16), vp(16), None) == -1
    assert L.sidwt_detect_peaks(vp(16), 1, 3, 64, 192, -1.0, 8, vp(16), vp(16), vp(16), None) == -1
    assert L.sidwt_detect_peaks(vp(16), 1, 3, 64, 192, 0.1, -1, vp(16), vp(16), vp(16), None) == -1
    assert L.sidwt_detect_peaks(vp(16), 1, 3, 64, 192, 0.1, 8, None, vp(16), vp(16), None) == -1
