"""The entry point that allocates nothing (sidwt_correlate_swapped_noalloc),
called through the C ABI: its output equals, bit for bit, that of
sidwt_correlate_swapped_on with a caller workspace (the same kernels), on
two calls in a row, the second with a smaller input; a request whose tree
exceeds the library's static scratch is refused before anything runs; and
the result stays within the float tolerance of the oracle."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_cs_0607001_amd as S
    S._lib.lib()
    return torch, S


def _noalloc(S, plan, rx, out, stream):
    vp = ctypes.c_void_p
    count, n = rx.shape
    N = S.transform_length(n, plan.J)
    return S._lib.lib().sidwt_correlate_swapped_noalloc(
        plan.handle, vp(rx.data_ptr()), n, count, n, vp(out.data_ptr()), plan.J * N,
        vp(stream.cuda_stream))


def _with_workspace(S, plan, rx, out, stream):
    torch = __import__("torch")
    vp = ctypes.c_void_p
    L = S._lib.lib()
    count, n = rx.shape
    N = S.transform_length(n, plan.J)
    need = L.sidwt_swap_workspace_bytes(plan.handle, n, count)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=rx.device)
    rc = L.sidwt_correlate_swapped_on(plan.handle, vp(rx.data_ptr()), n, count, n,
                                      vp(out.data_ptr()), plan.J * N, vp(ws.data_ptr()),
                                      ws.numel(), vp(stream.cuda_stream))
    return rc, ws


def test_noalloc_matches_the_workspace_entry_point_on_two_calls(dev):
    torch, S = dev
    stream = torch.cuda.current_stream()
    cases = [(24, 8192, 512, 5), (5, 2000, 200, 4)]   # second call: smaller input
    for count, n, m, J in cases:
        print(f"[case] noalloc swapped cdf97 count={count} n={n} m={m} J={J}", flush=True)
        b = W.batched_uniform(seed=7, count=count, n=n, m=m, J=J)
        rx = torch.from_numpy(b.rx).cuda()
        N = S.transform_length(n, J)
        with S.plan_create(b.filter, J, b.ref) as plan:
            out_a = torch.full((count, J, N), complex(7, 7), dtype=torch.complex64, device="cuda")
            out_b = torch.full((count, J, N), complex(-3, 1), dtype=torch.complex64, device="cuda")
            assert _noalloc(S, plan, rx, out_a, stream) == 0
            rc, ws = _with_workspace(S, plan, rx, out_b, stream)
            assert rc == 0
            torch.cuda.synchronize()
            assert torch.equal(out_a, out_b)
            got = out_a.cpu().numpy()
            i = count - 1
            want = O.correlate_swapped_at(b.filter, J, b.ref, b.rx[i].astype(np.complex128), J - 1,
                                          np.arange(0, N, 37))
            g = got[i, J - 1, np.arange(0, N, 37)]
            assert np.linalg.norm(g - want) <= 1e-5 * np.linalg.norm(want)
            del ws


def test_noalloc_refuses_requests_beyond_its_scratch(dev):
    torch, S = dev
    L = S._lib.lib()
    vp = ctypes.c_void_p
    b = W.batched_uniform(seed=7, count=1, n=8192, m=512, J=5)
    with S.plan_create(b.filter, 5, b.ref) as plan:
        limit = 64 << 20
        per_pulse = L.sidwt_swap_workspace_bytes(plan.handle, 8192, 1)
        fits = limit // per_pulse
        assert L.sidwt_swap_workspace_bytes(plan.handle, 8192, fits) <= limit
        # one pulse more than fits: refused before any pointer is read
        assert L.sidwt_correlate_swapped_noalloc(plan.handle, vp(16), 8192, fits + 1, 8192,
                                                 vp(16), 5 * 8192, None) == -6
        assert L.sidwt_strerror(-6).startswith(b"request needs more")
