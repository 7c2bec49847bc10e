"""Roles-exchanged correlation (redundant analysis on the received pulse,
critical on the reference) on the GPU against the oracle: every plane and
lag at small sizes (ragged lengths, a reference as long as the pulse, tiny
levels), the received-shift covariance the variant exists for, agreement
with the direct form on the common phase, and sampled lags at the benchmark
size in the benchmark's launch configuration."""
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


def crand(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("filt,J,n,m,count", [
    ("cdf97", 3, 1000, 70, 2),      # N = 1000: not a power of two
    ("d4", 4, 520, 33, 3),          # N = 528, ragged tail of zeros
    ("legall53", 2, 64, 64, 2),     # reference as long as the pulse
    ("legall53", 3, 16, 5, 2),      # N / 2^J = 2: tiny levels
    ("cdf97", 5, 4096, 512, 2),     # several tiles and phases per plane
    ("d4", 6, 3000, 200, 1),
    ("cdf97", 1, 300, 40, 2),       # J = 1: plane 0 only, no workspace
])
def test_swapped_matches_oracle(dev, filt, J, n, m, count):
    torch, S = dev
    rng = np.random.default_rng(n + 7 * J)
    ref, rx = crand(rng, m), crand(rng, count, n)
    print(f"[case] swapped {filt} J={J} n={n} m={m} count={count}", flush=True)
    with S.plan_create(filt, J, ref) as plan:
        got = S.correlate_swapped(plan, torch.from_numpy(rx).cuda())
        torch.cuda.synchronize()
        got = got.cpu().numpy().astype(np.complex128)
    for i in range(count):
        want = O.correlate_swapped(filt, J, ref.astype(np.complex128), rx[i].astype(np.complex128))
        for j in range(J):
            assert rel_l2(got[i, j], want[j]) <= 1e-5, (i, j)


@pytest.mark.parametrize("filt,J,n,m,count", [
    ("cdf97", 3, 24576, 100, 2),    # planes too long for one workgroup: chunks of one phase
    ("cdf97", 5, 32768, 512, 1),
    ("d4", 6, 65536, 2048, 1),
    ("legall53", 4, 40000, 300, 1),
])
def test_swapped_long_pulses_sampled(dev, filt, J, n, m, count):
    torch, S = dev
    rng = np.random.default_rng(n + J)
    ref, rx = crand(rng, m), crand(rng, count, n)
    N = O.transform_length(n, J)
    print(f"[case] swapped long {filt} J={J} n={n} m={m}", flush=True)
    with S.plan_create(filt, J, ref) as plan:
        out = S.correlate_swapped(plan, torch.from_numpy(rx).cuda())
        torch.cuda.synchronize()
        got_all = out.cpu().numpy().astype(np.complex128)
    lags = np.concatenate([[0, 1, 15, 16, 511, 512, N - 1], rng.integers(0, N, 25)])
    for i in range(count):
        for j in range(J):
            want = O.correlate_swapped_at(filt, J, ref.astype(np.complex128),
                                          rx[i].astype(np.complex128), j, lags)
            assert rel_l2(got_all[i, j, lags], want) <= 1e-5, (i, j)
    assert np.isfinite(got_all).all()


def test_swapped_is_covariant_in_the_received_shift_on_the_gpu(dev):
    torch, S = dev
    rng = np.random.default_rng(41)
    J, n = 4, 2048
    ref, rx = crand(rng, 120), crand(rng, 1, n)
    shifts = (1, 5, 16, 333)
    batch = np.concatenate([rx] + [np.roll(rx, t, axis=1) for t in shifts])
    print("[case] swapped covariance cdf97 J=4 n=2048", flush=True)
    with S.plan_create("cdf97", J, ref) as plan:
        got = S.correlate_swapped(plan, torch.from_numpy(batch).cuda()).cpu().numpy()
    for k, t in enumerate(shifts, start=1):
        for j in range(J):
            want = np.roll(got[0, j], t)
            assert rel_l2(got[k, j].astype(np.complex128), want.astype(np.complex128)) <= 1e-5


def test_swapped_equals_forward_on_the_common_phase(dev):
    torch, S = dev
    rng = np.random.default_rng(42)
    J, n = 5, 4096
    ref, rx = crand(rng, 300), crand(rng, 2, n)
    print("[case] swapped vs forward, d4 J=5 n=4096", flush=True)
    with S.plan_create("d4", J, ref) as plan:
        sw = S.correlate_swapped(plan, torch.from_numpy(rx).cuda()).cpu().numpy()
        fw = S.correlate_many(plan, torch.from_numpy(rx).cuda()).cpu().numpy()
    for j in range(J):
        s = np.arange(0, n, 1 << j)
        assert rel_l2(sw[:, j, s].astype(np.complex128), fw[:, j, s].astype(np.complex128)) <= 1e-5


def test_swapped_full_size_sampled(dev):
    torch, S = dev
    count, n, J = 4096, 8192, 5
    print("[case] swapped batched uniform 4096 x 8192 cdf97 J=5", flush=True)
    b = W.batched_uniform(seed=2, count=count, n=n, m=512, J=J)
    with S.plan_create(b.filter, J, b.ref) as plan:
        out = S.correlate_swapped(plan, torch.from_numpy(b.rx).cuda())
        torch.cuda.synchronize()
        rng = np.random.default_rng(0)
        for i in (0, 1, 2047, 4095):
            lags = np.concatenate([[0, 1, 2, 31, n - 1], rng.integers(0, n, 40)])
            got = out[i][:, lags].cpu().numpy().astype(np.complex128)
            for j in range(J):
                want = O.correlate_swapped_at(b.filter, J, b.ref, b.rx[i].astype(np.complex128), j,
                                              lags)
                assert rel_l2(got[j], want) <= 1e-5, (i, j)
        assert torch.isfinite(torch.view_as_real(out)).all().item()


def test_swapped_refuses_what_it_cannot_do(dev):
    torch, S = dev
    rng = np.random.default_rng(43)
    ref = crand(rng, 50)
    with S.plan_create("cdf97", 3, ref) as plan:
        rx = torch.from_numpy(crand(rng, 2, 512)).cuda()
        small = torch.empty(16, dtype=torch.uint8, device="cuda")
        with pytest.raises(S.SidwtError):
            S.correlate_swapped(plan, rx, workspace=small)
    # a reference whose weights and window exceed the LDS even in chunks
    with S.plan_create("cdf97", 3, crand(rng, 8192)) as plan:
        big = torch.zeros((1, 40000), dtype=torch.complex64, device="cuda")
        with pytest.raises(S.SidwtError):
            S.correlate_swapped(plan, big)
    iq = rng.integers(-100, 100, (20, 2)).astype(np.int16)
    with S.plan_create("legall53_int", 2, iq) as plan:
        import ctypes
        rc = S._lib.lib().sidwt_correlate_swapped(plan.handle, None, 64, 0, 64, None, 128, None, 0)
        assert rc == -5


def test_swapped_through_the_c_abi_with_padded_strides(dev):
    """rx_stride > n and out_stride > J N: rows of a padded batch, output
    planes at a padded pitch (the padding left untouched)."""
    import ctypes
    torch, S = dev
    rng = np.random.default_rng(44)
    J, n, m, count = 3, 1000, 60, 3
    N = O.transform_length(n, J)
    ref = crand(rng, m)
    rx = crand(rng, count, n)
    rxp = np.zeros((count, n + 37), np.complex64)
    rxp[:, :n] = rx
    rxp[:, n:] = 7 + 7j                      # must not be read
    ostride = J * N + 100
    out = torch.full((count, ostride), 3 + 3j, dtype=torch.complex64, device="cuda")
    rx_t = torch.from_numpy(rxp).cuda()
    with S.plan_create("cdf97", J, ref) as plan:
        L = S._lib.lib()
        ws = torch.empty(L.sidwt_swap_workspace_bytes(plan.handle, n, count), dtype=torch.uint8,
                         device="cuda")
        rc = L.sidwt_correlate_swapped(plan.handle, ctypes.c_void_p(rx_t.data_ptr()), n, count,
                                       n + 37, ctypes.c_void_p(out.data_ptr()), ostride,
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel())
        assert rc == 0
        torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(got[:, J * N:] == np.complex64(3 + 3j))
    for i in range(count):
        want = O.correlate_swapped("cdf97", J, ref.astype(np.complex128), rx[i].astype(np.complex128))
        for j in range(J):
            assert rel_l2(got[i, j * N:(j + 1) * N].astype(np.complex128), want[j]) <= 1e-5


def test_swapped_size_guards(dev):
    """Grids and workspaces beyond what one launch or one int64 can address
    are refused on the host (count = 0 is not needed for the check)."""
    torch, S = dev
    rng = np.random.default_rng(46)
    L = S._lib.lib()
    with S.plan_create("cdf97", 12, crand(rng, 64)) as plan:
        # count * 2^(J-1) tree workgroups above 2^31
        assert L.sidwt_correlate_swapped(plan.handle, None, 1 << 14, 1 << 20, 1 << 14, None,
                                         12 << 14, None, 0) == -2
        assert L.sidwt_swap_workspace_bytes(plan.handle, 1 << 30, (1 << 31) - 1) == -1
