"""Target declaration on the GPU: bit-exact lags and counts against the
oracle's detector on the same single-precision planes (oracle-made planes
of the five-target scene, random planes with exact ties and flat tops,
lengths below and across the block size), truncation at max_peaks, the
scene end to end through the correlation kernel, and the benchmark-size
planes checked against the local-maximum property."""
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


def compare(S, torch, planes, level_db, max_peaks=64):
    lags, db, found = S.detect_peaks(torch.from_numpy(planes).cuda(), level_db, max_peaks)
    lags, db, found = lags.cpu().numpy(), db.cpu().numpy(), found.cpu().numpy()
    rel = np.float32(10.0 ** (level_db / 10.0))
    count, J, N = planes.shape
    want = O.detect_peaks(planes, rel, max_peaks)
    for k, (wl, wd) in enumerate(want):
        i, j = divmod(k, J)
        assert found[i, j] == len(wl), (i, j)
        n = min(len(wl), max_peaks)
        assert np.array_equal(lags[i, j, :n], wl[:n]), (i, j)
        assert np.abs(db[i, j, :n] - wd[:n]).max(initial=0.0) < 1e-3, (i, j)
    return found


def test_detect_on_oracle_planes_of_the_scene(dev):
    torch, S = dev
    sc = W.multi_target(seed=5, count=3)
    planes = np.stack([O.correlate_direct(sc.filter, sc.J, sc.ref, sc.rx[i].astype(np.complex128))
                       for i in range(3)]).astype(np.complex64)
    print("[case] detect on oracle planes, five-target scene", flush=True)
    for level in (-10.0, -20.0, -3.0):
        compare(S, torch, planes, level)


@pytest.mark.parametrize("N", [3, 17, 64, 255, 256, 257, 1000, 2047, 2048, 2049, 4096, 40896, 40897, 50000])
def test_detect_random_planes_with_ties(dev, N):
    torch, S = dev
    rng = np.random.default_rng(N)
    planes = (rng.standard_normal((2, 3, N)) + 1j * rng.standard_normal((2, 3, N))).astype(
        np.complex64)
    planes[0, 1, :] = planes[0, 1, 0]                    # constant: no peak
    if N > 5:
        planes[1, 0, N // 2] = planes[1, 0, N // 2 + 1] = 10 + 0j   # flat top
        planes[1, 2, 0] = 20j                                          # peak at lag 0
        planes[1, 2, N - 1] = 5
    planes[0, 2, :] = 0                                  # all zero
    print(f"[case] detect random planes N={N}", flush=True)
    for level in (-100.0, -6.0, 0.0):
        compare(S, torch, planes, level)


def test_detect_truncates_at_max_peaks(dev):
    torch, S = dev
    rng = np.random.default_rng(9)
    planes = (rng.standard_normal((2, 2, 700)) + 1j * rng.standard_normal((2, 2, 700))).astype(
        np.complex64)
    found = compare(S, torch, planes, -100.0, max_peaks=3)
    assert (found > 3).all()
    lags, _, f0 = S.detect_peaks(torch.from_numpy(planes).cuda(), -100.0, 0)
    assert np.array_equal(f0.cpu().numpy(), found)


def test_scene_end_to_end_resolves_the_five_targets(dev):
    torch, S = dev
    sc = W.multi_target(seed=5, count=8)
    print("[case] five-target scene through correlate_many + detect", flush=True)
    with S.plan_create(sc.filter, sc.J, sc.ref) as plan:
        planes = S.correlate_many(plan, torch.from_numpy(sc.rx).cuda())
        lags, db, found = S.detect_peaks(planes, -10.0, 32)
    lags, found = lags.cpu().numpy(), found.cpu().numpy()
    for i in range(8):
        got = set(lags[i, 0, :found[i, 0]].tolist())
        assert set(sc.delays[i].tolist()) <= got, (i, sorted(got), sc.delays[i])


def test_detect_full_size_property(dev):
    torch, S = dev
    count, n, J = 4096, 8192, 5
    print("[case] detect on the 4096 x 8192 planes", flush=True)
    b = W.batched_uniform(seed=2, count=count, n=n, m=512, J=J)
    with S.plan_create(b.filter, J, b.ref) as plan:
        planes = S.correlate_many(plan, torch.from_numpy(b.rx).cuda())
        lags, db, found = S.detect_peaks(planes, -10.0, 64)
        torch.cuda.synchronize()
        f = found.cpu().numpy()
        assert (f >= 1).all()
        for i in (0, 1, 2047, 4095):
            P = planes[i].cpu().numpy()
            re, im = P.real.astype(np.float32), P.imag.astype(np.float32)
            p = re * re + im * im
            thr = np.float32(10.0 ** -1.0) * p.max(axis=1)
            pk = (p > np.roll(p, 1, 1)) & (p >= np.roll(p, -1, 1)) & (p >= thr[:, None])
            L = lags[i].cpu().numpy()
            for j in range(J):
                want = np.nonzero(pk[j])[0]
                assert f[i, j] == len(want)
                assert np.array_equal(L[j, :min(64, len(want))], want[:64])


def test_detect_through_the_c_abi_with_a_padded_pulse_stride(dev):
    import ctypes
    torch, S = dev
    rng = np.random.default_rng(45)
    count, J, N = 3, 2, 300
    planes = (rng.standard_normal((count, J, N)) + 1j * rng.standard_normal((count, J, N))).astype(
        np.complex64)
    pitch = J * N + 50
    padded = np.full((count, pitch), 100 + 0j, np.complex64)    # a tall peak in the padding
    padded[:, :J * N] = planes.reshape(count, J * N)
    pt = torch.from_numpy(padded).cuda()
    lags = torch.empty((count * J * 16,), dtype=torch.int32, device="cuda")
    db = torch.empty((count * J * 16,), dtype=torch.float32, device="cuda")
    found = torch.empty((count * J,), dtype=torch.int32, device="cuda")
    rel = np.float32(10.0 ** (-6.0 / 10.0))
    rc = S._lib.lib().sidwt_detect_peaks(ctypes.c_void_p(pt.data_ptr()), count, J, N, pitch,
                                         float(rel), 16, ctypes.c_void_p(lags.data_ptr()),
                                         ctypes.c_void_p(db.data_ptr()),
                                         ctypes.c_void_p(found.data_ptr()), None)
    assert rc == 0
    lags, found = lags.cpu().numpy().reshape(count, J, 16), found.cpu().numpy().reshape(count, J)
    want = O.detect_peaks(planes, rel, 16)
    for k, (wl, _) in enumerate(want):
        i, j = divmod(k, J)
        assert found[i, j] == len(wl)
        assert np.array_equal(lags[i, j, :min(16, len(wl))], wl[:16])
