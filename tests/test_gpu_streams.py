"""One plan shared by calls on several streams at once: the per-call-stream
entry points leave the plan untouched, so two host threads issuing
correlations with one plan on two torch streams get, bit for bit, what one
stream alone gives (float and integer plans, the roles-exchanged form with
one workspace per stream, and a pulse on the tiled path)."""
import threading

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


def _two_threads(torch, work, reps=6):
    """Run work(stream, k) for k < reps in each of two threads, each with
    its own stream; returns the results per thread."""
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    results = [[None] * reps, [None] * reps]
    errors = []
    barrier = threading.Barrier(2)

    def body(t):
        try:
            torch.cuda.set_device(0)
            barrier.wait()
            with torch.cuda.stream(streams[t]):
                for k in range(reps):
                    results[t][k] = work(streams[t], k)
            streams[t].synchronize()
        except Exception as e:  # noqa: BLE001
            errors.append(e)
    th = [threading.Thread(target=body, args=(t,)) for t in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    return results


def test_float_plan_on_two_streams_matches_one_stream(dev):
    torch, S = dev
    print("[case] cdf97 J=5 4 x 8 x 8192 on two streams", flush=True)
    b = W.batched_uniform(seed=2, count=32, n=8192, m=512, J=5)
    rx = torch.from_numpy(b.rx).cuda()
    with S.plan_create(b.filter, b.J, b.ref) as plan:
        want = [S.correlate_many(plan, rx[8 * k:8 * k + 8]) for k in range(4)]
        torch.cuda.synchronize()
        want = [w.cpu() for w in want]
        res = _two_threads(torch, lambda st, k: S.correlate_many(plan, rx[8 * (k % 4):8 * (k % 4) + 8],
                                                                 stream=st))
        torch.cuda.synchronize()
        for t in range(2):
            for k, got in enumerate(res[t]):
                assert torch.equal(got.cpu(), want[k % 4]), (t, k)
        # sanity: the shared result is the oracle's
        want0 = O.correlate_at(b.filter, b.J, b.ref, b.rx[0].astype(np.complex128), 0,
                               np.arange(0, 8192, 97))
        got0 = want[0][0, 0].numpy()[np.arange(0, 8192, 97)]
        assert np.abs(got0 - want0).max() <= 1e-4 * np.abs(want0).max()


def test_integer_plan_on_two_streams_matches_one_stream(dev):
    torch, S = dev
    print("[case] legall53_int J=6 16 x 4096 on two streams", flush=True)
    ib = W.integer_batch(seed=3, count=16, n=4096, m=512, J=6)
    rx = torch.from_numpy(ib.rx_iq).cuda()
    with S.plan_create("legall53_int", 6, ib.ref_iq) as plan:
        want = S.correlate_many(plan, rx)
        torch.cuda.synchronize()
        want = want.cpu()
        res = _two_threads(torch, lambda st, k: S.correlate_many(plan, rx, stream=st), reps=3)
        for t in range(2):
            for got in res[t]:
                assert torch.equal(got.cpu(), want)


def test_swapped_on_two_streams_matches_one_stream(dev):
    torch, S = dev
    print("[case] swapped cdf97 J=4 8 x 2048 on two streams", flush=True)
    b = W.batched_uniform(seed=2, count=8, n=2048, m=256, J=4)
    rx = torch.from_numpy(b.rx).cuda()
    with S.plan_create(b.filter, b.J, b.ref) as plan:
        want = S.correlate_swapped(plan, rx).cpu()
        res = _two_threads(torch, lambda st, k: S.correlate_swapped(plan, rx, stream=st), reps=3)
        for t in range(2):
            for got in res[t]:
                assert torch.equal(got.cpu(), want)


def test_tiled_pulse_on_two_streams_matches_one_stream(dev):
    torch, S = dev
    n = 50000   # beyond one workgroup's LDS: the tiled path
    print(f"[case] cdf97 J=8 one pulse n={n} on two streams", flush=True)
    rng = np.random.default_rng(11)
    ref = W.lfm_chirp(700, 175.0)
    y = W.echoes(n, ref, rng).astype(np.complex64)
    x = torch.from_numpy(y).cuda()
    with S.plan_create("cdf97", 8, ref) as plan:
        want = S.correlate(plan, x).cpu()
        res = _two_threads(torch, lambda st, k: S.correlate(plan, x, stream=st), reps=2)
        for t in range(2):
            for got in res[t]:
                assert torch.equal(got.cpu(), want)
        lags = np.array([0, 1, 12345, S.transform_length(n, 8) - 1])
        for j in (0, 7):
            w = O.correlate_at("cdf97", 8, ref, y.astype(np.complex128), j, lags)
            g = want[j].numpy()[lags]
            assert np.abs(g - w).max() <= 1e-4 * np.abs(w).max()


def test_binding_uses_the_current_stream(dev):
    """The binding's default stream is torch's current stream of the
    current device, also inside a stream context."""
    torch, S = dev

    def ptr(p):  # the null (default) stream reads back as None
        return p.value or 0

    assert ptr(S._stream_ptr()) == torch.cuda.current_stream().cuda_stream
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        assert ptr(S._stream_ptr()) == s.cuda_stream != 0
    assert ptr(S._stream_ptr(s)) == s.cuda_stream
