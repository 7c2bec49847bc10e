"""Shift equivariance of the GPU planes, in exactly the forms the method
guarantees (checked on the oracle in the pins): delaying the reference by
any t moves every plane by -t lags; delaying (circularly) the received pulse
by a multiple of 2^J moves every plane by +t; plane 0 follows any delay of
the pulse.  Float filters within 1e-5 relative L2 per plane (the GPU sums in
a different order for the shifted input), the integer filter bit for bit;
also at the benchmark size, compared on the device."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_cs_0607001_amd as S
    S._lib.lib()
    return torch, S


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def rel_err(torch, a, b):
    """Worst relative L2 error over planes (last axis is the lag)."""
    d = torch.linalg.vector_norm((a - b).reshape(-1, a.shape[-1]).to(torch.complex128), dim=-1)
    r = torch.linalg.vector_norm(b.reshape(-1, b.shape[-1]).to(torch.complex128), dim=-1)
    return float((d / r).max())


@pytest.mark.parametrize("filt", ["legall53", "cdf97", "d4"])
def test_float_shift_equivariance(dev, filt):
    torch, S = dev
    rng = np.random.default_rng(21)
    J, count, n, m = 5, 6, 4096, 300     # n a multiple of 2^J: the delay is circular over N
    ref = crandn(rng, m)
    rx = torch.from_numpy(crandn(rng, count, n)).cuda()
    print(f"[case] shift equivariance {filt}", flush=True)
    with S.plan_create(filt, J, ref) as plan:
        R = S.correlate_many(plan, rx)
        # (i) the reference delayed by t: every plane moves by -t
        t = 37
        with S.plan_create(filt, J, np.concatenate([np.zeros(t, np.complex64), ref])) as pd:
            Rd = S.correlate_many(pd, rx)
        assert rel_err(torch, Rd, torch.roll(R, -t, dims=-1)) <= 1e-5
        # (ii) the pulse delayed by a multiple of 2^J: every plane moves by +t
        t = 3 << J
        Ry = S.correlate_many(plan, torch.roll(rx, t, dims=-1).contiguous())
        assert rel_err(torch, Ry, torch.roll(R, t, dims=-1)) <= 1e-5
        # (iii) plane 0 follows any delay of the pulse
        t = 5
        R0 = S.correlate_many(plan, torch.roll(rx, t, dims=-1).contiguous())
        assert rel_err(torch, R0[:, 0], torch.roll(R[:, 0], t, dims=-1)) <= 1e-5
        torch.cuda.synchronize()
    # and the planes themselves against the oracle on one pulse
    want = O.correlate_direct(filt, J, ref, rx[1].cpu().numpy())
    got = R[1].cpu().numpy()
    for j in range(J):
        assert np.linalg.norm(got[j] - want[j]) <= 1e-5 * np.linalg.norm(want[j]), j


def test_integer_shift_equivariance_is_exact(dev):
    torch, S = dev
    rng = np.random.default_rng(22)
    J, count, n, m = 6, 4, 4096, 200
    ref = rng.integers(-2047, 2048, (m, 2)).astype(np.int16)
    rx = torch.from_numpy(rng.integers(-32768, 32768, (count, n, 2)).astype(np.int16)).cuda()
    print("[case] integer shift equivariance", flush=True)
    with S.plan_create("legall53_int", J, ref) as plan:
        R = S.correlate_many(plan, rx)
        t = 7
        refd = np.concatenate([np.zeros((t, 2), np.int16), ref])
        with S.plan_create("legall53_int", J, refd) as pd:
            Rd = S.correlate_many(pd, rx)
        assert torch.equal(Rd, torch.roll(R, -t, dims=-2))
        t = 5 << J
        Ry = S.correlate_many(plan, torch.roll(rx, t, dims=-2).contiguous())
        assert torch.equal(Ry, torch.roll(R, t, dims=-2))
        torch.cuda.synchronize()
    assert np.array_equal(R[2].cpu().numpy(), O.correlate_int(J, ref, rx[2].cpu().numpy()))


def test_shift_equivariance_at_the_benchmark_size(dev):
    """4096 pulses x 8192, CDF 9/7, J = 5 (the bench launch): the pulse batch
    delayed by 32 samples gives every plane delayed by 32 lags."""
    torch, S = dev
    import workloads as W
    b = W.batched_uniform(seed=2, count=4096, n=8192, m=512, J=5)
    rx = torch.from_numpy(b.rx).cuda()
    print("[case] shift equivariance 4096 x 8192", flush=True)
    with S.plan_create(b.filter, 5, b.ref) as plan:
        R = S.correlate_many(plan, rx)
        Ry = S.correlate_many(plan, torch.roll(rx, 32, dims=-1).contiguous())
        torch.cuda.synchronize()
        err = 0.0
        for k in range(0, 4096, 512):   # in slices, to keep the temporaries small
            err = max(err, rel_err(torch, Ry[k:k + 512], torch.roll(R[k:k + 512], 32, dims=-1)))
        assert err <= 1e-5, err
