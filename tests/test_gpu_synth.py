"""Coarse-to-fine formation (the inverse y-side lifting of eq. (21)) on the
GPU against the oracle: from an oracle-computed pyramid to every finer
approximation, and end to end (lift_many, then synth_many back to the
zero-padded pulse)."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

FLOAT = ["legall53", "cdf97", "d4"]


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_cs_0607001_amd as S
    S._lib.lib()
    return torch, S


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def oracle_pyramid(filt, J, u):
    """(details, approximations) of the y-side lifting of each row of u."""
    c, details, approx = u, [], [u]
    for _ in range(J):
        c, d = O.i2i_lift_y(c) if filt == "legall53_int" else O.lift_y(filt, c)
        details.append(d)
        approx.append(c)
    return details, approx


@pytest.mark.parametrize("filt,J,N", [("legall53", 3, 1024), ("cdf97", 5, 4096),
                                      ("d4", 4, 8192), ("cdf97", 6, 640), ("d4", 5, 192),
                                      ("d4", 3, 16), ("legall53", 4, 32), ("cdf97", 2, 8),
                                      ("cdf97", 5, 26624)])   # the largest c_0 in LDS
def test_synthesis_from_oracle_pyramid(dev, filt, J, N):
    torch, S = dev
    rng = np.random.default_rng(J * 100 + N % 97)
    u = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    details, approx = oracle_pyramid(filt, J, u)
    pyr = np.concatenate(details + [approx[J]], axis=-1).astype(np.complex64)
    print(f"[case] synth {filt} J={J} N={N}", flush=True)
    for to in sorted({0, 1, J - 1}):
        got = S.synth_many(filt, J, torch.from_numpy(pyr).cuda(), to=to)
        torch.cuda.synchronize()
        want = O.synthesize_y(filt, details, approx[J], to)
        for i in range(3):
            assert rel_l2(got[i].cpu().numpy().astype(np.complex128), want[i]) <= 1e-5, (to, i)


def test_integer_synthesis_is_bit_exact(dev):
    torch, S = dev
    rng = np.random.default_rng(4)
    J, N = 6, 4096
    re = rng.integers(-2048, 2048, (5, N))
    im = rng.integers(-2048, 2048, (5, N))
    dre, are = oracle_pyramid("legall53_int", J, re)
    dim, aim = oracle_pyramid("legall53_int", J, im)
    pyr = np.stack([np.concatenate(dre + [are[J]], -1), np.concatenate(dim + [aim[J]], -1)],
                   -1).astype(np.int32)
    print("[case] synth integer 5/3 J=6 N=4096", flush=True)
    for to in (0, 2, J - 1):
        got = S.synth_many("legall53_int", J, torch.from_numpy(pyr).cuda(), to=to)
        torch.cuda.synchronize()
        g = got.cpu().numpy()
        assert np.array_equal(g[..., 0], are[to]) and np.array_equal(g[..., 1], aim[to]), to


@pytest.mark.parametrize("filt", FLOAT + ["legall53_int"])
def test_lift_then_synthesize_returns_the_pulse(dev, filt):
    torch, S = dev
    rng = np.random.default_rng(7)
    J, n = 5, 3000                        # N = 3008: the padding comes back as zeros
    N = O.transform_length(n, J)
    print(f"[case] round trip {filt} n={n}", flush=True)
    if filt == "legall53_int":
        rx = rng.integers(-2048, 2048, (4, n, 2)).astype(np.int16)
        pyr = S.lift_many(filt, J, torch.from_numpy(rx).cuda())
        back = S.synth_many(filt, J, pyr, to=0).cpu().numpy()
        want = np.zeros((4, N, 2), np.int64)
        want[:, :n] = rx
        assert np.array_equal(back, want)
    else:
        rx = (rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))).astype(np.complex64)
        pyr = S.lift_many(filt, J, torch.from_numpy(rx).cuda())
        back = S.synth_many(filt, J, pyr, to=0).cpu().numpy().astype(np.complex128)
        for i in range(4):
            want = O.zero_pad(rx[i].astype(np.complex128), N)
            assert rel_l2(back[i], want) <= 1e-5, i


def test_synthesis_full_size_round_trips(dev):
    """At the benchmark sizes and launch configuration: lift_many then
    synth_many over the whole batch gives every sampled pulse back (FP32
    within 1e-5; the reversible integer filter bit for bit)."""
    torch, S = dev
    import workloads as W
    print("[case] synthesis round trip 4096 x 8192 cdf97 J=5", flush=True)
    b = W.batched_uniform(seed=2, count=4096, n=8192, m=512, J=5)
    rx = torch.from_numpy(b.rx).cuda()
    back = S.synth_many("cdf97", 5, S.lift_many("cdf97", 5, rx), to=0)
    torch.cuda.synchronize()
    for i in (0, 1, 2047, 4095):
        got = back[i].cpu().numpy().astype(np.complex128)
        assert rel_l2(got, b.rx[i].astype(np.complex128)) <= 1e-5, i
    del rx, back
    print("[case] synthesis round trip 16384 x 4096 integer 5/3 J=6", flush=True)
    ib = W.integer_batch(seed=3, count=16384, n=4096, m=512, J=6)
    rxi = torch.from_numpy(ib.rx_iq).cuda()
    backi = S.synth_many("legall53_int", 6, S.lift_many("legall53_int", 6, rxi), to=0)
    torch.cuda.synchronize()
    for i in (0, 8191, 16383):
        assert np.array_equal(backi[i].cpu().numpy(), ib.rx_iq[i].astype(np.int64)), i
