"""Uneven batches through the persistent kernel: parity with the oracle for
whole-pulse and tiled pulses, agreement between work splits, graph replay."""
import math

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


LENGTHS = [300, 517, 1500, 2100, 5000, 9000, 17000, 33000, 65536]


def make_batch(S, torch, seed=41):
    rng = np.random.default_rng(seed)
    refs = W.reference_set(seed, count=5, m_lo=40, m_hi=600)
    plans, rx, meta = [], [], []
    cache = {}
    for i, n in enumerate(LENGTHS):
        J = W.levels_for(n)
        filt = "d4" if i % 2 else "cdf97"
        elig = [k for k, r in enumerate(refs) if len(r) <= n // 2]
        k = elig[i % len(elig)]
        key = (k, filt, J)
        if key not in cache:
            cache[key] = S.plan_create(filt, J, refs[k])
        plans.append(cache[key])
        y = W.echoes(n, refs[k], rng)
        rx.append(torch.from_numpy(y.astype(np.complex64)).cuda())
        meta.append((filt, J, refs[k], y))
    return plans, rx, meta, cache


def check_against_oracle(got, meta, full_max_N=2200, nlags=24):
    rng = np.random.default_rng(5)
    for o, (filt, J, ref, y) in zip(got, meta):
        N = O.transform_length(len(y), J)
        g = o.cpu().numpy().astype(np.complex128)
        assert g.shape == (J, N)
        if N <= full_max_N:
            want = O.correlate_direct(filt, J, ref, y)
            for j in range(J):
                e = np.linalg.norm(g[j] - want[j]) / np.linalg.norm(want[j])
                assert e <= 1e-5, (len(y), j, e)
        else:
            for j in range(J):
                lags = np.concatenate([[0, N - 1], rng.integers(0, N, nlags)])
                want = O.correlate_at(filt, J, ref, y, j, lags)
                e = np.linalg.norm(g[j, lags] - want) / np.linalg.norm(want)
                assert e <= 1e-5, (len(y), j, e)


def test_uneven_batch_matches_oracle(dev):
    torch, S = dev
    plans, rx, meta, cache = make_batch(S, torch)
    print("[case] uneven batch", LENGTHS, flush=True)
    with S.Batch(plans, [x.numel() for x in rx]) as b:
        b.config(4096, 1024)
        info = b.info()
        assert info["whole_pulse_items"] > 0 and info["tile_items"] > 0
        out = S.batch_outputs(plans, [x.numel() for x in rx], rx[0].device)
        b.run(rx, out)
        torch.cuda.synchronize()
        check_against_oracle(out, meta)
    for p in cache.values():
        p.free()


@pytest.mark.parametrize("window", [1024, 4096])
def test_all_tile_split_matches_oracle(dev, window):
    """Every pulse as lag tiles: short pulses give levels of one to four
    tiles, whose groups are cut over several waves and summed through LDS."""
    torch, S = dev
    plans, rx, meta, cache = make_batch(S, torch, seed=45)
    ns = [x.numel() for x in rx]
    print(f"[case] all tiles, tile_window={window}", flush=True)
    with S.Batch(plans, ns) as b:
        b.config(0, window)
        info = b.info()
        assert info["whole_pulse_items"] == 0 and info["tile_items"] > 0
        out = S.batch_outputs(plans, ns, rx[0].device)
        b.run(rx, out)
        torch.cuda.synchronize()
        check_against_oracle(out, meta)
        first = [o.clone() for o in out]
        b.run(rx, out)
        torch.cuda.synchronize()
        for o, r in zip(out, first):
            assert torch.equal(o, r)
    for p in cache.values():
        p.free()


def test_work_splits_agree_and_graph_replays(dev):
    torch, S = dev
    plans, rx, meta, cache = make_batch(S, torch, seed=43)
    ns = [x.numel() for x in rx]
    results = []
    with S.Batch(plans, ns) as b:
        for fmax, rows in [(0, 512), (16384, 6144), (4096, 2048)]:
            print(f"[case] split fused_max_N={fmax} tile_window={rows}", flush=True)
            b.config(fmax, rows)
            out = S.batch_outputs(plans, ns, rx[0].device)
            b.run(rx, out)
            torch.cuda.synchronize()
            results.append([o.clone() for o in out])
            # replay of the captured graph gives the same bits
            b.run(rx, out)
            torch.cuda.synchronize()
            for o, r in zip(out, results[-1]):
                assert torch.equal(o, r)
    for r in results[1:]:
        for a, c in zip(results[0], r):
            d = (a - c).abs().max().item()
            assert d <= 1e-6 * max(1.0, a.abs().max().item()), d
    one_shot = S.correlate_batch(plans, rx)
    torch.cuda.synchronize()
    for a, c in zip(results[0], one_shot):
        assert (a - c).abs().max().item() <= 1e-6 * max(1.0, a.abs().max().item())
    for p in cache.values():
        p.free()


def test_bound_buffers_replay_the_same_planes(dev):
    """bind() + run_bound() (pointer arrays marshalled once) gives the same
    bits as run() on the same buffers, on repeated replays."""
    torch, S = dev
    plans, rx, meta, cache = make_batch(S, torch, seed=47)
    ns = [x.numel() for x in rx]
    with S.Batch(plans, ns) as b:
        with pytest.raises(RuntimeError):
            b.run_bound()
        out = S.batch_outputs(plans, ns, rx[0].device)
        b.run(rx, out)
        torch.cuda.synchronize()
        want = [o.clone() for o in out]
        out2 = S.batch_outputs(plans, ns, rx[0].device)
        b.bind(rx, out2)
        for _ in range(3):
            for o in out2:
                o.zero_()
            got = b.run_bound()
            torch.cuda.synchronize()
            assert got is not None and len(got) == len(want)
            for o, w in zip(out2, want):
                assert torch.equal(o, w)
    for p in cache.values():
        p.free()


def test_autotuner_picks_a_valid_split(dev):
    torch, S = dev
    plans, rx, meta, cache = make_batch(S, torch, seed=47)
    ns = [x.numel() for x in rx]
    with S.Batch(plans, ns) as b:
        out = S.batch_outputs(plans, ns, rx[0].device)
        info = b.tune(rx, out)
        print("[case] tuned", info, flush=True)
        assert info["tuned"] == 1 and info["tuned_us"] > 0
        assert info["tile_window"] in (1024, 2048, 3072, 4096, 6144)
        assert info["fused_max_N"] in (0, 2048, 4096, 8192, 16384)
        b.run(rx, out)
        torch.cuda.synchronize()
        check_against_oracle(out, meta, full_max_N=600, nlags=8)
    for p in cache.values():
        p.free()


def test_batch_refuses_an_integer_pulse_no_path_holds(dev):
    """A J = 8 integer plan (no int8 path) with a pulse beyond one
    workgroup's LDS: SIDWT_E_UNSUPPORTED at creation."""
    torch, S = dev
    ref = np.ones((40, 2), np.int16)
    with S.plan_create("legall53_int", 8, ref) as p:
        with pytest.raises(S.SidwtError) as e:
            S.Batch([p], [65536])
        assert e.value.code == -5


@pytest.mark.parametrize("n,J,count", [(65536, 12, 1), (40000, 11, 3)])
def test_plain_path_handles_pulses_beyond_one_workgroup(dev, n, J, count):
    """sidwt_correlate / sidwt_correlate_many on pulses too long for the
    whole-pulse LDS layout (tiled path), against the oracle at sampled lags,
    twice (the plan's cached tiled buffers are reused)."""
    torch, S = dev
    rng = np.random.default_rng(n + count)
    ref = W.reference_set(61, count=1, m_lo=900, m_hi=1000)[0]
    ys = [W.echoes(n, ref, rng) for _ in range(count)]
    print(f"[case] plain tiled n={n} J={J} count={count}", flush=True)
    with S.plan_create("cdf97", J, ref) as plan:
        rx = torch.from_numpy(np.stack(ys).astype(np.complex64)).cuda()
        for rep in range(2):
            if count == 1:
                out = S.correlate(plan, rx[0])[None]
            else:
                out = S.correlate_many(plan, rx)
            torch.cuda.synchronize()
            N = O.transform_length(n, J)
            for i in range(count):
                g = out[i].cpu().numpy()
                for j in (0, J // 2, J - 1):
                    lags = np.concatenate([[0, N - 1], rng.integers(0, N, 12)])
                    want = O.correlate_at("cdf97", J, ref, ys[i], j, lags)
                    e = np.linalg.norm(g[j, lags] - want) / np.linalg.norm(want)
                    assert e <= 1e-5, (rep, i, j, e)


def test_integer_batch_is_bit_exact(dev):
    """A batch of integer plans: pulses of several lengths and plans grouped
    by (plan, n), on the int8 whole-pulse kernel, the int8 block path (pulses
    beyond one workgroup's LDS) and the FP64 kernel (J = 8); every plane
    bit-exact against the oracle (whole planes for short pulses, sampled lags
    for long ones), on two runs with different output buffers."""
    torch, S = dev
    rng = np.random.default_rng(77)
    refs = [rng.integers(-2047, 2048, (m, 2)).astype(np.int16) for m in (60, 200, 300)]
    spec = [(0, 5, 700), (1, 6, 1500), (0, 5, 700), (2, 8, 2048), (1, 6, 20000),
            (1, 6, 20000), (0, 5, 3000), (2, 8, 2560)]
    plans, rx, cache = [], [], {}
    for k, J, n in spec:
        if (k, J) not in cache:
            cache[(k, J)] = S.plan_create("legall53_int", J, refs[k])
        plans.append(cache[(k, J)])
        rx.append(rng.integers(-32768, 32768, (n, 2)).astype(np.int16))
    print("[case] integer batch", [(J, n) for _, J, n in spec], flush=True)
    rx_d = [torch.from_numpy(x).cuda() for x in rx]
    ns = [n for _, _, n in spec]
    with S.Batch(plans, ns) as b:
        info = b.info()
        assert info["items"] == len(spec)
        assert info["tile_items"] == 2 and info["whole_pulse_items"] == len(spec) - 2
        outs = []
        for _ in range(2):
            out = S.batch_outputs(plans, ns, rx_d[0].device)
            b.run(rx_d, out)
            torch.cuda.synchronize()
            outs.append([o.cpu().numpy() for o in out])
    for i, (k, J, n) in enumerate(spec):
        N = O.transform_length(n, J)
        if n <= 3000:
            want = O.correlate_int(J, refs[k], rx[i])
            for got in outs:
                assert np.array_equal(got[i], want), (i, J, n)
        else:
            lags = np.unique(np.concatenate([[0, 1, N - 1], rng.integers(0, N, 12)]))
            for j in range(J):
                want = O.correlate_int_at(J, refs[k], rx[i], j, lags)
                for got in outs:
                    assert np.array_equal(got[i][j, lags], want), (i, j)


def test_integer_and_float_plans_do_not_mix(dev):
    torch, S = dev
    ri = np.ones((40, 2), np.int16)
    rf = np.ones(40, np.complex64)
    with S.plan_create("legall53_int", 4, ri) as pi, S.plan_create("cdf97", 4, rf) as pf:
        with pytest.raises(S.SidwtError):
            S.Batch([pi, pf], [512, 512])
