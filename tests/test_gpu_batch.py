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


def test_batch_rejects_integer_plans(dev):
    torch, S = dev
    ref = np.ones((16, 2), np.int16)
    with S.plan_create("legall53_int", 3, ref) as p:
        with pytest.raises(S.SidwtError) as e:
            S.Batch([p], [256])
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
