"""Serving with continuous batching: each result is the same alone and in
the mix; admission keeps the in-flight footprint within the HBM budget and
never drops a request."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

LENGTHS = [300, 517, 800, 1500, 2100, 3000, 5000, 7000, 9000, 12000, 17000, 24000]


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_cs_0607001_amd as S
    from paper_cs_0607001_amd import serving
    S._lib.lib()
    refs = W.reference_set(31, count=8, m_lo=24, m_hi=400)
    bank = S.Bank("cdf97", 12, refs, "fp16")
    yield torch, S, serving, bank, refs
    bank.free()


def requests(serving, torch, rate_hz, seed=5, keep=True):
    rng = np.random.default_rng(seed)            # pulses: same for every arrival pattern
    arrivals = np.random.default_rng(seed + 1000)
    refs = W.reference_set(31, count=8, m_lo=24, m_hi=400)
    t = np.zeros(len(LENGTHS)) if rate_hz <= 0 else np.cumsum(
        arrivals.exponential(1.0 / rate_hz, len(LENGTHS)))
    out = []
    for i, n in enumerate(LENGTHS):
        y = W.echoes(n, refs[i % 3], rng)
        x = torch.from_numpy(y.astype(np.complex64)).pin_memory()
        out.append(serving.Request(i, float(t[i]), x, W.levels_for(n), keep=keep))
    return out


def test_each_result_is_the_same_alone_and_in_the_mix(env):
    torch, S, serving, bank, refs = env
    reqs = requests(serving, torch, rate_hz=0)
    alone = {}
    for r in reqs:
        o = bank.correlate([r.rx.cuda()], [r.J])[0]
        torch.cuda.synchronize()
        alone[r.rid] = o.cpu()
    srv = serving.Server(bank, slots=4, budget_bytes=4 << 30, max_group=3)
    recs = srv.run(requests(serving, torch, rate_hz=4000.0))
    torch.cuda.synchronize()
    assert len(recs) == len(reqs)
    assert len({r.group for r in recs}) > 1           # several groups overlapped
    for rid, want in alone.items():
        got = srv.outputs[rid].cpu()
        assert got.shape == want.shape
        # same decomposition for a request alone and in the mix: same bits
        assert torch.equal(got, want), rid
        rel = (got - want).abs().max() / want.abs().max().clamp_min(1e-30)
        assert rel.item() <= 1e-5
    srv.close()


def test_admission_respects_the_budget_and_drops_nothing(env):
    torch, S, serving, bank, refs = env
    reqs = requests(serving, torch, rate_hz=0, keep=False)
    srv = serving.Server(bank, slots=4, budget_bytes=1 << 30)
    biggest = max(srv.footprint(r.rx.numel(), r.J) for r in reqs)
    budget = int(biggest * 1.5)
    srv = serving.Server(bank, slots=4, budget_bytes=budget)
    recs = srv.run(reqs)
    assert sorted(r.rid for r in recs) == list(range(len(reqs)))
    assert srv.max_inflight_bytes <= budget
    for r in recs:
        assert r.completed >= r.admitted >= r.arrival - 1e-6
    srv.close()
    # a budget below one request's footprint still serves it, alone
    small = biggest // 4
    srv = serving.Server(bank, slots=2, budget_bytes=small)
    reqs2 = requests(serving, torch, rate_hz=0, keep=False)
    fp = {r.rid: srv.footprint(r.rx.numel(), r.J) for r in reqs2}
    recs = srv.run(reqs2)
    assert len(recs) == len(reqs2)
    groups = {}
    for r in recs:
        groups.setdefault(r.group, []).append(r.rid)
    for members in groups.values():
        # an oversize request runs alone; any other group fits the budget
        assert len(members) == 1 or sum(fp[m] for m in members) <= small
    assert any(fp[m] > small for ms in groups.values() for m in ms)
    srv.close()


def test_summary_reports_latency_percentiles(env):
    torch, S, serving, bank, refs = env
    srv = serving.Server(bank, slots=2)
    recs = srv.run(requests(serving, torch, rate_hz=2000.0, keep=False))
    s = serving.summarize(recs)
    assert s["requests"] == len(LENGTHS)
    assert 0 < s["p50_ms"] <= s["p99_ms"]
    assert s["samples_per_s"] > 0
    srv.close()


def test_steady_serving_reuses_the_slot_arenas(env):
    """After a first pass the slots' device arenas hold every group, so a
    second pass over the same requests allocates nothing and gives the same
    planes."""
    torch, S, serving, bank, refs = env
    srv = serving.Server(bank, slots=1, budget_bytes=4 << 30, max_group=1)
    srv.run(requests(serving, torch, rate_hz=0))
    first = {rid: o.cpu() for rid, o in srv.outputs.items()}
    grows = srv.arena_grows
    assert grows >= 2
    srv.outputs = {}
    srv.run(requests(serving, torch, rate_hz=0))
    assert srv.arena_grows == grows
    for rid, want in first.items():
        assert torch.equal(srv.outputs[rid].cpu(), want)
    srv.close()
