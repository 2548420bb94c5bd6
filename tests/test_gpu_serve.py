"""GPU tests of the serving loop: concurrent requests give the same result as
each request alone (bit for bit), the HBM ledger bounds what is admitted and
the device memory the server really holds, and sampled results meet the error
bound."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

T_BITS = {"dd": 100, "td": 150, "qd": 200}


@pytest.fixture(scope="module")
def srv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_09960_amd as mp
    mp.lib()
    from paper_2301_09960_amd import serve
    return serve, serve.DevicePool(elements=1 << 20, seed=3)


def test_mix_equals_alone(srv, orc):
    import torch

    import paper_2301_09960_amd as mp
    serve, pool = srv
    reqs = serve.make_requests(60, rate=5000.0, seed=8, lo=16, hi=256, pool=pool.elements)
    st = serve.Server(pool, budget_gb=64, streams=6).run(reqs, keep_results=True)
    print(f"mix: p50 {st.p50_ms:.2f} ms p99 {st.p99_ms:.2f} ms inflight<= {st.max_inflight}", flush=True)
    assert st.max_inflight > 1  # requests did overlap
    for r in reqs:
        A = pool.operand(r.fmt, r.m, r.k, r.a_off)
        B = pool.operand(r.fmt, r.k, r.n, r.b_off)
        alone = mp.gemm(r.fmt, A, B)
        torch.cuda.synchronize()
        assert torch.equal(alone, r.kept), r.rid
    for r in reqs[::12]:
        A = pool.operand(r.fmt, r.m, r.k, r.a_off).cpu().numpy()
        B = pool.operand(r.fmt, r.k, r.n, r.b_off).cpu().numpy()
        diff, absab, _ = orc.exact_check(A, B, r.kept.cpu().numpy())
        ok, worst = orc.bound_report(diff, absab, T_BITS[r.fmt])
        assert ok, (r.rid, r.fmt, worst)


def reservation(serve, mp, reqs, streams, mode="float"):
    need = max(mp.workspace_bytes(r.fmt, mode, r.m, r.n, r.k) for r in reqs)
    return streams * serve.Server.units(need)  # an upper bound of the slot workspaces' charge


def test_budget_limits_admission(srv):
    import paper_2301_09960_amd as mp
    serve, pool = srv
    reqs = serve.make_requests(30, rate=1e6, seed=9, lo=64, hi=256, pool=pool.elements)
    server = serve.Server(pool, budget_gb=64, streams=8)
    biggest = max(server.cost(r) for r in reqs)
    # the slot workspaces and room for two of the largest requests at a time
    budget = (reservation(serve, mp, reqs, 8) + 2.2 * biggest) / serve.GB
    server = serve.Server(pool, budget_gb=budget, streams=8)
    st = server.run(reqs)
    assert st.peak_ledger_gb <= budget + 1e-9
    assert all(r.done >= r.start >= r.arrival for r in reqs)
    tiny = serve.Server(pool, budget_gb=biggest / serve.GB / 2, streams=2)
    with pytest.raises(ValueError):
        tiny.run(reqs)


@pytest.mark.parametrize("mode", ["float", "int8"])
def test_ledger_bounds_device_memory(srv, mode):
    """At every admission and completion, the device memory allocated beyond
    the pool is at most the ledger, and the ledger at most the budget."""
    import torch

    import paper_2301_09960_amd as mp
    serve, pool = srv
    reqs = serve.make_requests(80, rate=20000.0, seed=10, lo=32, hi=512, pool=pool.elements)
    probe = serve.Server(pool, budget_gb=64, streams=6, mode=mode)
    biggest = max(probe.cost(r) for r in reqs)
    budget = (reservation(serve, mp, reqs, 6, mode) + 3.5 * biggest) / serve.GB
    server = serve.Server(pool, budget_gb=budget, streams=6, mode=mode)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    over = []

    def check(s):
        over.append(torch.cuda.memory_allocated() - base - s.ledger)
        assert s.ledger <= s.budget

    server.on_change = check
    st = server.run(reqs)
    print(f"ledger {mode}: {len(over)} checks, worst excess {max(over)} bytes, peak {st.peak_ledger_gb:.3f} GB, "
          f"budget {budget:.3f} GB, inflight<= {st.max_inflight}", flush=True)
    assert len(over) == 2 * len(reqs)
    assert max(over) <= 0
    assert st.max_inflight > 1
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
