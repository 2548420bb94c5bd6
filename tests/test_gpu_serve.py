"""GPU tests of the serving loop: concurrent requests give the same result as
each request alone (bit for bit), the HBM ledger bounds what is admitted, and
sampled results meet the error bound."""
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
        assert torch.equal(alone, r.C), r.rid
    for r in reqs[::12]:
        A = pool.operand(r.fmt, r.m, r.k, r.a_off).cpu().numpy()
        B = pool.operand(r.fmt, r.k, r.n, r.b_off).cpu().numpy()
        diff, absab, _ = orc.exact_check(A, B, r.C.cpu().numpy())
        ok, worst = orc.bound_report(diff, absab, T_BITS[r.fmt])
        assert ok, (r.rid, r.fmt, worst)


def test_budget_limits_admission(srv):
    serve, pool = srv
    reqs = serve.make_requests(30, rate=1e6, seed=9, lo=64, hi=256, pool=pool.elements)
    server = serve.Server(pool, budget_gb=64, streams=8)
    biggest = max(server.cost(r) for r in reqs)
    budget = 2.2 * biggest / serve.GB  # room for two of the largest at a time
    server = serve.Server(pool, budget_gb=budget, streams=8)
    st = server.run(reqs)
    assert st.peak_ledger_gb <= budget + 1e-9
    assert all(r.done >= r.start >= r.arrival for r in reqs)
    tiny = serve.Server(pool, budget_gb=biggest / serve.GB / 2, streams=2)
    with pytest.raises(ValueError):
        tiny.run(reqs)
