"""The benchmark's batched workloads, exactly as it builds them: 512 DD and 512
QD products with m, n, k each log-uniform in [64, 1024] (seeded), operands
sliced out of the device pool of e ~ U{0..8} values, in both slice forms, and
a mixed batch of 256 DD and 256 QD products (two batched launches on one
stream).  Every product equals its single call bit for bit; a sample meets
the error bound against the oracle's exact product on sampled rows."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

T_BITS = {"dd": 100, "td": 150, "qd": 200}
SEED = 31  # the benchmark's batch seed


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_09960_amd as mp
    from paper_2301_09960_amd import serve
    mp.lib()
    assert mp.check_device() == 0
    pool = serve.DevicePool(elements=1 << 24, seed=99)  # the benchmark's pool
    yield mp, serve, pool
    mp.batched_cache_clear()


def say(*a):
    print(*a, flush=True)


def check_batch(mp, orc, fmt, mode, As, Bs, Cs, sample):
    import torch
    for i, (A, B) in enumerate(zip(As, Bs)):
        single = mp.gemm(fmt, A, B, mode=mode)
        assert torch.equal(single, Cs[i]), (fmt, mode, i, tuple(A.shape), tuple(B.shape))
    torch.cuda.synchronize()
    for i in sample:
        A, B, C = As[i].cpu().numpy(), Bs[i].cpu().numpy(), Cs[i].cpu().numpy()
        m = A.shape[2]
        rows = sorted({0, m // 2, m - 1})
        diff, absab, _ = orc.exact_check(A, B, C, rows=rows)
        ok, worst = orc.bound_report(diff, absab, T_BITS[fmt])
        assert ok, (fmt, mode, i, worst)


@pytest.mark.parametrize("fmt", ["dd", "qd"])
@pytest.mark.parametrize("mode", ["float", "int8"])
def test_bench_batch_512(env, orc, fmt, mode):
    import torch
    mp, serve, pool = env
    As, Bs, m, n, k = serve.batch_operands(pool, fmt, 512, SEED)
    say(f"bench batch {fmt} {mode}: 512 products, sum 2mnk = {float(np.sum(2.0 * m * n * k)):.3e}")
    Cs = mp.gemm_batched(fmt, As, Bs, mode=mode)  # captures the graph
    Cs2 = mp.gemm_batched(fmt, As, Bs, mode=mode)  # a replay
    torch.cuda.synchronize()
    for a, b in zip(Cs, Cs2):
        assert torch.equal(a, b)
    big = int(np.argmax(m * n * k))
    check_batch(mp, orc, fmt, mode, As, Bs, Cs, [0, 100, 255, 511, big])
    mp.batched_cache_clear()


@pytest.mark.parametrize("mode", ["float", "int8"])
def test_bench_batch_mixed(env, orc, mode):
    """256 DD and 256 QD products (the first and second halves of the seeded
    shape sequence) as two batched launches on one stream."""
    import torch
    mp, serve, pool = env
    Ad, Bd, *_ = serve.batch_operands(pool, "dd", 256, SEED)
    Aq, Bq, *_ = serve.batch_operands(pool, "qd", 256, SEED, first=256)
    say(f"bench batch mixed {mode}: 256 DD + 256 QD")
    Cd = mp.gemm_batched("dd", Ad, Bd, mode=mode)
    Cq = mp.gemm_batched("qd", Aq, Bq, mode=mode)
    torch.cuda.synchronize()
    check_batch(mp, orc, "dd", mode, Ad, Bd, Cd, [3, 200])
    check_batch(mp, orc, "qd", mode, Aq, Bq, Cq, [7, 255])
    mp.batched_cache_clear()
