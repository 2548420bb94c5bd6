"""GPU tests of the batched path (one graph-captured launch sequence for many
uneven products): every product equals the single call bit for bit, meets the
error bound, and graph replays with new inputs (with eager work in between)
give the eager results."""
import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu

T_BITS = {"dd": 100, "td": 150, "qd": 200, "ts": 66}


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_09960_amd as mp
    mp.lib()
    assert mp.check_device() == 0
    yield mp
    mp.batched_cache_clear()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def say(*a):
    print(*a, flush=True)


def shapes(seed, count, lo, hi):
    m = W.log_uniform_sizes(seed, count, lo, hi, draw=0)
    n = W.log_uniform_sizes(seed, count, lo, hi, draw=1)
    k = W.log_uniform_sizes(seed, count, lo, hi, draw=2)
    return list(zip(m.tolist(), n.tolist(), k.tolist()))


def make_batch(fmt, sh, seed, E=8):
    return [W.gen_pair(fmt, m, n, k, E=E, seed=seed * 1000 + i) for i, (m, n, k) in enumerate(sh)]


@pytest.mark.parametrize("fmt", ["dd", "qd", "ts"])
def test_batched_equals_single_calls(mp, orc, fmt):
    import torch
    sh = shapes(1, 30, 1, 300) + [(0, 5, 7), (6, 0, 3), (5, 4, 0), (1, 1, 1), (64, 64, 64), (65, 1, 129)]
    say(f"batched {fmt}: {len(sh)} products")
    host = make_batch(fmt, sh, seed=7)
    As = [dev(A) for A, _ in host]
    Bs = [dev(B) for _, B in host]
    Cs = mp.gemm_batched(fmt, As, Bs)
    torch.cuda.synchronize()
    for i, (A, B) in enumerate(zip(As, Bs)):
        single = mp.gemm(fmt, A, B)
        torch.cuda.synchronize()
        assert torch.equal(single, Cs[i]), i
    for i in range(0, len(sh), 5):
        m, n, k = sh[i]
        if m == 0 or n == 0:
            continue
        A, B = host[i]
        diff, absab, _ = orc.exact_check(A, B, Cs[i].cpu().numpy())
        ok, worst = orc.bound_report(diff, absab, T_BITS[fmt])
        assert ok, (i, sh[i], worst)


@pytest.mark.parametrize("fmt", ["dd", "qd", "ts"])
def test_batched_split_kernels_agree(mp, fmt):
    """A batch whose operands are split partly by the fused kernel and partly
    by the per-pass kernels (k beyond the fused limit) gives the same C as the
    per-pass split alone and as single calls."""
    import torch
    sh = shapes(3, 12, 1, 700) + [(9, 7, 4097), (3, 5, 8200), (40, 33, 4096), (17, 2, 1)]
    say(f"batched split kernels {fmt}: {len(sh)} products")
    host = make_batch(fmt, sh, seed=11)
    As = [dev(A) for A, _ in host]
    Bs = [dev(B) for _, B in host]
    try:
        out = []
        for kind in (0, 1):
            mp.set_split_kernel(kind)
            out.append(mp.gemm_batched(fmt, As, Bs))
            torch.cuda.synchronize()
        for i, (A, B) in enumerate(zip(As, Bs)):
            assert torch.equal(out[0][i], out[1][i]), (i, sh[i])
            single = mp.gemm(fmt, A, B)
            torch.cuda.synchronize()
            assert torch.equal(single, out[1][i]), (i, sh[i])
    finally:
        mp.set_split_kernel(0)


def test_batched_literal_last_slice(mp):
    """Algorithm 1's printed last slice in a batch: the same C as single calls
    with that option, and a different one from the default extraction."""
    import torch
    fmt = "qd"
    sh = shapes(5, 10, 1, 300) + [(9, 7, 4097)]
    host = make_batch(fmt, sh, seed=13)
    As = [dev(A) for A, _ in host]
    Bs = [dev(B) for _, B in host]
    try:
        mp.set_last_slice("remainder")
        Cs = mp.gemm_batched(fmt, As, Bs)
        singles = [mp.gemm(fmt, A, B) for A, B in zip(As, Bs)]
    finally:
        mp.set_last_slice("extract")
    Cd = mp.gemm_batched(fmt, As, Bs)
    torch.cuda.synchronize()
    differs = 0
    for i in range(len(sh)):
        assert torch.equal(singles[i], Cs[i]), (i, sh[i])
        differs += int(not torch.equal(Cd[i], Cs[i]))
    assert differs > 0


@pytest.mark.parametrize("fmt", ["dd", "td", "qd"])
def test_batched_int8_equals_single_calls(mp, orc, fmt):
    """The INT8 form batched: every product equals its single INT8 call bit for
    bit (exact digit sums, same combination order), and meets the bound."""
    import torch
    sh = shapes(4, 26, 1, 400) + [(0, 5, 7), (5, 4, 0), (1, 1, 1), (300, 257, 129)]
    say(f"batched int8 {fmt}: {len(sh)} products")
    host = make_batch(fmt, sh, seed=17, E=16)
    As = [dev(A) for A, _ in host]
    Bs = [dev(B) for _, B in host]
    Cs = mp.gemm_batched(fmt, As, Bs, mode="int8")
    torch.cuda.synchronize()
    for i, (A, B) in enumerate(zip(As, Bs)):
        single = mp.gemm(fmt, A, B, mode="int8")
        torch.cuda.synchronize()
        assert torch.equal(single, Cs[i]), (i, sh[i])
    for i in range(0, len(sh), 6):
        m, n, k = sh[i]
        if m == 0 or n == 0:
            continue
        A, B = host[i]
        diff, absab, _ = orc.exact_check(A, B, Cs[i].cpu().numpy())
        ok, worst = orc.bound_report(diff, absab, T_BITS[fmt])
        assert ok, (i, sh[i], worst)


@pytest.mark.parametrize("mode", ["float", "int8"])
@pytest.mark.parametrize("sh", [[(1, 1, 1)], [(70, 9, 33), (5, 130, 64)], [(64, 64, 64), (3, 3, 300), (129, 65, 2)]])
def test_batches_with_fewer_items_than_work_lists(mp, mode, sh):
    """Batches of one to three small products give fewer work items than
    there are per-XCD lists (and a persistent grid that small): every product
    still equals its single call bit for bit."""
    import torch
    host = make_batch("dd", sh, seed=29)
    As = [dev(A) for A, _ in host]
    Bs = [dev(B) for _, B in host]
    Cs = mp.gemm_batched("dd", As, Bs, mode=mode)
    torch.cuda.synchronize()
    for i, (A, B) in enumerate(zip(As, Bs)):
        assert torch.equal(mp.gemm("dd", A, B, mode=mode), Cs[i]), (i, sh[i])


def test_graph_replays_with_new_inputs(mp):
    import torch
    sh = shapes(2, 24, 16, 200)
    batches = [make_batch("td", sh, seed=s) for s in (11, 12, 13)]
    outs = []
    for r, host in enumerate(batches + batches[:1]):
        As = [dev(A) for A, _ in host]
        Bs = [dev(B) for _, B in host]
        Cs = mp.gemm_batched("td", As, Bs)  # first call captures, the rest replay
        torch.cuda.synchronize()
        # eager work between replays
        eager = [mp.gemm("td", A, B) for A, B in zip(As, Bs)]
        torch.cuda.synchronize()
        for i in range(len(sh)):
            assert torch.equal(eager[i], Cs[i]), (r, i)
        outs.append([c.cpu() for c in Cs])
        say(f"replay {r} ok")
    for a, b in zip(outs[0], outs[3]):  # same inputs, same results
        assert torch.equal(a, b)


def test_config3_like_batch(mp, orc):
    """128 DD products, m, n, k log-uniform in [64, 512], e ~ U{0..8}: a sample
    equals single calls bit for bit and meets the bound."""
    import torch
    sh = shapes(3, 128, 64, 512)
    host = make_batch("dd", sh, seed=21)
    As = [dev(A) for A, _ in host]
    Bs = [dev(B) for _, B in host]
    Cs = mp.gemm_batched("dd", As, Bs)
    torch.cuda.synchronize()
    for i in range(0, 128, 9):
        assert torch.equal(mp.gemm("dd", As[i], Bs[i]), Cs[i]), i
    for i in (0, 77):
        A, B = host[i]
        diff, absab, _ = orc.exact_check(A, B, Cs[i].cpu().numpy(), rows=[0, sh[i][0] - 1])
        ok, worst = orc.bound_report(diff, absab, 100)
        assert ok, worst
