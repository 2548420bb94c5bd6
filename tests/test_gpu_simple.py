"""GPU tests of the simple in-format matrix multiplication (the non-Ozaki
comparison of Section 4.4) and of the D+S format.

* DD, TD, QD, TS simple products (staged through LDS and direct): C within
  k 2^-(L - 3) (|A||B|) of the exact product (L = 106, 159, 212, 72), the
  bound the oracle's own triple loop is pinned to; the staged and direct
  kernels give the same C bit for bit.
* D+S simple product: within (k 2^-103 + 2^-76) (|A||B|); staged = direct.
* D+S Ozaki product: within 2^-76 (|A||B|), and equal to the oracle's D+S
  rounding (hi = RN53, lo = RN24 of the rest) of the DD product of the inputs
  read as DD, computed by mpgemm_dd.
"""
import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu

L_BITS = {"dd": 106, "td": 159, "qd": 212, "ts": 72}


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_09960_amd as mp
    mp.lib()
    assert mp.check_device() == 0
    return mp


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def say(*a):
    print(*a, flush=True)


def within(orc, A, B, C, slack_of_k, rows=None):
    diff, absab, _ = orc.exact_check(A, B, C, rows=rows)
    bound = slack_of_k * absab
    ok = bool(np.all(diff <= bound))
    ratio = np.max(diff[absab > 0] / absab[absab > 0]) if np.any(absab > 0) else 0.0
    return ok, float(np.log2(ratio)) if ratio > 0 else float("-inf")


@pytest.mark.parametrize("fmt", ["dd", "td", "qd", "ts"])
@pytest.mark.parametrize("m,n,k", [(150, 97, 333), (1, 77, 5), (65, 1, 130), (64, 64, 16)])
def test_simple_within_bound_and_staging_agrees(mp, orc, fmt, m, n, k):
    import torch
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=m + 3 * n + 7 * k)
    dA, dB = dev(A), dev(B)
    say(f"simple {fmt} m={m} n={n} k={k}")
    C1 = mp.simple(fmt, dA, dB, staging=1)
    C0 = mp.simple(fmt, dA, dB, staging=0)
    torch.cuda.synchronize()
    assert torch.equal(C0, C1), "staged and direct differ"
    ok, worst = within(orc, A, B, C1.cpu().numpy(), k * 2.0 ** -(L_BITS[fmt] - 3))
    say(f"  worst log2 ratio {worst:.1f} (bound log2(k) - {L_BITS[fmt] - 3})")
    assert ok


@pytest.mark.parametrize("fmt,rows", [("dd", [0, 700, 1023]), ("ts", [5, 1000])])
def test_simple_n1024_sampled(mp, orc, fmt, rows):
    import torch
    n = 1024
    A, B = W.gen_pair(fmt, n, n, n, E=16, seed=1024)
    C = mp.simple(fmt, dev(A), dev(B), staging=1)
    torch.cuda.synchronize()
    ok, worst = within(orc, A, B, C.cpu().numpy(), n * 2.0 ** -(L_BITS[fmt] - 3), rows=rows)
    say(f"simple {fmt} n={n}: worst log2 ratio {worst:.1f}")
    assert ok


def test_simple_edge_cases(mp):
    import torch
    C = torch.full((2, 5, 4), 7.0, dtype=torch.float64, device="cuda")
    mp.simple("dd", torch.zeros((2, 0, 4), dtype=torch.float64, device="cuda"),
              torch.zeros((2, 5, 0), dtype=torch.float64, device="cuda"), C)
    torch.cuda.synchronize()
    assert torch.all(C == 0)
    # exact small integers: the triple loop is exact
    A = torch.zeros((3, 9, 6), dtype=torch.float32, device="cuda")
    B = torch.zeros((3, 4, 9), dtype=torch.float32, device="cuda")
    A[0] = torch.arange(54, dtype=torch.float32, device="cuda").reshape(9, 6) - 20
    B[0] = torch.arange(36, dtype=torch.float32, device="cuda").reshape(4, 9) % 7 - 3
    C = mp.simple("ts", A, B)
    want = (A[0].double().t() @ B[0].double().t()).t()
    torch.cuda.synchronize()
    assert torch.equal(C[0].double(), want) and torch.all(C[1:] == 0)


def ds_dev(X):
    return dev(X)


@pytest.mark.parametrize("m,n,k", [(150, 97, 333), (1, 1, 1), (33, 70, 4)])
def test_ds_simple(mp, orc, m, n, k):
    import torch
    Ahi, Alo = W.gen_ds(m, k, E=16, seed=m + k, operand="A")
    Bhi, Blo = W.gen_ds(k, n, E=16, seed=m + k, operand="B")
    d = [dev(x) for x in (Ahi, Alo, Bhi, Blo)]
    say(f"ds simple m={m} n={n} k={k}")
    h1, l1 = mp.ds_simple(*d, staging=1)
    h0, l0 = mp.ds_simple(*d, staging=0)
    torch.cuda.synchronize()
    assert torch.equal(h0, h1) and torch.equal(l0, l1)
    C = orc.ds_as_dd(h1.cpu().numpy(), l1.cpu().numpy())
    ok, worst = within(orc, orc.ds_as_dd(Ahi, Alo), orc.ds_as_dd(Bhi, Blo), C, k * 2.0 ** -103 + 2.0 ** -76)
    say(f"  worst log2 ratio {worst:.1f}")
    assert ok
    assert np.all(np.abs(C[1]) <= np.abs(C[0]) * 2.0 ** -53)


@pytest.mark.parametrize("mode", ["float", "int8"])
def test_ds_ozaki_equals_rounded_dd_product(mp, orc, mode):
    import torch
    m, n, k = 130, 90, 257
    Ahi, Alo = W.gen_ds(m, k, E=16, seed=5, operand="A")
    Bhi, Blo = W.gen_ds(k, n, E=16, seed=5, operand="B")
    A, B = orc.ds_as_dd(Ahi, Alo), orc.ds_as_dd(Bhi, Blo)
    say(f"ds ozaki {mode} m={m} n={n} k={k}")
    hi, lo = mp.ds_gemm(*[dev(x) for x in (Ahi, Alo, Bhi, Blo)], mode=mode)
    Cdd = mp.gemm("dd", dev(A), dev(B), mode=mode)
    torch.cuda.synchronize()
    want_hi, want_lo = orc.ds_round(Cdd.cpu().numpy())
    assert np.array_equal(hi.cpu().numpy()[0], want_hi) and np.array_equal(lo.cpu().numpy()[0], want_lo)
    ok, worst = within(orc, A, B, orc.ds_as_dd(hi.cpu().numpy(), lo.cpu().numpy()), 2.0 ** -76)
    say(f"  worst log2 ratio {worst:.1f} (bound -76)")
    assert ok
