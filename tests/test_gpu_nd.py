"""GPU parity of the longer binary64 expansions (c = 2 .. 14 components,
INT8-slice form, mpgemm_nd) against the CPU oracle: digit slices and
exponents bit-exact, diagonal sums bit-exact, and C within 2^-(50 c) (|A||B|)
of the exact product."""
import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu


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


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


def fmt_of(c):
    return {2: "dd", 3: "td", 4: "qd"}.get(c, f"{c}d")


def test_two_components_equal_dd_int8(mp):
    """c = 2 runs the DD INT8 path: identical bits to mpgemm_dd in the INT8 form."""
    A, B = W.gen_pair("dd", 150, 97, 333, E=16, seed=1)
    dA, dB = dev(A), dev(B)
    C1 = host(mp.gemm_nd(dA, dB))
    C2 = host(mp.gemm("dd", dA, dB, mode="int8"))
    assert np.array_equal(C1, C2)


@pytest.mark.parametrize("c", [5, 8, 14])
def test_nd_digits_bit_exact(mp, orc, c):
    m, k, n = 70, 90, 40
    A, B = W.gen_pair(fmt_of(c), m, n, k, E=16, seed=10 + c)
    D = mp.nd_num_slices(c, k)
    say(f"nd digits c={c} D={D}")
    da, ea = orc.split_int8(A, D, "rows")
    db, eb = orc.split_int8(B, D, "cols")
    ga, gea = mp.nd_debug_split(dev(A), 0, D)
    gb, geb = mp.nd_debug_split(dev(B), 1, D)
    assert np.array_equal(host(ga), da)
    assert np.array_equal(host(gea), ea)
    assert np.array_equal(host(gb), db)
    assert np.array_equal(host(geb), eb)


@pytest.mark.parametrize("c,D", [(5, 41), (8, 59), (14, 112)])
def test_nd_digits_on_rounding_boundaries(mp, orc, c, D):
    """Exact and near ties at every digit the expansion carries (as in the
    INT8 tests of the DD/TD/QD formats), with the digit counts that take the
    9-, 13- and 25-word integers of the long-expansion kernel."""
    from digit_cases import tie_cases
    rows = [tie_cases(c, D, E, seed=c + E + 200) for E in (5, -33)]
    k = max(len(r) for r in rows)
    A = np.zeros((c, k, len(rows) + 1))
    for i, cases in enumerate(rows):
        for p, comps in enumerate(cases):
            A[:, p, i] = comps
    B = np.ascontiguousarray(np.transpose(A, (0, 2, 1)))
    say(f"nd digits on boundaries c={c} D={D} k={k}")
    da, ea = orc.split_int8(A, D, "rows")
    db, eb = orc.split_int8(B, D, "cols")
    ga, gea = mp.nd_debug_split(dev(A), 0, D)
    gb, geb = mp.nd_debug_split(dev(B), 1, D)
    assert np.array_equal(host(gea), ea) and np.array_equal(host(geb), eb)
    assert np.array_equal(host(ga), da)
    assert np.array_equal(host(gb), db)


def test_nd_diagonal_sums_bit_exact(mp, orc):
    c, m, n, k = 9, 45, 38, 150
    A, B = W.gen_pair(fmt_of(c), m, n, k, E=8, seed=3)
    D = mp.nd_num_slices(c, k)
    da, _ = orc.split_int8(A, D, "rows")
    db, _ = orc.split_int8(B, D, "cols")
    S = orc.int8_diag_sums(da, db)
    dA, dB = dev(A), dev(B)
    for g in (1, D // 3, D - 1, D):
        say(f"nd diagonal c={c} g={g} D={D}")
        assert np.array_equal(host(mp.nd_debug_products(dA, dB, g, D)), S[g - 1]), g


@pytest.mark.parametrize("c,m,n,k", [(5, 130, 70, 200), (6, 33, 129, 65), (7, 1, 1, 1), (8, 100, 90, 300),
                                     (10, 64, 64, 64), (12, 40, 50, 77), (14, 70, 30, 120)])
def test_nd_meets_bound(mp, orc, c, m, n, k):
    A, B = W.gen_pair(fmt_of(c), m, n, k, E=16, seed=m + n + k + c)
    say(f"nd gemm c={c} m={m} n={n} k={k}")
    C = host(mp.gemm_nd(dev(A), dev(B)))
    diff, absab, _ = orc.exact_check(A, B, C)
    ok, worst = orc.bound_report(diff, absab, 50 * c)
    say(f"  D={mp.nd_num_slices(c, k)} worst log2 ratio {worst:.1f} (bound -{50 * c})")
    assert ok
    # the oracle's INT8-form product with the same D sums the same exact terms
    # (rounded once; the GPU adds them with TwoSum): leading components agree
    Co = orc.int8_gemm(A, B, mp.nd_num_slices(c, k))
    rel = np.abs(C[0] - Co[0]) / np.maximum(np.abs(Co[0]), 1e-300)
    assert np.all(rel <= 2.0 ** -52)


def test_nd_larger_sampled(mp, orc):
    """c = 8 (424 bits) at n = 1024 (one k chunk, 128 x 128 tiles): sampled rows."""
    c, nn = 8, 1024
    A, B = W.gen_pair(fmt_of(c), nn, nn, nn, E=16, seed=1024)
    C = host(mp.gemm_nd(dev(A), dev(B)))
    diff, absab, _ = orc.exact_check(A, B, np.ascontiguousarray(C), rows=[0, 777])
    ok, worst = orc.bound_report(diff, absab, 50 * c)
    say(f"  worst log2 ratio {worst:.1f} (bound -{50 * c})")
    assert ok
