"""GPU parity of the INT8-slice form against the CPU oracle: digit slices and
exponents bit-exact, diagonal sums S_g bit-exact (int64), C within
2^-t (|A||B|) of the exact product (t = 100 / 150 / 200)."""
import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu

T_BITS = {"dd": 100, "td": 150, "qd": 200}


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


@pytest.mark.parametrize("fmt", ["dd", "td", "qd"])
@pytest.mark.parametrize("E", [0, 16])
def test_int8_split_bit_exact(mp, orc, fmt, E):
    m, k, n = 140, 100, 70
    A, B = W.gen_pair(fmt, m, n, k, E=E, seed=300 + E)
    D = mp.num_slices(fmt, "int8", k)
    say(f"int8 split {fmt} E={E} D={D}")
    da, ea = orc.split_int8(A, D, "rows")
    db, eb = orc.split_int8(B, D, "cols")
    ga, gea = mp.debug_split(fmt, dev(A), 0, D, mode="int8")
    gb, geb = mp.debug_split(fmt, dev(B), 1, D, mode="int8")
    assert np.array_equal(host(ga), da)
    assert np.array_equal(host(gea), ea)
    assert np.array_equal(host(gb), db)
    assert np.array_equal(host(geb), eb)


@pytest.mark.parametrize("fmt,c,D", [("dd", 2, 17), ("dd", 2, 21), ("td", 3, 24), ("td", 3, 35), ("qd", 4, 31),
                                     ("qd", 4, 40)])
def test_int8_digits_on_rounding_boundaries(mp, orc, fmt, c, D):
    """Exact ties and ties moved by 2^-70 of a unit either way, at every digit
    the expansion can carry, as rows of A and as columns of B (several rows
    with different exponents, one of them all zero): the digits equal the
    oracle's bit for bit (the rounding follows the whole expansion, not its
    leading component).  The D values use each integer width of the kernel
    (4 to 9 words)."""
    from digit_cases import tie_cases
    rows = [tie_cases(c, D, E, seed=c + E + 100) for E in (3, -40, 77)]
    k = max(len(r) for r in rows)
    A = np.zeros((c, k, len(rows) + 1))  # the last row stays zero
    for i, cases in enumerate(rows):
        for p, comps in enumerate(cases):
            A[:, p, i] = comps
    B = np.ascontiguousarray(np.transpose(A, (0, 2, 1)))  # the same values as columns of B
    say(f"int8 digits on boundaries {fmt} D={D} k={k}")
    da, ea = orc.split_int8(A, D, "rows")
    db, eb = orc.split_int8(B, D, "cols")
    ga, gea = mp.debug_split(fmt, dev(A), 0, D, mode="int8")
    gb, geb = mp.debug_split(fmt, dev(B), 1, D, mode="int8")
    assert np.array_equal(host(gea), ea) and np.array_equal(host(geb), eb)
    assert np.array_equal(host(ga), da)
    assert np.array_equal(host(gb), db)


@pytest.mark.parametrize("fmt", ["dd", "qd"])
def test_int8_diagonal_sums_bit_exact(mp, orc, fmt):
    m, n, k = 150, 130, 200
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=9)
    D = mp.num_slices(fmt, "int8", k)
    da, _ = orc.split_int8(A, D, "rows")
    db, _ = orc.split_int8(B, D, "cols")
    S = orc.int8_diag_sums(da, db)
    dA, dB = dev(A), dev(B)
    for g in sorted({1, 2, D // 2, D}):
        say(f"int8 diagonal {fmt} g={g} D={D}")
        got = host(mp.debug_products(fmt, dA, dB, g, 0, D, mode="int8"))
        assert np.array_equal(got, S[g - 1]), g


@pytest.mark.parametrize("fmt,m,n,k,E", [
    ("dd", 128, 128, 128, 8),
    ("dd", 200, 150, 333, 16),
    ("td", 200, 150, 333, 16),
    ("qd", 200, 150, 333, 16),
    ("qd", 1, 1, 1, 0),
    ("td", 130, 3, 65, 8),
    ("dd", 5, 129, 700, 16),
])
def test_int8_gemm_meets_bound(mp, orc, fmt, m, n, k, E):
    A, B = W.gen_pair(fmt, m, n, k, E=E, seed=m * n + k)
    say(f"int8 gemm {fmt} m={m} n={n} k={k} E={E}")
    C = host(mp.gemm(fmt, dev(A), dev(B), mode="int8"))
    D = mp.last_num_slices()
    diff, absab, _ = orc.exact_check(A, B, C)
    ok, worst = orc.bound_report(diff, absab, T_BITS[fmt])
    say(f"  D={D} worst log2 ratio {worst:.1f} (bound -{T_BITS[fmt]})")
    assert ok
    # the oracle's INT8-form product with the same D: both round the same exact sum
    Co = orc.int8_gemm(A, B, D)
    assert np.array_equal(C[0], Co[0]) or np.max(np.abs(C[0] - Co[0]) / np.maximum(np.abs(Co[0]), 1e-300)) < 2.0 ** -100


def test_int8_zero_rows_and_chunking(mp, orc):
    """Zero rows/columns give zero output; a long k (several 32-bit chunks for
    D = 40) still gives exact diagonal sums."""
    import torch
    m, n, k = 70, 66, 14000
    A, B = W.gen_pair("dd", m, n, k, E=4, seed=5)
    A[:, :, 3] = 0.0
    D = 40
    C = host(mp.gemm("dd", dev(A), dev(B), mode="int8", slices=D))
    assert np.all(C[:, :, 3] == 0)
    rows = [0, 3, 69]
    diff, absab, _ = orc.exact_check(A, B, C, rows=rows)
    ok, worst = orc.bound_report(diff, absab, 100)
    say(f"  chunked k={k} D={D} worst {worst:.1f}")
    assert ok


@pytest.mark.parametrize("cfg", [1, 3, 4])
@pytest.mark.parametrize("fmt,m,n,k,D", [("dd", 70, 90, 60, 0), ("td", 300, 40, 170, 0), ("qd", 33, 270, 420, 0),
                                         ("dd", 20, 12, 14500, 37)])
def test_int8_short_last_step(mp, orc, cfg, fmt, m, n, k, D):
    """k padded to 64: with 128-deep steps (configurations 1, 3 and 4) a pair's
    last step in a k chunk holds 64 k when the chunk's 32-wide k blocks are 2
    mod 4 (k = 60, 170, 420; and D = 37, whose 32-bit chunks are 442 blocks,
    at k = 14500): diagonal sums bit-exact, C within the bound."""
    A, B = W.gen_pair(fmt, m, n, k, E=8, seed=k + cfg)
    D = D or mp.num_slices(fmt, "int8", k)
    da, _ = orc.split_int8(A, D, "rows")
    db, _ = orc.split_int8(B, D, "cols")
    S = orc.int8_diag_sums(da, db)
    dA, dB = dev(A), dev(B)
    say(f"int8 short last step cfg={cfg} {fmt} {m}x{n}x{k} D={D}")
    mp.set_int8_tile(cfg)
    try:
        for g in sorted({1, D // 2, D}):
            got = host(mp.debug_products(fmt, dA, dB, g, 0, D, mode="int8"))
            assert np.array_equal(got, S[g - 1]), g
        C = host(mp.gemm(fmt, dA, dB, mode="int8", slices=D))
    finally:
        mp.set_int8_tile(0)
    rows = None if m * n * k < 5e6 else [0, m // 2, m - 1]
    diff, absab, _ = orc.exact_check(A, B, C, rows=rows)
    ok, worst = orc.bound_report(diff, absab, T_BITS[fmt])
    assert ok, worst


@pytest.mark.parametrize("cfg", [1, 2, 3, 4])
def test_int8_every_tile_config(mp, orc, cfg):
    """Each INT8 tile configuration gives the exact diagonal sums and a C within
    the bound (sizes span several 256-wide tiles with ragged edges)."""
    m, n, k = 300, 270, 200
    A, B = W.gen_pair("td", m, n, k, E=16, seed=61)
    D = mp.num_slices("td", "int8", k)
    da, _ = orc.split_int8(A, D, "rows")
    db, _ = orc.split_int8(B, D, "cols")
    S = orc.int8_diag_sums(da, db)
    say(f"int8 tile config {cfg}")
    mp.set_int8_tile(cfg)
    try:
        C = host(mp.gemm("td", dev(A), dev(B), mode="int8"))
        got = host(mp.debug_products("td", dev(A), dev(B), D // 2, 0, D, mode="int8"))
    finally:
        mp.set_int8_tile(0)
    assert np.array_equal(got, S[D // 2 - 1])
    diff, absab, _ = orc.exact_check(A, B, C)
    ok, worst = orc.bound_report(diff, absab, 150)
    assert ok, worst
