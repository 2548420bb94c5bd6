"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

* slices and exponents of the split: bit-exact;
* every slice product C_ab: bit-exact;
* C: |C - AB| <= 2^-t (|A||B|) elementwise against the exact product, with
  t = 100 / 150 / 200 / 66 (DD / TD / QD / TS), the log2 of the worst ratio
  printed for every case.
"""
import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu

FMTS = ["dd", "td", "qd", "ts"]
T_BITS = {"dd": 100, "td": 150, "qd": 200, "ts": 66}


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_09960_amd as mp
    mp.lib()  # must load: there is no fallback
    assert mp.check_device() == 0, "device is not gfx950"
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


@pytest.fixture
def split_kernel(mp):
    """Select the split kernel for one test and restore the default after."""
    def use(kind):
        mp.set_split_kernel(kind)
    yield use
    mp.set_split_kernel(0)


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("E", [0, 16])
@pytest.mark.parametrize("kind", [0, 1], ids=["fused", "passes"])
def test_split_bit_exact(mp, orc, split_kernel, fmt, E, kind):
    m, k, n = 130, 75, 70
    A, B = W.gen_pair(fmt, m, n, k, E=E, seed=100 + E)
    D = mp.num_slices(fmt, "float", k)
    split_kernel(kind)
    say(f"split {fmt} E={E} m={m} n={n} k={k} D={D} kernel={kind}")
    sa, ea = orc.split_plain(A, D, "rows")
    sb, eb = orc.split_plain(B, D, "cols")
    ga, gea = mp.debug_split(fmt, dev(A), 0, D)
    gb, geb = mp.debug_split(fmt, dev(B), 1, D)
    assert np.array_equal(host(ga), sa)
    assert np.array_equal(host(gea), ea)
    assert np.array_equal(host(gb), sb)
    assert np.array_equal(host(geb), eb)


# Shapes around the fused split's limits: 16, 8, 4 and 2 vectors per
# workgroup, the longest fused k of QD (4096) and TD (5120), and k just past
# them (one launch per pass even in automatic mode), with ragged m and n.
FUSED_EDGE = [(300, 200, 1000), (70, 45, 2050), (33, 17, 4096), (21, 9, 4097), (7, 12, 5120), (5, 3, 8200)]


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("m,n,k", FUSED_EDGE)
def test_split_kernels_agree(mp, split_kernel, fmt, m, n, k):
    """The fused split and the per-pass split give the same slices, exponents
    and C, bit for bit (the per-pass split is checked against the oracle at
    small sizes above)."""
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=m + n + k)
    dA, dB = dev(A), dev(B)
    D = mp.num_slices(fmt, "float", k)
    say(f"split kernels {fmt} m={m} n={n} k={k} D={D}")
    out = []
    for kind in (0, 1):
        split_kernel(kind)
        ga, gea = mp.debug_split(fmt, dA, 0, D)
        gb, geb = mp.debug_split(fmt, dB, 1, D)
        C = mp.gemm(fmt, dA, dB)
        out.append([host(x) for x in (ga, gea, gb, geb, C)])
    for x, y in zip(*out):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("fmt", FMTS)
def test_slice_products_bit_exact(mp, orc, fmt):
    m, n, k = 70, 90, 300
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=7)
    D = mp.num_slices(fmt, "float", k)
    S = 24 if fmt == "ts" else 53
    rho = orc.rho(S, k)
    sa, ea = orc.split_plain(A, D, "rows")
    sb, eb = orc.split_plain(B, D, "cols")
    dA, dB = dev(A), dev(B)
    for a, b in sorted({(1, 1), (1, D), (D, 1), (2, 2), (1, 2), (D // 2, D // 2 + 1)}):
        if a + b > D + 1 or a < 1 or b < 1:
            continue
        say(f"product {fmt} pair ({a},{b}) D={D}")
        want = orc.slice_product(sa[a - 1], ea[a - 1], sb[b - 1], eb[b - 1], rho, S)
        got = host(mp.debug_products(fmt, dA, dB, a, b, D))
        assert np.array_equal(got, want), (a, b, np.max(np.abs(got - want)))


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("kind", [0, 1], ids=["fused", "passes"])
def test_literal_last_slice(mp, orc, split_kernel, fmt, kind):
    """Algorithm 1 as printed (last slice = leading component of the residual
    after D - 1 passes): slices and exponents bit-exact against the oracle in
    both split kernels, and C, whose products with the full-width last slice
    are rounded, still within 2^-t |A||B| (the log2 of the worst ratio is
    printed beside the extracting reading's)."""
    m, k, n = 130, 75, 70
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=140)
    D = mp.num_slices(fmt, "float", k)
    dA, dB = dev(A), dev(B)
    split_kernel(kind)
    try:
        mp.set_last_slice("remainder")
        say(f"literal last slice {fmt} m={m} n={n} k={k} D={D} kernel={kind}")
        sa, ea = orc.split_plain(A, D, "rows", last="remainder")
        sb, eb = orc.split_plain(B, D, "cols", last="remainder")
        ga, gea = mp.debug_split(fmt, dA, 0, D)
        gb, geb = mp.debug_split(fmt, dB, 1, D)
        assert np.array_equal(host(ga), sa) and np.array_equal(host(gea), ea)
        assert np.array_equal(host(gb), sb) and np.array_equal(host(geb), eb)
        lit = host(mp.gemm(fmt, dA, dB))
    finally:
        mp.set_last_slice("extract")
    ext = host(mp.gemm(fmt, dA, dB))
    ok, worst = _check_bound(orc, fmt, A, B, lit)
    _, worst_ext = _check_bound(orc, fmt, A, B, ext)
    say(f"  log2 worst ratio: remainder {worst:.1f}, extract {worst_ext:.1f}")
    assert ok, worst


def _check_bound(orc, fmt, A, B, C, rows=None):
    diff, absab, _ = orc.exact_check(A, B, C, rows=rows)
    ok, worst = orc.bound_report(diff, absab, T_BITS[fmt])
    return ok, worst


@pytest.mark.parametrize("fmt,m,n,k,E", [
    ("dd", 128, 128, 128, 8),   # DD, m = n = k = 128, e ~ U{0..8}
    ("dd", 200, 150, 333, 16),
    ("td", 200, 150, 333, 16),
    ("qd", 200, 150, 333, 16),
    ("ts", 200, 150, 333, 16),
    ("qd", 64, 64, 64, 0),
    ("dd", 1, 1, 1, 8),
    ("td", 1, 77, 5, 8),
    ("qd", 77, 1, 130, 8),
    ("ts", 65, 63, 1, 16),
])
def test_gemm_meets_bound(mp, orc, fmt, m, n, k, E):
    A, B = W.gen_pair(fmt, m, n, k, E=E, seed=m + n + k)
    say(f"gemm {fmt} m={m} n={n} k={k} E={E}")
    C = host(mp.gemm(fmt, dev(A), dev(B)))
    D = mp.last_num_slices()
    ok, worst = _check_bound(orc, fmt, A, B, C)
    say(f"  D={D} worst log2(|C-AB|/|A||B|) = {worst:.1f} (bound -{T_BITS[fmt]})")
    assert ok


def test_deterministic_and_identical_to_single_calls(mp):
    import torch
    A, B = W.gen_pair("td", 150, 130, 257, E=16, seed=3)
    dA, dB = dev(A), dev(B)
    C1 = host(mp.gemm("td", dA, dB))
    C2 = host(mp.gemm("td", dA, dB))
    assert np.array_equal(C1, C2)
    # the same product computed on another stream
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        C3 = mp.gemm("td", dA, dB, stream=s)
    s.synchronize()
    assert np.array_equal(C3.cpu().numpy(), C1)


def test_edge_cases(mp, orc):
    import torch
    # k = 0: C is zeroed
    C = torch.full((2, 5, 4), 7.0, dtype=torch.float64, device="cuda")
    A = torch.zeros((2, 0, 4), dtype=torch.float64, device="cuda")
    B = torch.zeros((2, 5, 0), dtype=torch.float64, device="cuda")
    mp.gemm("dd", A, B, C)
    assert torch.all(C == 0)
    # m = 0: no work, no error
    A = torch.zeros((2, 3, 0), dtype=torch.float64, device="cuda")
    B = torch.ones((2, 5, 3), dtype=torch.float64, device="cuda")
    C = torch.zeros((2, 5, 0), dtype=torch.float64, device="cuda")
    mp.gemm("dd", A, B, C)
    # zero operand and zero rows
    A, B = W.gen_pair("qd", 33, 20, 40, E=4, seed=1)
    A[:, :, 5] = 0.0
    B[:, 7, :] = 0.0
    C = host(mp.gemm("qd", dev(A), dev(B)))
    assert np.all(C[:, :, 5] == 0) and np.all(C[:, 7, :] == 0)
    ok, worst = _check_bound(orc, "qd", A, B, C)
    assert ok
    Z = np.zeros_like(A)
    C = host(mp.gemm("qd", dev(Z), dev(B)))
    assert np.all(C == 0)


def test_identity_gives_input(mp, orc):
    m, k = 40, 48
    A = W.gen_matrix("dd", m, k, E=4, seed=6, operand="A")
    B = np.zeros((2, k, k))
    B[0] = np.eye(k)
    C = host(mp.gemm("dd", dev(A), dev(B), slices=12))
    for i in range(0, m, 7):
        for j in range(0, k, 5):
            assert list(C[:, j, i]) == list(orc.exact_sum(list(A[:, j, i]), 2))


def test_power_of_two_scaling_exact(mp):
    A, B = W.gen_pair("dd", 96, 80, 100, E=8, seed=12)
    C = host(mp.gemm("dd", dev(A), dev(B)))
    A2 = A.copy()
    A2[:, :, 3] *= 2.0 ** 37
    B2 = B.copy()
    B2[:, 2, :] *= 2.0 ** -21
    C2 = host(mp.gemm("dd", dev(A2), dev(B2)))
    expect = C.copy()
    expect[:, :, 3] *= 2.0 ** 37
    expect[:, 2, :] *= 2.0 ** -21
    assert np.array_equal(C2, expect)


@pytest.mark.parametrize("fmt,mode", [("dd", "float"), ("qd", "float"), ("dd", "int8"), ("qd", "int8"),
                                      ("ts", "float")])
def test_edges_of_the_magnitude_range(mp, orc, fmt, mode):
    """Rows and columns scaled to the edges of the documented input range
    (binary64 formats: |x| in [2^-400, 2^400]; TS: [2^-16, 2^40]), so that
    slices, slice products and C sit near the ends of the exponent range:
    every entry within the bound of the exact product, and rows scaled by a
    power of two give results scaled by it, bit for bit."""
    m, n, k = 70, 60, 150
    A, B = W.gen_pair(fmt, m, n, k, E=8, seed=77)
    hi, lo = (31, -6) if fmt == "ts" else (390, -390)
    A[:, :, : m // 2] *= 2.0 ** hi  # products near 2^(hi - 10) for the top-left block
    B[:, : n // 3, :] *= 2.0 ** (lo + 8)
    A[:, :, m // 2:] *= 2.0 ** lo
    C = host(mp.gemm(fmt, dev(A), dev(B), mode=mode))
    ok, worst = _check_bound(orc, fmt, A, B, C)
    say(f"magnitude edges {fmt} {mode}: worst {worst:.1f}")
    assert ok, worst
    assert np.all(np.isfinite(C))
    if fmt != "ts":
        A2 = A.copy()
        A2[:, :, 5] *= 2.0 ** -7
        C2 = host(mp.gemm(fmt, dev(A2), dev(B), mode=mode))
        expect = C.copy()
        expect[:, :, 5] *= 2.0 ** -7
        assert np.array_equal(C2, expect)


def test_attached_workspace(mp):
    import torch
    A, B = W.gen_pair("dd", 100, 90, 120, E=8, seed=2)
    dA, dB = dev(A), dev(B)
    C1 = host(mp.gemm("dd", dA, dB))
    need = mp.workspace_bytes("dd", "float", 100, 90, 120)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    mp.set_workspace(ws)
    try:
        C2 = host(mp.gemm("dd", dA, dB))
        small = ws[: need // 2]
        mp.set_workspace(small)
        with pytest.raises(mp.MpgemmError) as ei:
            mp.gemm("dd", dA, dB)
        assert ei.value.status == 2
    finally:
        mp.set_workspace(None)
    assert np.array_equal(C1, C2)


@pytest.mark.parametrize("layout", [1, 2, 3])
@pytest.mark.parametrize("fmt", ["dd", "qd", "ts"])
def test_every_tile_layout(mp, orc, fmt, layout):
    """Every wavefront layout gives the same slice products (bit-exact) and a C
    within the bound; layouts only reorder independent work."""
    m, n, k = 150, 130, 333
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=51)
    say(f"layout {layout} {fmt}")
    mp.set_tile_layout(fmt, layout)
    try:
        C = host(mp.gemm(fmt, dev(A), dev(B)))
        D = mp.last_num_slices()
        P = host(mp.debug_products(fmt, dev(A), dev(B), 1, D, D))
    finally:
        mp.set_tile_layout(fmt, 0)
    ok, worst = _check_bound(orc, fmt, A, B, C)
    assert ok, worst
    S = 24 if fmt == "ts" else 53
    sa, ea = orc.split_plain(A, D, "rows")
    sb, eb = orc.split_plain(B, D, "cols")
    assert np.array_equal(P, orc.slice_product(sa[0], ea[0], sb[D - 1], eb[D - 1], orc.rho(S, k), S))


@pytest.mark.parametrize("fmt,mode,fewer", [("dd", "float", 2), ("qd", "float", 2), ("dd", "int8", 3),
                                            ("qd", "int8", 3)])
def test_automatic_slice_count_is_tight(mp, orc, fmt, mode, fewer):
    """The automatic D meets the bound, and its guard is at most one slice
    (binary64 slices, about 21 bits at k = 1024) or two digits (INT8, 7 bits
    each): two slices or three digits fewer miss the bound on the same inputs
    (e ~ U{0..16}, k = 1024)."""
    m, n, k = 64, 48, 1024
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=99)
    dA, dB = dev(A), dev(B)
    D = mp.num_slices(fmt, mode, k)
    C = host(mp.gemm(fmt, dA, dB, mode=mode))
    ok, worst = _check_bound(orc, fmt, A, B, C)
    Cf = host(mp.gemm(fmt, dA, dB, mode=mode, slices=D - fewer))
    ok_f, worst_f = _check_bound(orc, fmt, A, B, Cf)
    say(f"{fmt} {mode}: D={D} worst {worst:.1f}; D={D - fewer} worst {worst_f:.1f} (bound -{T_BITS[fmt]})")
    assert ok and not ok_f


def test_slice_autotuner_table(mp, orc, tmp_path):
    """The autotuner's slice counts, loaded as a table, give products within the
    bound (checked exactly) on inputs it did not tune on."""
    from paper_2301_09960_amd import tune
    lines = tune.slice_table([("dd", "float"), ("qd", "int8")], ks=(128, 512), size=64, seeds=(1,))
    f = tmp_path / "slices.txt"
    f.write_text("\n".join(lines) + "\n")
    try:
        mp.load_tune_file(f)
        for fmt, mode, k in (("dd", "float", 100), ("dd", "float", 512), ("qd", "int8", 300)):
            A, B = W.gen_pair(fmt, 48, 40, k, E=16, seed=777)
            C = host(mp.gemm(fmt, dev(A), dev(B), mode=mode))
            D = mp.last_num_slices()
            want = [int(l.split()[4]) for l in lines if l.split()[1:3] == [fmt, mode] and int(l.split()[3]) >= k][0]
            assert D == want
            ok, worst = _check_bound(orc, fmt, A, B, C)
            say(f"tuned {fmt} {mode} k={k}: D={D} worst {worst:.1f} (bound -{T_BITS[fmt]})")
            assert ok
    finally:
        mp.load_tune_file(None)
