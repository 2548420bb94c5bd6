"""GPU: blocked DD LU with the Schur updates by the slice-product GEMM
(Section 4.6), against exact rational checks: the backward error
|A - L U| / (|L||U|) in every entry, and the solution of A x = b against the
exact one.  Diagonally dominant matrices (no pivoting, as in the paper), block
widths spanning one, several and ragged blocks, both slice forms."""
import numpy as np
import pytest

import oracle.exact as X

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_09960_amd as mp
    mp.lib()
    assert mp.check_device() == 0, "device is not gfx950"
    return mp


def say(*a):
    print(*a, flush=True)


def dd_dominant(n, seed, c=2):
    """(c, n, n) DD (TD) matrix: uniform [0, 1) entries with lower components,
    n added on the diagonal."""
    rng = np.random.default_rng(seed)
    hi = rng.random((n, n)) + n * np.eye(n)
    A = np.zeros((c, n, n))
    A[0] = hi.T  # column-major planes: A[r, j, i]
    prev = hi
    for r in range(1, c):
        nxt = (rng.random((n, n)) - 0.5) * np.spacing(prev)  # below half an ulp of the previous component
        A[r] = nxt.T
        prev = np.abs(nxt) + np.finfo(float).tiny
    return A


# bounds: the Schur products meet 2^-t |L21||U12| (t = 100 / 150), the panels
# are DD (TD) arithmetic; a few bits of margin for the sums over blocks
BACKWARD = {"dd": 2.0 ** -92, "td": 2.0 ** -140}
SOLVE = {"dd": 2.0 ** -88, "td": 2.0 ** -135}


@pytest.mark.parametrize("fmt,n,K,mode", [("dd", 40, 16, "float"), ("dd", 40, 8, "float"), ("dd", 40, 64, "float"),
                                          ("dd", 40, 1, "float"), ("dd", 37, 16, "int8"), ("dd", 33, 32, "float"),
                                          ("td", 40, 16, "float"), ("td", 37, 8, "int8"), ("td", 30, 64, "float"),
                                          ("dd", 150, 100, "float"), ("td", 120, 96, "float")])
def test_lu_backward_error(mp, fmt, n, K, mode):
    import torch
    c = 2 if fmt == "dd" else 3
    A = dd_dominant(n, seed=n + K, c=c)
    dA = torch.from_numpy(A.copy()).cuda()
    mp.lu(fmt, dA, K, mode=mode)
    LU = dA.cpu().numpy()
    err = X.lu_backward_error(A, LU)
    say(f"{fmt}_lu n={n} K={K} {mode}: log2 backward error {np.log2(err) if err > 0 else -np.inf:.1f}")
    assert np.isfinite(LU).all()
    assert err <= BACKWARD[fmt]


@pytest.mark.parametrize("fmt", ["dd", "td"])
def test_lu_wide_panel(mp, fmt):
    """K = 520 > 512: the panel solves take the thread-per-vector kernels
    (every step of the substitution in one thread) and the diagonal block is
    factored in inner blocks.  Exact backward error on sampled entries of all
    four blocks, their corners included."""
    import torch
    n, K = 600, 520
    c = 2 if fmt == "dd" else 3
    A = dd_dominant(n, seed=11, c=c)
    dA = torch.from_numpy(A.copy()).cuda()
    mp.lu(fmt, dA, K)
    LU = dA.cpu().numpy()
    assert np.isfinite(LU).all()
    rng = np.random.default_rng(12)
    corners = [(0, 0), (K - 1, K - 1), (n - 1, n - 1), (n - 1, 0), (0, n - 1), (K, K - 1), (K - 1, K),
               (n - 1, K - 1), (K - 1, n - 1), (K, K)]
    blocks = [(0, K, 0, K), (K, n, 0, K), (0, K, K, n), (K, n, K, n)]
    entries = corners + [(int(rng.integers(r0, r1)), int(rng.integers(c0, c1)))
                         for r0, r1, c0, c1 in blocks for _ in range(40)]
    err = X.lu_backward_error(A, LU, entries=entries)
    say(f"{fmt}_lu n={n} K={K}: log2 backward error (sampled) {np.log2(err) if err > 0 else -np.inf:.1f}")
    assert err <= BACKWARD[fmt]


@pytest.mark.parametrize("fmt,n,K", [("dd", 40, 16), ("dd", 24, 24), ("td", 40, 16)])
def test_lu_solve(mp, fmt, n, K):
    import torch
    c = 2 if fmt == "dd" else 3
    A = dd_dominant(n, seed=7 * n, c=c)
    b = np.zeros((c, n))
    # the paper's right-hand side [1, 1/2, ..., 1/n], rounded to c components
    for i in range(1, n + 1):
        rest = X.Fraction(1, i)
        for r in range(c):
            b[r, i - 1] = float(rest)
            rest -= X.Fraction(b[r, i - 1])
    dA = torch.from_numpy(A.copy()).cuda()
    mp.lu(fmt, dA, K)
    x = mp.lu_solve(fmt, dA, torch.from_numpy(b).cuda()).cpu().numpy()
    exact = X.solve_exact(A, b)
    rel = max(abs(X.value(x[:, i]) - exact[i]) / abs(exact[i]) for i in range(n) if exact[i] != 0)
    say(f"{fmt}_lu_solve n={n} K={K}: log2 max relative error {np.log2(float(rel)):.1f}")
    assert rel <= X.Fraction(SOLVE[fmt])


@pytest.mark.parametrize("mode", ["float", "int8"])
def test_lu_residual_n512(mp, orc, mode):
    """n = 512, K = 128 (three Schur updates): the exact residual of the solve,
    |b - A x| against |A||x| in every row."""
    import torch
    n, K = 512, 128
    A = dd_dominant(n, seed=3)
    b = np.zeros((2, n))
    b[0] = 1.0 / np.arange(1, n + 1)
    dA = torch.from_numpy(A.copy()).cuda()
    mp.dd_lu(dA, K, mode=mode)
    x = mp.dd_lu_solve(dA, torch.from_numpy(b).cuda()).cpu().numpy()
    # A x as the product of A (c, k=n, m=n) and x as an n x 1 matrix (c, 1, n)
    diff, absab, _ = orc.exact_check(A, x.reshape(2, 1, n), b.reshape(2, 1, n))
    worst = float(np.max(diff / absab))
    say(f"dd_lu n={n} K={K} {mode}: log2 max |b - A x| / (|A||x|) {np.log2(worst):.1f}")
    assert worst <= 2.0 ** -95


def paper_system(n, seed, c):
    """Section 4.6's test system: a_ij uniform random on [0, 1) (here with
    lower components below half an ulp), b = [1, 1/2, ..., 1/n] rounded to c
    components.  Not diagonally dominant: without pivoting the pivots can be
    small and the factors grow."""
    rng = np.random.default_rng(seed)
    hi = rng.random((n, n))
    A = np.zeros((c, n, n))
    A[0] = hi.T
    prev = hi
    for r in range(1, c):
        nxt = (rng.random((n, n)) - 0.5) * np.spacing(prev)
        A[r] = nxt.T
        prev = np.abs(nxt) + np.finfo(float).tiny
    b = np.zeros((c, n))
    for i in range(1, n + 1):
        rest = X.Fraction(1, i)
        for r in range(c):
            b[r, i - 1] = float(rest)
            rest -= X.Fraction(b[r, i - 1])
    return A, b


@pytest.mark.parametrize("fmt,mode", [("dd", "float"), ("dd", "int8"), ("td", "float")])
def test_lu_paper_system_n512(mp, orc, fmt, mode):
    """Section 4.6's own system at n = 512, K = 128: the exact residual
    |b - A x| in every row against the componentwise backward-error scale
    (|L||U||x|)_i of an elimination without pivoting (the growth of the
    factors included), and the paper's max relative error of x, for DD
    against the TD solution of the same system."""
    import torch
    n, K = 512, 128
    c = 2 if fmt == "dd" else 3
    A, b = paper_system(n, seed=46, c=c)
    dA = torch.from_numpy(A.copy()).cuda()
    mp.lu(fmt, dA, K, mode=mode)
    x = mp.lu_solve(fmt, dA, torch.from_numpy(b).cuda()).cpu().numpy()
    LU = dA.cpu().numpy()[0].T  # leading components, row-major (i, j)
    assert np.isfinite(LU).all() and np.isfinite(x).all()
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    scale = np.abs(L) @ (np.abs(U) @ np.abs(x[0])) * (1 + 2.0 ** -40)  # float64: relative error ~ n 2^-53
    growth = np.max(np.abs(U)) / np.max(np.abs(A[0]))
    diff, _, _ = orc.exact_check(A, x.reshape(c, 1, n), b.reshape(c, 1, n))
    ratio = float(np.max(diff[0] / scale))
    t = {"dd": 100, "td": 150}[fmt]
    rel = None
    if fmt == "dd":
        Ah, bh = paper_system(n, seed=46, c=3)
        dT = torch.from_numpy(Ah.copy()).cuda()
        mp.lu("td", dT, K)
        xt = mp.lu_solve("td", dT, torch.from_numpy(bh).cuda()).cpu().numpy()
        rel = float(np.max(np.abs((x[0] - xt[0]) + (x[1] - xt[1]) - xt[2]) / np.abs(xt[0])))
    say(f"{fmt}_lu paper system n={n} K={K} {mode}: growth {growth:.3g}, log2 max |b - A x| / (|L||U||x|) "
        f"{np.log2(ratio):.1f}" + (f", max relative error of x vs TD {rel:.3g}" if rel is not None else ""))
    # the Schur products meet 2^-t |L21||U12| per update (n / K of them); the
    # panels and the substitutions add up to about n roundings of the format
    # (2^-106 / 2^-159 each, n / 16 in units of 2^-t)
    assert ratio <= (n / K + n / 16) * 2.0 ** -t


def test_lu_edge_cases(mp):
    import torch
    # 1 x 1, and K larger than n
    A = torch.tensor([[[3.0]], [[2.0 ** -60]]], dtype=torch.float64, device="cuda")
    mp.dd_lu(A, 4)
    assert A[0, 0, 0].item() == 3.0 and A[1, 0, 0].item() == 2.0 ** -60
    x = mp.dd_lu_solve(A, torch.tensor([[6.0], [0.0]], dtype=torch.float64, device="cuda"))
    assert abs(x[0, 0].item() - 2.0) < 1e-15
    # n = 0 is a no-op; bad arguments are refused
    E = torch.zeros((2, 0, 0), dtype=torch.float64, device="cuda")
    mp.dd_lu(E, 8)
    with pytest.raises(mp.MpgemmError):
        mp.dd_lu(torch.zeros((2, 4, 4), dtype=torch.float64, device="cuda"), 0)
