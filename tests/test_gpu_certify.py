"""GPU: the a-posteriori certificate (mpgemm_certify) against the oracle.

* C is the product mpgemm_<fmt> computes, bit for bit;
* the error bound beta dominates the oracle's exact truncation bound T1 + T2 +
  T3 and stays within 2^-30 of it plus the final-rounding term, and it bounds
  the actual |C - AB| (exact arithmetic) in every entry;
* lambda is a lower bound of (|A||B|)_ij within a few ulps of it;
* the automatic slice counts are certified (worst <= 2^-t); too few are not.
"""
from fractions import Fraction

import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu

T_BITS = {"dd": 100, "td": 150, "qd": 200, "ts": 66}
SC = {"dd": 106, "td": 159, "qd": 212, "ts": 72}  # S * c


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_09960_amd as mp
    mp.lib()
    assert mp.check_device() == 0, "device is not gfx950"
    return mp


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("fmt,mode", [("dd", "float"), ("td", "float"), ("qd", "float"), ("ts", "float"),
                                      ("dd", "int8"), ("td", "int8"), ("qd", "int8")])
def test_certificate_against_oracle(mp, orc, fmt, mode):
    import torch
    m, n, k = 9, 7, 37
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=41)
    dA, dB = dev(A), dev(B)
    C, cert, worst = mp.certify(fmt, dA, dB, mode=mode)
    D = mp.last_num_slices()
    say(f"certify {fmt} {mode} m={m} n={n} k={k} D={D}")
    ref = mp.gemm(fmt, dA, dB, mode=mode)
    torch.cuda.synchronize()
    assert torch.equal(C, ref)
    beta, lam = cert[0].cpu().numpy(), cert[1].cpu().numpy()  # (n, m)
    tr, t1, t23, absab = orc.certificate_terms(A, B, D, form=mode)
    diff, _, _ = orc.exact_check(A, B, C.cpu().numpy())  # (n, m): |C - AB| rounded once
    ratios = []
    for i in range(m):
        for j in range(n):
            b, l = Fraction(float(beta[j, i])), Fraction(float(lam[j, i]))
            T = t1[i][j] + t23[i][j]
            assert T <= b <= T * (1 + Fraction(2) ** -30) + Fraction(2) ** (6 - SC[fmt]) * absab[i][j], (i, j)
            # lambda gives up (k + 2) 2^-52 for the rounding of |A_0||B_0| and
            # 2^(2 - S) per factor for |x_0| against |x|
            slack = (k + 2) * Fraction(2) ** -52 + Fraction(2) ** (3 - (24 if fmt == "ts" else 53))
            assert absab[i][j] * (1 - 2 * slack) <= l <= absab[i][j], (i, j)
            assert diff[j, i] <= float(beta[j, i]) * (1 + 2.0 ** -50), (i, j)
            ratios.append(float(beta[j, i]) / float(lam[j, i]))
    w = float(worst.cpu()[0])
    assert abs(w - max(ratios)) <= 2.0 ** -40 * max(ratios)
    say(f"  log2 worst beta/lambda {np.log2(w):.1f} (t = {T_BITS[fmt]})")


@pytest.mark.parametrize("fmt,mode,m,n,k,extra", [("dd", "float", 300, 200, 1000, 0), ("td", "float", 130, 70, 600, 0),
                                                  ("qd", "float", 200, 150, 333, 0), ("ts", "float", 256, 129, 700, 1),
                                                  ("dd", "float", 4096, 4096, 4096, 0),
                                                  ("dd", "int8", 300, 200, 1000, 0), ("td", "int8", 130, 70, 600, 0),
                                                  ("qd", "int8", 200, 150, 333, 0),
                                                  ("qd", "int8", 4096, 4096, 4096, 1)])
def test_certified_at_automatic_slices(mp, orc, fmt, mode, m, n, k, extra):
    """The automatic slice counts certify DD / TD / QD on the workload; TS (7 to
    9 bits per binary32 slice) and INT8 QD at k = 4096 need one slice more,
    since the bound takes every left-out pair at its largest.  The bound also
    holds against the exact error on sampled rows."""
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=m + k)
    D = mp.num_slices(fmt, mode, k) + extra
    C, cert, worst = mp.certify(fmt, dev(A), dev(B), mode=mode, slices=D)
    w = float(worst.cpu()[0])
    say(f"certify {fmt} {mode} {m}x{n}x{k} D={mp.last_num_slices()}: log2 worst {np.log2(w):.1f} "
        f"(t = {T_BITS[fmt]})")
    assert w <= 2.0 ** -T_BITS[fmt]
    rows = [0, m // 2, m - 1]
    diff, _, _ = orc.exact_check(A, B, C.cpu().numpy(), rows=rows)
    beta = cert[0].cpu().numpy()
    for c, i in enumerate(rows):
        assert np.all(diff[:, c] <= beta[:, i] * (1 + 2.0 ** -50))


def test_too_few_slices_not_certified(mp, orc):
    """D = 3 for DD cannot reach 2^-100: the certificate says so, and its bound
    still holds against the exact error."""
    m, n, k = 40, 30, 200
    A, B = W.gen_pair("dd", m, n, k, E=16, seed=5)
    C, cert, worst = mp.certify("dd", dev(A), dev(B), slices=3)
    w = float(worst.cpu()[0])
    say(f"certify dd D=3: log2 worst {np.log2(w):.1f}")
    assert w > 2.0 ** -100
    diff, _, _ = orc.exact_check(A, B, C.cpu().numpy())
    assert np.all(diff <= cert[0].cpu().numpy() * (1 + 2.0 ** -50))


def test_zero_lines_and_empty(mp):
    import torch
    m, n, k = 20, 18, 33
    A, B = W.gen_pair("qd", m, n, k, E=8, seed=9)
    A[:, :, 3] = 0.0   # row 3 of A
    B[:, 5, :] = 0.0   # column 5 of B
    C, cert, worst = mp.certify("qd", dev(A), dev(B))
    beta, lam = cert[0].cpu().numpy(), cert[1].cpu().numpy()
    assert np.all(beta[:, 3] == 0) and np.all(lam[:, 3] == 0)
    assert np.all(beta[5, :] == 0) and np.all(lam[5, :] == 0)
    assert float(worst.cpu()[0]) <= 2.0 ** -200
    # k = 0: C = 0, nothing to bound
    A0 = torch.zeros((4, 0, 6), dtype=torch.float64, device="cuda")
    B0 = torch.zeros((4, 5, 0), dtype=torch.float64, device="cuda")
    C0, cert0, worst0 = mp.certify("qd", A0, B0)
    assert not C0.any() and not cert0.any() and float(worst0.cpu()[0]) == 0.0


def test_thread_mode_and_unsupported(mp):
    """The C entry point follows the thread's slice form (INT8 here: same C as
    the INT8 product); the printed last slice is refused."""
    import torch
    A, B = W.gen_pair("dd", 8, 8, 8, E=0, seed=1)
    dA, dB = dev(A), dev(B)
    mp.set_mode("dd", "int8")
    try:
        C = _certify_in_mode(mp, dA, dB)
        ref = mp.gemm("dd", dA, dB)
        torch.cuda.synchronize()
        assert torch.equal(C, ref)
    finally:
        mp.set_mode("dd", "float")
    mp.set_last_slice("remainder")
    try:
        with pytest.raises(mp.MpgemmError):
            mp.certify("dd", dA, dB)
    finally:
        mp.set_last_slice("extract")


def _certify_in_mode(mp, dA, dB):
    """Calls the C entry point directly, with the thread's (INT8) mode in force."""
    import ctypes

    import torch
    m, k = dA.shape[2], dA.shape[1]
    n = dB.shape[1]
    C = torch.empty((2, n, m), dtype=torch.float64, device="cuda")
    cert = torch.empty((2, n, m), dtype=torch.float64, device="cuda")
    worst = torch.empty((1,), dtype=torch.float64, device="cuda")
    P = ctypes.c_void_p
    st = mp.lib().mpgemm_certify(mp.FORMATS["dd"], m, n, k, P(dA.data_ptr()), m, P(dB.data_ptr()), k,
                                 P(C.data_ptr()), m, P(cert.data_ptr()), P(worst.data_ptr()),
                                 P(torch.cuda.current_stream().cuda_stream))
    if st != 0:
        raise mp.MpgemmError(st, "mpgemm_certify")
    return C


@pytest.mark.parametrize("c", [6, 10])
def test_nd_certificate(mp, orc, c):
    """Longer expansions (INT8 form, c components): the bound against the
    oracle's exact terms and the exact error, and certification at the
    automatic digit count (target 2^-(50 c))."""
    import torch
    m, n, k = 8, 7, 29
    A, B = W.gen_pair(f"{c}d", m, n, k, E=8, seed=c)
    dA, dB = dev(A), dev(B)
    C, cert, worst = mp.nd_certify(dA, dB)
    ref = mp.gemm_nd(dA, dB)
    torch.cuda.synchronize()
    assert torch.equal(C, ref)
    D = mp.nd_num_slices(c, k)
    beta, lam = cert[0].cpu().numpy(), cert[1].cpu().numpy()
    _, t1, t23, absab = orc.certificate_terms(A, B, D, form="int8")
    diff, _, _ = orc.exact_check(A, B, C.cpu().numpy())
    for i in range(m):
        for j in range(n):
            b = Fraction(float(beta[j, i]))
            T = t1[i][j] + t23[i][j]
            assert T <= b <= T * (1 + Fraction(2) ** -30) + Fraction(2) ** (6 - 53 * c) * absab[i][j], (i, j)
            assert float(lam[j, i]) <= absab[i][j]
            assert diff[j, i] <= float(beta[j, i]) * (1 + 2.0 ** -50)
    w = float(worst.cpu()[0])
    say(f"nd certify c={c} D={D}: log2 worst {np.log2(w):.1f} (target {-50 * c})")
    assert w <= 2.0 ** (-50 * c)
    # a larger shape with a wider spread: certified with one digit more than
    # the automatic count (the bound takes every left-out pair at its largest)
    A2, B2 = W.gen_pair(f"{c}d", 130, 90, 300, E=16, seed=c + 1)
    D2 = mp.nd_num_slices(c, 300) + 1
    _, _, worst2 = mp.nd_certify(dev(A2), dev(B2), slices=D2)
    w2 = float(worst2.cpu()[0])
    say(f"nd certify c={c} 130x90x300 D={D2}: log2 worst {np.log2(w2):.1f}")
    assert w2 <= 2.0 ** (-50 * c)


@pytest.mark.parametrize("mode", ["float", "int8"])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (1, 5, 3), (6, 1, 70), (3, 4, 1)])
def test_certificate_thin_shapes(mp, orc, mode, m, n, k):
    """Single rows, columns and k = 1: the bound still dominates the oracle's
    exact terms and the exact error."""
    A, B = W.gen_pair("dd", m, n, k, E=8, seed=m * 100 + n * 10 + k)
    C, cert, worst = mp.certify("dd", dev(A), dev(B), mode=mode)
    D = mp.last_num_slices()
    beta = cert[0].cpu().numpy()
    _, t1, t23, _ = orc.certificate_terms(A, B, D, form=mode)
    diff, _, _ = orc.exact_check(A, B, C.cpu().numpy())
    for i in range(m):
        for j in range(n):
            assert t1[i][j] + t23[i][j] <= Fraction(float(beta[j, i]))
            assert diff[j, i] <= float(beta[j, i]) * (1 + 2.0 ** -50)
    assert float(worst.cpu()[0]) <= 2.0 ** -100


@pytest.mark.parametrize("fmt,mode,E", [("dd", "float", 0), ("dd", "float", 16), ("qd", "float", 0),
                                        ("td", "int8", 0), ("dd", "int8", 16)])
def test_adaptive_slice_count(mp, orc, fmt, mode, E):
    """mpgemm_certify_adaptive stops at the first certified D: its C, cert and
    worst equal mpgemm_certify's at that D, worst meets 2^-t, one slice fewer
    does not, and |C - AB| (exact) is within the certificate in every entry."""
    import torch
    m, n, k = 48, 40, 300
    A, B = W.gen_pair(fmt, m, n, k, E=E, seed=61)
    dA, dB = dev(A), dev(B)
    auto = mp.num_slices(fmt, mode, k)
    d_first = 2 if mode == "float" else 8
    C, cert, worst, D = mp.certify_adaptive(fmt, dA, dB, d_first=d_first, d_last=auto + 2, mode=mode)
    target = 2.0 ** -T_BITS[fmt]
    w = float(worst.cpu()[0])
    say(f"adaptive {fmt} {mode} E={E} m={m} n={n} k={k}: D = {D} (a-priori {auto}), log2 worst {np.log2(w):.1f}")
    assert d_first <= D <= auto + 2
    assert w <= target
    C2, cert2, worst2 = mp.certify(fmt, dA, dB, mode=mode, slices=D)
    torch.cuda.synchronize()
    assert torch.equal(C, C2) and torch.equal(cert, cert2) and torch.equal(worst, worst2)
    if D > d_first:
        _, _, w1 = mp.certify(fmt, dA, dB, mode=mode, slices=D - 1)
        assert float(w1.cpu()[0]) > target
    beta, lam = cert[0].cpu().numpy(), cert[1].cpu().numpy()
    diff, _, _ = orc.exact_check(A, B, C.cpu().numpy())
    assert (diff <= beta * (1 + 2.0 ** -50)).all()
    assert (beta <= target * lam).all()


def test_adaptive_not_certified(mp):
    """A range that ends too early returns its last attempt, uncertified."""
    import torch
    m, n, k = 33, 17, 200
    A, B = W.gen_pair("dd", m, n, k, E=16, seed=62)
    dA, dB = dev(A), dev(B)
    C, cert, worst, D = mp.certify_adaptive("dd", dA, dB, d_first=2, d_last=3)
    assert D == 3
    assert float(worst.cpu()[0]) > 2.0 ** -100
    C2, _, worst2 = mp.certify("dd", dA, dB, slices=3)
    torch.cuda.synchronize()
    assert torch.equal(C, C2) and torch.equal(worst, worst2)
