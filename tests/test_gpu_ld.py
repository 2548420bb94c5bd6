"""GPU tests of the input contract's leading dimensions, through the C-ABI.

Plane r of A starts at A + r * lda * k, of B at B + r * ldb * n, of C at
C + r * ldc * n (column-major planes, Section 3's C := AB on BLAS-style
operands).  Every case here passes lda > m, ldb > k and ldc > m, with the
padding of A and B filled with NaN (a read of it would poison C) and C's
padding filled with a sentinel that must survive.  The result must equal the
compact call bit for bit and meet the error bound against the oracle.
"""
import ctypes

import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu

T_BITS = {"dd": 100, "td": 150, "qd": 200, "ts": 66}
SENTINEL = -1234.5


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


def say(*a):
    print(*a, flush=True)


def padded(X, ld, fill):
    """Device buffer (c, cols, ld) holding X (c, cols, rows) in its first rows."""
    import torch
    c, cols, rows = X.shape
    buf = torch.full((c, cols, ld), fill, dtype=torch.from_numpy(X[:1, :1, :1]).dtype, device="cuda")
    buf[:, :, :rows] = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    return buf


def check_padding(buf, rows):
    """C's rows beyond m still hold the sentinel, bit for bit."""
    import torch
    pad = buf[:, :, rows:]
    return bool(torch.all(pad == SENTINEL))


CASES = [("dd", "float"), ("td", "float"), ("qd", "float"), ("ts", "float"), ("dd", "int8"), ("qd", "int8")]


@pytest.mark.parametrize("fmt,mode", CASES)
def test_padded_leading_dimensions(mp, orc, fmt, mode):
    import torch
    m, n, k = 150, 97, 333
    lda, ldb, ldc = m + 37, k + 5, m + 11
    A, B = W.gen_pair(fmt, m, n, k, E=16, seed=606)
    say(f"ld {fmt} {mode}: m={m} n={n} k={k} lda={lda} ldb={ldb} ldc={ldc}")
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    compact = mp.gemm(fmt, dA, dB, mode=mode)
    Ab, Bb = padded(A, lda, float("nan")), padded(B, ldb, float("nan"))
    Cb = torch.full((A.shape[0], n, ldc), SENTINEL, dtype=dA.dtype, device="cuda")
    L = mp.lib()
    old = mp.get_mode(fmt)
    mp.set_mode(fmt, mode)
    try:
        st = getattr(L, "mpgemm_" + fmt)(m, n, k, ctypes.c_void_p(Ab.data_ptr()), lda, ctypes.c_void_p(Bb.data_ptr()),
                                         ldb, ctypes.c_void_p(Cb.data_ptr()), ldc,
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    finally:
        mp.set_mode(fmt, old)
    assert st == 0, st
    torch.cuda.synchronize()
    assert check_padding(Cb, m), "C's padding was written"
    got = Cb[:, :, :m]
    assert torch.equal(got, compact), "strided call differs from the compact call"
    diff, absab, _ = orc.exact_check(A, B, got.cpu().numpy())
    ok, worst = orc.bound_report(diff, absab, T_BITS[fmt])
    say(f"  worst log2 ratio {worst:.1f} (bound -{T_BITS[fmt]})")
    assert ok


@pytest.mark.parametrize("fmt,mode", [("dd", "float"), ("ts", "float"), ("qd", "int8")])
def test_binding_views_pass_their_leading_dimension(mp, fmt, mode):
    """The binding turns views X[:, :, :rows] of wider buffers into the
    buffers' leading dimensions (no copies): the same C as the compact call,
    C's padding untouched; also through the certified product."""
    import torch
    m, n, k = 70, 45, 129
    A, B = W.gen_pair(fmt, m, n, k, E=8, seed=607)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    Ab, Bb = padded(A, m + 3, float("nan")), padded(B, k + 64, float("nan"))
    Cb = torch.full((A.shape[0], n, m + 9), SENTINEL, dtype=dA.dtype, device="cuda")
    compact = mp.gemm(fmt, dA, dB, mode=mode)
    out = mp.gemm(fmt, Ab[:, :, :m], Bb[:, :, :k], Cb[:, :, :m], mode=mode)
    torch.cuda.synchronize()
    assert out.data_ptr() == Cb.data_ptr()
    assert torch.equal(Cb[:, :, :m], compact) and check_padding(Cb, m)
    if fmt != "ts":
        C1, cert1, w1 = mp.certify(fmt, dA, dB, mode=mode)
        Cb.fill_(SENTINEL)
        _, cert2, w2 = mp.certify(fmt, Ab[:, :, :m], Bb[:, :, :k], Cb[:, :, :m], mode=mode)
        torch.cuda.synchronize()
        assert torch.equal(Cb[:, :, :m], C1) and check_padding(Cb, m)
        assert torch.equal(cert1, cert2) and torch.equal(w1, w2)


@pytest.mark.parametrize("fmt,mode", [("dd", "float"), ("qd", "float"), ("ts", "float"), ("dd", "int8"),
                                      ("qd", "int8")])
def test_batched_mixed_leading_dimensions(mp, fmt, mode):
    """A batch whose products have different paddings (some compact): each
    equals its compact single call bit for bit, paddings untouched."""
    import torch
    sh = [(37, 21, 64), (1, 5, 7), (130, 66, 257), (64, 64, 64), (9, 1, 300), (200, 150, 1000)]
    pads = [(0, 0, 0), (3, 1, 2), (37, 5, 11), (1, 0, 64), (0, 9, 0), (17, 3, 5)]
    As, Bs, Cs, bufs, singles = [], [], [], [], []
    for i, ((m, n, k), (pa, pb, pc)) in enumerate(zip(sh, pads)):
        A, B = W.gen_pair(fmt, m, n, k, E=8, seed=700 + i)
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        singles.append(mp.gemm(fmt, dA, dB, mode=mode))
        Ab, Bb = padded(A, m + pa, float("nan")), padded(B, k + pb, float("nan"))
        Cb = torch.full((A.shape[0], n, m + pc), SENTINEL, dtype=dA.dtype, device="cuda")
        As.append(Ab[:, :, :m])
        Bs.append(Bb[:, :, :k])
        Cs.append(Cb[:, :, :m])
        bufs.append(Cb)
    say(f"batched ld {fmt} {mode}: {len(sh)} products")
    mp.gemm_batched(fmt, As, Bs, Cs, mode=mode)
    torch.cuda.synchronize()
    for i, (m, n, k) in enumerate(sh):
        assert torch.equal(Cs[i], singles[i]), (i, sh[i])
        assert check_padding(bufs[i], m), (i, sh[i])
