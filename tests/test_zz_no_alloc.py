"""The allocation-free DD entry point (mpgemm_dd_noalloc), through the C-ABI:
the same C as mpgemm_dd bit for bit, in both slice forms, on two calls in a
row (the second with a smaller input, so stale scratch contents from the
first must not leak into it), with padded leading dimensions; shapes whose
workspace exceeds the fixed scratch are refused without touching C."""
import ctypes

import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu

MPGEMM_ERR_TOO_LARGE = 5
SCRATCH = 64 << 20  # MPGEMM_NOALLOC_SCRATCH_BYTES


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_09960_amd as mp
    L = mp.lib()
    L.mpgemm_dd_noalloc.restype = ctypes.c_int
    L.mpgemm_dd_noalloc.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p, ctypes.c_int] * 3 + [ctypes.c_void_p]
    assert mp.check_device() == 0
    return mp


def say(*a):
    print(*a, flush=True)


def call_noalloc(mp, A, B, C, m, n, k, lda, ldb, ldc):
    import torch
    P = ctypes.c_void_p
    return mp.lib().mpgemm_dd_noalloc(m, n, k, P(A.data_ptr()), lda, P(B.data_ptr()), ldb, P(C.data_ptr()), ldc,
                                      P(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("mode", ["float", "int8"])
def test_noalloc_equals_mpgemm_dd(mp, orc, mode):
    import torch
    old = mp.get_mode("dd")
    mp.set_mode("dd", mode)
    try:
        for call, (m, n, k, pad) in enumerate([(500, 470, 520, 0), (130, 97, 333, 7)]):
            need = mp.workspace_bytes("dd", mode, m, n, k)
            assert need <= SCRATCH, need
            say(f"noalloc dd {mode} call {call}: m={m} n={n} k={k} pad={pad} workspace {need} bytes")
            A, B = W.gen_pair("dd", m, n, k, E=16, seed=900 + call)
            dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
            want = mp.gemm("dd", dA, dB)
            torch.cuda.synchronize()
            Ab = torch.full((2, k, m + pad), float("nan"), dtype=torch.float64, device="cuda")
            Bb = torch.full((2, n, k + pad), float("nan"), dtype=torch.float64, device="cuda")
            Ab[:, :, :m] = dA
            Bb[:, :, :k] = dB
            Cb = torch.full((2, n, m + pad), -3.0, dtype=torch.float64, device="cuda")
            st = call_noalloc(mp, Ab, Bb, Cb, m, n, k, m + pad, k + pad, m + pad)
            assert st == 0, st
            torch.cuda.synchronize()
            assert torch.equal(Cb[:, :, :m], want), "differs from mpgemm_dd"
            assert bool(torch.all(Cb[:, :, m:] == -3.0)), "C's padding was written"
            rows = [0, m // 2, m - 1]
            diff, absab, _ = orc.exact_check(A, B, Cb[:, :, :m].cpu().numpy(), rows=rows)
            ok, worst = orc.bound_report(diff, absab, 100)
            say(f"  worst log2 ratio {worst:.1f} (bound -100)")
            assert ok
    finally:
        mp.set_mode("dd", old)


def test_noalloc_refuses_beyond_scratch(mp):
    import torch
    m = n = k = 1024
    assert mp.workspace_bytes("dd", "float", m, n, k) > SCRATCH
    A = torch.zeros((2, k, m), dtype=torch.float64, device="cuda")
    B = torch.zeros((2, n, k), dtype=torch.float64, device="cuda")
    C = torch.full((2, n, m), 5.0, dtype=torch.float64, device="cuda")
    st = call_noalloc(mp, A, B, C, m, n, k, m, k, m)
    torch.cuda.synchronize()
    assert st == MPGEMM_ERR_TOO_LARGE
    assert bool(torch.all(C == 5.0))
    # argument errors as mpgemm_dd
    assert call_noalloc(mp, A, B, C, -1, n, k, m, k, m) == -1
    assert call_noalloc(mp, A, B, C, m, n, k, m - 1, k, m) == -5
