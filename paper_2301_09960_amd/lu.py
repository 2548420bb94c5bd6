"""Timing of the blocked DD LU with slice-product Schur updates (Section 4.6):
``mpgemm_dd_lu`` and ``mpgemm_dd_lu_solve`` for n and a range of block widths
K, in either slice form of the Schur GEMM.  One JSON line per case:

    python -m paper_2301_09960_amd.lu [--n 2048] [--K 64,128,256,512] [--modes float,int8]

The matrix is diagonally dominant (uniform [0, 1) entries with a lo part, n on
the diagonal), since the factorization does not pivot.  The accuracy of the
same path is checked exactly, at smaller n, by the GPU tests.
"""
from __future__ import annotations

import argparse
import json

import numpy as np


def dominant(n: int, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    hi = rng.random((n, n)) + n * np.eye(n)
    lo = (rng.random((n, n)) - 0.5) * np.spacing(hi)
    return np.ascontiguousarray(np.stack([hi.T, lo.T]))


def measure(n: int, K: int, mode: str, reps: int = 3):
    import torch

    from . import dd_lu, dd_lu_solve
    A0 = torch.from_numpy(dominant(n)).cuda()
    b = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    b[0] = 1.0 / torch.arange(1, n + 1, dtype=torch.float64, device="cuda")
    A = A0.clone()
    dd_lu(A, K, mode=mode)  # warm: plans, workspaces
    dd_lu_solve(A, b)
    torch.cuda.synchronize()
    lu_ms, sv_ms = [], []
    for _ in range(reps):
        A.copy_(A0)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        dd_lu(A, K, mode=mode)
        e1.record()
        dd_lu_solve(A, b)
        e2.record()
        torch.cuda.synchronize()
        lu_ms.append(e0.elapsed_time(e1))
        sv_ms.append(e1.elapsed_time(e2))
    lu = float(np.median(lu_ms))
    return {"n": n, "K": K, "mode": mode, "lu_ms": round(lu, 3), "solve_ms": round(float(np.median(sv_ms)), 3),
            "effective_gflops": round(2.0 * n ** 3 / 3.0 / (lu * 1e-3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--K", default="64,128,256,512")
    ap.add_argument("--modes", default="float,int8")
    a = ap.parse_args()
    for mode in a.modes.split(","):
        for K in [int(x) for x in a.K.split(",")]:
            print(json.dumps(measure(a.n, K, mode)), flush=True)


if __name__ == "__main__":
    main()
