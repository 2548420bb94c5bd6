"""Timing of the blocked DD / TD LU with slice-product Schur updates (Section
4.6): ``mpgemm_{dd,td}_lu`` and ``mpgemm_{dd,td}_lu_solve`` for n and a range of
block widths K, in either slice form of the Schur GEMM.  One JSON line per case:

    python -m paper_2301_09960_amd.lu [--n 2048] [--K 64,128,256,512] [--modes float,int8] [--formats dd,td]

The matrix is diagonally dominant (uniform [0, 1) entries with a lo part, n on
the diagonal), since the factorization does not pivot.  The accuracy of the
same path is checked exactly, at smaller n, by the GPU tests.
"""
from __future__ import annotations

import argparse
import json

import numpy as np


def dominant(n: int, seed: int = 1, c: int = 2) -> np.ndarray:
    """(c, n, n): uniform [0, 1) entries with lower components, n on the diagonal."""
    rng = np.random.default_rng(seed)
    hi = rng.random((n, n)) + n * np.eye(n)
    planes, prev = [hi.T], hi
    for _ in range(1, c):
        nxt = (rng.random((n, n)) - 0.5) * np.spacing(prev)
        planes.append(nxt.T)
        prev = np.abs(nxt) + np.finfo(float).tiny
    return np.ascontiguousarray(np.stack(planes))


def measure(n: int, K: int, mode: str, reps: int = 3, fmt: str = "dd"):
    import torch

    from . import lu, lu_solve
    c = 2 if fmt == "dd" else 3
    A0 = torch.from_numpy(dominant(n, c=c)).cuda()
    b = torch.zeros((c, n), dtype=torch.float64, device="cuda")
    b[0] = 1.0 / torch.arange(1, n + 1, dtype=torch.float64, device="cuda")
    A = A0.clone()
    lu(fmt, A, K, mode=mode)  # warm: plans, workspaces
    lu_solve(fmt, A, b)
    torch.cuda.synchronize()
    lu_ms, sv_ms = [], []
    for _ in range(reps):
        A.copy_(A0)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        lu(fmt, A, K, mode=mode)
        e1.record()
        lu_solve(fmt, A, b)
        e2.record()
        torch.cuda.synchronize()
        lu_ms.append(e0.elapsed_time(e1))
        sv_ms.append(e1.elapsed_time(e2))
    lu_t = float(np.median(lu_ms))
    return {"fmt": fmt, "n": n, "K": K, "mode": mode, "lu_ms": round(lu_t, 3), "solve_ms": round(float(np.median(sv_ms)), 3),
            "effective_gflops": round(2.0 * n ** 3 / 3.0 / (lu_t * 1e-3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--K", default="64,128,256,512")
    ap.add_argument("--modes", default="float,int8")
    ap.add_argument("--formats", default="dd,td")
    a = ap.parse_args()
    for fmt in a.formats.split(","):
        for mode in a.modes.split(","):
            for K in [int(x) for x in a.K.split(",")]:
                print(json.dumps(measure(a.n, K, mode, fmt=fmt)), flush=True)


if __name__ == "__main__":
    main()
