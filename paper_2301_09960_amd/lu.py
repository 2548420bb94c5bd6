"""Timing of the blocked DD / TD LU with slice-product Schur updates (Section
4.6): ``mpgemm_{dd,td}_lu`` and ``mpgemm_{dd,td}_lu_solve`` for n and a range of
block widths K, in either slice form of the Schur GEMM.  One JSON line per case:

    python -m paper_2301_09960_amd.lu [--n 2048] [--K 64,128,256,512] [--modes float,int8] [--formats dd,td]

The matrix is diagonally dominant (uniform [0, 1) entries with a lo part, n on
the diagonal), since the factorization does not pivot.  The accuracy of the
same path is checked exactly, at smaller n, by the GPU tests.

Section 4.6's own experiment (its test system a_ij = ru, b = [1, 1/2, ...,
1/n], no pivoting): time and the max relative error of x over n and K,

    python -m paper_2301_09960_amd.lu --paper [--sizes 512,1024,1536,2048,2560] [--K 32,128,512]

The reference solution is the TD solution refined once with a residual
b - A x formed by the QD product (A and x read as QD, exact), solved with the
TD factors: the refinement removes the TD solution's error to second order,
so it serves as the reference for both DD and TD.
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


def paper_system(n: int, c: int, seed: int = 46):
    """(A, b): a_ij uniform on [0, 1) with lower components below half an ulp
    (c components), b = [1, 1/2, ..., 1/n] rounded to c components (each
    component the binary64 rounding of what the previous ones leave)."""
    from fractions import Fraction
    rng = np.random.default_rng(seed)
    hi = rng.random((n, n))
    planes, prev = [hi.T], hi
    for _ in range(1, c):
        nxt = (rng.random((n, n)) - 0.5) * np.spacing(prev)
        planes.append(nxt.T)
        prev = np.abs(nxt) + np.finfo(float).tiny
    b = np.zeros((c, n))
    for i in range(1, n + 1):
        rest = Fraction(1, i)
        for r in range(c):
            b[r, i - 1] = float(rest)
            rest -= Fraction(b[r, i - 1])
    return np.ascontiguousarray(np.stack(planes)), b


def reference_solution(n: int, seed: int = 46):
    """TD solution of the system refined once with a QD residual (see module
    doc); returned as six binary64 components per entry, (6, n): the TD
    solution's three and the correction's three."""
    import torch

    from . import gemm, lu, lu_solve
    A3, b3 = paper_system(n, 3, seed)
    dA = torch.from_numpy(A3.copy()).cuda()
    lu("td", dA, 128)
    x = lu_solve("td", dA, torch.from_numpy(b3).cuda())
    # r = b - A x = [A b] [-x; 1] as one QD product (A, b, x padded to four
    # components, exact): within 2^-200 (|A||x| + |b|) of the true residual
    M = torch.zeros((4, n + 1, n), dtype=torch.float64, device="cuda")
    M[:3, :n] = torch.from_numpy(A3).cuda()
    M[:3, n] = torch.from_numpy(b3).cuda()
    v = torch.zeros((4, 1, n + 1), dtype=torch.float64, device="cuda")
    v[:3, 0, :n] = -x
    v[0, 0, n] = 1.0
    r = gemm("qd", M, v)[:3, 0, :].contiguous()
    d = lu_solve("td", dA, r)
    torch.cuda.synchronize()
    return np.concatenate([x.cpu().numpy(), d.cpu().numpy()])


def relative_error(x, ref) -> float:
    """max_i |x_i - ref_i| / |ref_i| over expansions (components along axis 0),
    in exact rational arithmetic."""
    from fractions import Fraction
    worst = Fraction(0)
    for i in range(x.shape[1]):
        xv = sum((Fraction(float(t)) for t in x[:, i]), Fraction(0))
        rv = sum((Fraction(float(t)) for t in ref[:, i]), Fraction(0))
        if rv != 0:
            worst = max(worst, abs(xv - rv) / abs(rv))
    return float(worst)


def measure_paper(n: int, K: int, fmt: str, ref, mode: str = "float", reps: int = 2):
    import torch

    from . import lu, lu_solve
    c = 2 if fmt == "dd" else 3
    A0, b = paper_system(n, c)
    A0d = torch.from_numpy(A0).cuda()
    bd = torch.from_numpy(b).cuda()
    A = A0d.clone()
    lu(fmt, A, K, mode=mode)
    x = lu_solve(fmt, A, bd)
    torch.cuda.synchronize()
    lu_ms, sv_ms = [], []
    for _ in range(reps):
        A.copy_(A0d)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        lu(fmt, A, K, mode=mode)
        e1.record()
        x = lu_solve(fmt, A, bd)
        e2.record()
        torch.cuda.synchronize()
        lu_ms.append(e0.elapsed_time(e1))
        sv_ms.append(e1.elapsed_time(e2))
    return {"fmt": fmt, "n": n, "K": K, "mode": mode, "lu_ms": round(float(np.median(lu_ms)), 3),
            "solve_ms": round(float(np.median(sv_ms)), 3),
            "max_relative_error": relative_error(x.cpu().numpy(), ref)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--paper", action="store_true", help="Section 4.6's test system: time and relative error")
    ap.add_argument("--sizes", default="512,1024,1536,2048,2560")
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--K", default="64,128,256,512")
    ap.add_argument("--modes", default="float,int8")
    ap.add_argument("--formats", default="dd,td")
    a = ap.parse_args()
    if a.paper:
        Ks = [int(x) for x in a.K.split(",")]
        for n in [int(x) for x in a.sizes.split(",")]:
            ref = reference_solution(n)
            for fmt in a.formats.split(","):
                if fmt == "td" and n > 2048:
                    continue  # the paper's TD runs stop at 2048
                for K in Ks:
                    print(json.dumps(measure_paper(n, K, fmt, ref)), flush=True)
        return
    for fmt in a.formats.split(","):
        for mode in a.modes.split(","):
            for K in [int(x) for x in a.K.split(",")]:
                print(json.dumps(measure(a.n, K, mode, fmt=fmt)), flush=True)


if __name__ == "__main__":
    main()
