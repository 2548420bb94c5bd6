"""Throughput over the grid of square products: n in {1024, 2048, 4096},
DD / TD / QD with e ~ U{0..0} and e ~ U{0..16} (binary64 slices), TS at
n = 4096 (binary32 slices), and the INT8 form of the DD / TD / QD products at
n = 4096.

Stage times come from the library's own HIP events on the launch stream
(split kernels, then the slice-product kernel or the INT8 GEMM plus combine).
One JSON line per case:

    python -m paper_2301_09960_amd.sweep [--reps 3] [--sizes 1024,2048,4096]
    python -m paper_2301_09960_amd.sweep --nd --sizes 1024,2048   (5 .. 14 components)
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import COMPONENTS, gemm, gemm_nd, last_num_slices, nd_num_slices, profile_enable, profile_read

PEAK = {"float64": 78.6, "float32": 157.3, "int8": 5000.0}  # dense matrix-core TFLOP/s (TOP/s for int8)


def measure(fmt: str, n: int, E: int, mode: str, reps: int):
    import torch

    from workload import gen_pair
    A, B = gen_pair(fmt, n, n, n, E=E, seed=n + E)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    del A, B
    C = torch.empty((COMPONENTS[fmt], n, n), dtype=dA.dtype, device="cuda")
    gemm(fmt, dA, dB, C, mode=mode)  # warm: plan, workspace
    torch.cuda.synchronize()
    profile_enable(True)
    for _ in range(reps):
        gemm(fmt, dA, dB, C, mode=mode)
    torch.cuda.synchronize()
    profile_enable(False)
    sp, gm = profile_read()
    D = last_num_slices()
    split_ms, gemm_ms = float(np.median(sp)), float(np.median(gm))
    ops = D * (D + 1) / 2 * 2.0 * n ** 3
    kind = "int8" if mode == "int8" else ("float32" if fmt == "ts" else "float64")
    rate = ops / (gemm_ms * 1e-3) / 1e12
    return {
        "fmt": fmt, "n": n, "E": E, "mode": mode, "D": D,
        "split_ms": round(split_ms, 3), "gemm_ms": round(gemm_ms, 3),
        "effective_gflops": round(2.0 * n ** 3 / ((split_ms + gemm_ms) * 1e-3) / 1e9, 1),
        "slice_rate": round(rate, 2), "slice_rate_unit": "TOP/s" if mode == "int8" else "TFLOP/s",
        "peak_frac": round(rate / PEAK[kind], 4),
    }


def measure_nd(c: int, n: int, reps: int, E: int = 16):
    """Longer expansions (c binary64 components), INT8 form."""
    import torch

    from workload import gen_pair
    A, B = gen_pair(f"{c}d" if c > 4 else {2: "dd", 3: "td", 4: "qd"}[c], n, n, n, E=E, seed=n + c)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    del A, B
    C = torch.empty((c, n, n), dtype=torch.float64, device="cuda")
    gemm_nd(dA, dB, C)
    torch.cuda.synchronize()
    profile_enable(True)
    for _ in range(reps):
        gemm_nd(dA, dB, C)
    torch.cuda.synchronize()
    profile_enable(False)
    sp, gm = profile_read()
    D = nd_num_slices(c, n)
    split_ms, gemm_ms = float(np.median(sp)), float(np.median(gm))
    ops = D * (D + 1) / 2 * 2.0 * n ** 3
    return {
        "components": c, "bits": 53 * c, "n": n, "E": E, "mode": "int8", "D": D,
        "split_ms": round(split_ms, 3), "gemm_ms": round(gemm_ms, 3),
        "effective_gflops": round(2.0 * n ** 3 / ((split_ms + gemm_ms) * 1e-3) / 1e9, 1),
        "slice_rate": round(ops / (gemm_ms * 1e-3) / 1e12, 2), "slice_rate_unit": "TOP/s",
        "peak_frac": round(ops / (gemm_ms * 1e-3) / 1e12 / PEAK["int8"], 4),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--sizes", default="1024,2048,4096")
    ap.add_argument("--nd", action="store_true", help="time the longer expansions (5 to 14 components) instead")
    a = ap.parse_args()
    if a.nd:
        for n in [int(x) for x in a.sizes.split(",")]:
            for c in (4, 5, 6, 8, 10, 12, 14):
                print(json.dumps(measure_nd(c, n, a.reps)), flush=True)
        return
    sizes = [int(x) for x in a.sizes.split(",")]
    cases = [(f, n, E, "float") for n in sizes for f in ("dd", "td", "qd") for E in (0, 16)]
    big = max(sizes)
    cases += [("ts", big, E, "float") for E in (0, 16)]
    cases += [(f, big, E, "int8") for f in ("dd", "td", "qd") for E in (0, 16)]
    for fmt, n, E, mode in cases:
        print(json.dumps(measure(fmt, n, E, mode, a.reps)), flush=True)


if __name__ == "__main__":
    main()
