"""Autotuner for the slice-product kernel's wavefront layout.

Times every layout (1: 4 wavefronts of 32 x 32, 2: 8 of 32 x 16, 3: 16 of
16 x 16 per 64 x 64 tile) for each format on square products of the given
sizes, with the library's own stage timer (HIP events around the kernel on
its stream), and writes the fastest layout per format as lines
"<fmt> <layout>" -- the file format the library reads from MPGEMM_TUNE_FILE.

    python -m paper_2301_09960_amd.tune --formats dd,td,qd,ts --n 4096 --out tune.txt
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import COMPONENTS, gemm, profile_enable, profile_read, set_int8_tile, set_tile_layout

LAYOUTS = (1, 2, 3)


def time_layouts(fmt: str, n: int, reps: int = 3, E: int = 16):
    import torch

    from workload import gen_pair
    A, B = gen_pair(fmt, n, n, n, E=E, seed=77)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = torch.empty((COMPONENTS[fmt], n, n), dtype=dA.dtype, device="cuda")
    out = {}
    for lay in LAYOUTS:
        set_tile_layout(fmt, lay)
        gemm(fmt, dA, dB, C)  # warm
        torch.cuda.synchronize()
        profile_enable(True)
        for _ in range(reps):
            gemm(fmt, dA, dB, C)
        torch.cuda.synchronize()
        profile_enable(False)
        _, g = profile_read()
        out[lay] = float(np.median(g))
    set_tile_layout(fmt, 0)
    return out


def time_int8_tiles(fmt: str, n: int, reps: int = 3, E: int = 16):
    """INT8-form tile configurations 1..4 (GEMM + combine milliseconds)."""
    import torch

    from workload import gen_pair
    A, B = gen_pair(fmt, n, n, n, E=E, seed=77)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = torch.empty((COMPONENTS[fmt], n, n), dtype=dA.dtype, device="cuda")
    out = {}
    for cfg in (1, 2, 3, 4):
        set_int8_tile(cfg)
        gemm(fmt, dA, dB, C, mode="int8")
        torch.cuda.synchronize()
        profile_enable(True)
        for _ in range(reps):
            gemm(fmt, dA, dB, C, mode="int8")
        torch.cuda.synchronize()
        profile_enable(False)
        _, g = profile_read()
        out[cfg] = float(np.median(g))
    set_int8_tile(0)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--formats", default="dd,td,qd,ts")
    ap.add_argument("--n", default="4096", help="comma-separated sizes; the largest decides")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default="")
    ap.add_argument("--int8", action="store_true", help="time the INT8-form tile configurations instead")
    args = ap.parse_args()
    sizes = [int(x) for x in args.n.split(",")]
    if args.int8:
        for fmt in args.formats.split(","):
            for n in sizes:
                print(json.dumps({"fmt": fmt, "n": n, "int8_gemm_and_combine_ms": time_int8_tiles(fmt, n, args.reps)}),
                      flush=True)
        return
    table = {}
    best = {}
    for fmt in args.formats.split(","):
        table[fmt] = {}
        for n in sizes:
            t = time_layouts(fmt, n, args.reps)
            table[fmt][n] = t
            print(json.dumps({"fmt": fmt, "n": n, "gemm_kernel_ms": t}), flush=True)
        big = max(sizes)
        best[fmt] = min(table[fmt][big], key=table[fmt][big].get)
    if args.out:
        with open(args.out, "w") as f:
            for fmt, lay in best.items():
                f.write(f"{fmt} {lay}\n")
    print(json.dumps({"best": best}), flush=True)


if __name__ == "__main__":
    main()
