"""Autotuner: wavefront layouts of the slice-product kernel, and slice counts.

Layouts: times every layout (1: 4 wavefronts of 32 x 32, 2: 8 of 32 x 16,
3: 16 of 16 x 16 per 64 x 64 tile) for each format on square products of the
given sizes, with the library's own stage timer (HIP events around the kernel
on its stream), and writes the fastest layout per format as lines
"<fmt> <layout>".

Slice counts (--slices): for each format, slice form and inner dimension k,
the smallest D whose products stay below 2^-(t + guard) (|A||B|) on seeded
inputs (e ~ U{0..16}), the error measured against the same product with a few
more slices (about 20 bits more accurate) and |A||B| from the leading
components; written as lines "slices <fmt> <mode> <kmax> <D>", each D the
largest over its k and every smaller tuned k (so an entry covers the k range
below it).  Both kinds of line form the file the library reads from
MPGEMM_TUNE_FILE or mpgemm_load_tune_file.

    python -m paper_2301_09960_amd.tune --formats dd,td,qd,ts --n 4096 --out tune.txt
    python -m paper_2301_09960_amd.tune --slices --out slices.txt
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import (COMPONENTS, gemm, load_tune_file, num_slices, profile_enable, profile_read, set_int8_tile,
               set_tile_layout)

LAYOUTS = (1, 2, 3)
T_BITS = {"dd": 100, "td": 150, "qd": 200, "ts": 66}
MAX_D = {"float": 16, "int8": 40}
SLICE_KS = (64, 128, 256, 512, 1024, 2048, 4096)


def slice_error_log2(fmt, mode, dA, dB, D, Cref, absab):
    """log2 of max |C(D) - Cref| / (|A||B|) over the elements (component
    differences summed from the smallest up, in binary64)."""
    import torch
    C = gemm(fmt, dA, dB, mode=mode, slices=D).double()
    err = torch.zeros_like(absab)
    for r in range(C.shape[0] - 1, -1, -1):
        err += C[r] - Cref[r]
    ratio = (err.abs() / absab.clamp_min(1e-300)).max().item()
    return float(np.log2(ratio)) if ratio > 0 else -np.inf


def tune_slices(fmt, mode, ks=SLICE_KS, size=128, seeds=(1, 2, 3), E=16, guard=4):
    """{k: smallest D meeting 2^-(T + guard) on every seed}."""
    import torch

    from workload import gen_pair
    out = {}
    for k in ks:
        Df = num_slices(fmt, mode, k)
        Dref = min(Df + (2 if mode == "float" else 4), MAX_D[mode])
        need = 1
        for seed in seeds:
            A, B = gen_pair(fmt, size, size, k, E=E, seed=seed)
            dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
            Cref = gemm(fmt, dA, dB, mode=mode, slices=Dref).double()
            absab = dB[0].double().abs() @ dA[0].double().abs()  # (n, m): sum_p |b_pj| |a_ip|
            D = need
            while D < Dref and slice_error_log2(fmt, mode, dA, dB, D, Cref, absab) > -(T_BITS[fmt] + guard):
                D += 1
            need = max(need, D)
        out[k] = need
    return out


def slice_table(cases, ks=SLICE_KS, **kw):
    """Lines "slices <fmt> <mode> <kmax> <D>", D non-decreasing in k per case."""
    load_tune_file(None)  # tune against the compiled-in formula
    lines = []
    for fmt, mode in cases:
        found = tune_slices(fmt, mode, ks, **kw)
        best = 0
        for k in ks:
            best = max(best, found[k])
            lines.append(f"slices {fmt} {mode} {k} {best}")
            print(json.dumps({"fmt": fmt, "mode": mode, "k": k, "D_tuned": found[k], "D_entry": best,
                              "D_formula": num_slices(fmt, mode, k)}), flush=True)
    return lines


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


def time_int8_tiles(fmt: str, n: int, reps: int = 3, E: int = 16, cfgs=(1, 2, 3, 4)):
    """INT8-form tile configurations (GEMM + combine milliseconds)."""
    import torch

    from workload import gen_pair
    A, B = gen_pair(fmt, n, n, n, E=E, seed=77)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = torch.empty((COMPONENTS[fmt], n, n), dtype=dA.dtype, device="cuda")
    out = {}
    for cfg in cfgs:
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
    ap.add_argument("--slices", action="store_true", help="tune slice counts instead")
    ap.add_argument("--cfgs", default="1,2,3,4", help="INT8 tile configurations to time (with --int8)")
    args = ap.parse_args()
    if args.slices:
        cases = [(f, "float") for f in ("dd", "td", "qd", "ts")] + [(f, "int8") for f in ("dd", "td", "qd")]
        lines = slice_table(cases)
        if args.out:
            with open(args.out, "w") as f:
                f.write("\n".join(lines) + "\n")
        return
    sizes = [int(x) for x in args.n.split(",")]
    if args.int8:
        for fmt in args.formats.split(","):
            for n in sizes:
                print(json.dumps({"fmt": fmt, "n": n, "int8_gemm_and_combine_ms": time_int8_tiles(
                    fmt, n, args.reps, cfgs=[int(c) for c in args.cfgs.split(",")])}),
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
