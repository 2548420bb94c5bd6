"""Benchmark: Ozaki-scheme DD and QD GEMM at n = 4096 on one MI355X.

One step = one DD and one QD product C = A B at m = n = k = 4096 (synthetic
inputs, exponent spread e ~ U{0..16}, binary64 slices on the FP64 matrix
cores), each a full pass of the path: split of A and B, every slice product
of the triangle, error-free accumulation into C.  Inputs are resident in HBM
before the timed region.  ``value`` is the whole job's effective 2 n^3 / s.

Extra objects on the JSON line:
  roofline     -- the dominant kernel (the fused slice-product GEMM of the QD
                  call) against the FP64 matrix peak: algorithmic slice-GEMM
                  flops per launch, D (D + 1) / 2 x 2 n^3, over its average
                  launch time measured with HIP events on its stream.
  cpu_baseline -- the CPU oracle's Ozaki product timed on a bounded sample.
  stages       -- per format: split and fused-GEMM milliseconds per call.
  int8         -- the same products with INT8 digit slices on the INT8 matrix
                  cores (precision form), timed the same way; speedup over
                  the binary64-slice form at the same error bound.
  data_chosen_pairs -- the same products with the slice products chosen
                  from the data (per-tile pair sets, certified by
                  construction): call time, mean pairs per tile, certificate.
  batched      -- 512 independent DD (and QD) products with m, n, k each
                  log-uniform in [64, 1024], e ~ U{0..8}, as one graph launch:
                  sum of 2mnk over the batch / launch time; and 256 DD + 256
                  QD products as two launches on one stream ("mixed").
  serving      -- Poisson arrivals of DD/TD/QD requests (m, n, k log-uniform in
                  [64, 2048]) under a 64 GB HBM budget at 0.75 of the measured
                  capacity: p50/p99 latency and throughput.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DD/QD GEMM 2n³/s at n=4096, %MFMA peak, INT8 vs FP64 slices; served p50/p99"
FP64_MFMA_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3
INT8_MFMA_PEAK_TOPS = 5000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gemm_plain_qd_n4096.json")
GEMM_SOURCE = os.path.join(ROOT, "paper_2301_09960_amd", "csrc", "gemm_fp.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(epilog=MODES_HELP, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--E", type=int, default=16)
    ap.add_argument("--formats", default="dd,qd")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-int8", action="store_true", help="skip the INT8-slice form")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-certify", action="store_true", help="skip the certified calls")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--no-data", action="store_true", help="skip the data-chosen slice products")
    ap.add_argument("--serve-requests", type=int, default=2000, help="served requests timed (after a tenth as many)")
    ap.add_argument("--cpu-rows", type=int, default=0, help="rows of C in the CPU sample (0: auto)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 1 GiB (for scaling HBM counters)")
    # other measurement modes (each prints its own lines and exits)
    ap.add_argument("--sweep", choices=("grid", "nd", "simple"), default="",
                    help="grid: the square grid of products; nd: longer expansions; "
                         "simple: the simple in-format products against the Ozaki products")
    ap.add_argument("--sizes", default="", help="sweep sizes, comma separated")
    ap.add_argument("--reps", type=int, default=3, help="sweep repetitions per case")
    ap.add_argument("--traffic", action="store_true", help="summarize two rocprofv3 --pmc runs (no GPU)")
    ap.add_argument("--fetch", help="rocprofv3 -d folder of the FETCH_SIZE run")
    ap.add_argument("--write", help="rocprofv3 -d folder of the WRITE_SIZE run")
    ap.add_argument("--kernel", help="substring of the kernel's name")
    ap.add_argument("--label", default="", help="name written into the summary (default: --kernel)")
    ap.add_argument("--algorithmic-bytes", type=float)
    ap.add_argument("--source", help="the kernel's source file (hashed)")
    ap.add_argument("--command", action="append", default=[], help="command of a run, recorded as given")
    ap.add_argument("--out", default="")
    return ap.parse_args()


MODES_HELP = """measurement modes besides the benchmark line:
  python bench.py --sweep grid [--sizes 1024,2048,4096] [--reps 3]
      square products n x {DD, TD, QD} x e ~ U{0..0}, U{0..16} (binary64
      slices), TS at the largest n, the INT8 form at the largest n: one JSON
      line per case with split / slice-product milliseconds from the library's
      own HIP events on the launch stream
  python bench.py --sweep nd [--sizes 1024,2048]
      longer binary64 expansions (4 .. 14 components), INT8 form
  python bench.py --sweep simple [--sizes 512,1024,...,4096]
      the simple in-format products (DD, TS, D+S; with and without LDS
      staging; Section 4.4) beside the Ozaki products of the same inputs
  python bench.py --traffic --fetch DIR1 --write DIR2 --kernel NAME
      --algorithmic-bytes B --source FILE [--out traffic.json]
      HBM bytes per launch of one kernel from two rocprofv3 --pmc runs
      (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by what the
      counter reads for the plain 1 GiB copies of --copy-calibration
"""


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(kernel_key):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256_16") != source_hash(GEMM_SOURCE) or t.get("kernel") != kernel_key:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(n, E, rows_req):
    """The oracle's Ozaki product (split, exact slice products, exact
    accumulation; the CPU reference of this path) on rows 0..R-1 of the DD
    n = 4096 product, scaled to effective 2 n^3 / s."""
    import oracle
    import workload as W
    A, B = W.gen_pair("dd", n, n, n, E=E, seed=2023)
    D = 6
    cores = oracle.threads()
    rows = rows_req or 2 * cores  # about 10 s of CPU work
    t0 = time.perf_counter()
    oracle.ozaki_gemm(A, B, D, rows=list(range(rows)))
    dt = time.perf_counter() - t0
    flops = 2.0 * rows * n * n
    # the same on one core, on 2 rows
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.ozaki_gemm(A, B, D, rows=[0, 1])
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    return {
        "value": flops / dt / 1e9,
        "unit": "GFLOP/s (effective 2mnk/s)",
        "cores": cores,
        "kind": "oracle",
        "sample": f"DD n={n} E~U{{0..{E}}} D={D}: full split of B, split of {rows} rows of A, exact slice products "
                  f"and exact accumulation for {rows} x {n} entries of C ({dt:.1f} s)",
        "one_core": {"value": 2.0 * 2 * n * n / dt1 / 1e9, "cores": 1,
                     "sample": f"the same for 2 rows of C on one thread ({dt1:.1f} s)"},
    }


def run_batched(mp, torch, pool, fmt, count=512, seed=31, mode="float"):
    """One graph launch of `count` products with sizes log-uniform in [64, 1024]."""
    from paper_2301_09960_amd import serve
    As, Bs, m, n, k = serve.batch_operands(pool, fmt, count, seed)
    Cs = mp.gemm_batched(fmt, As, Bs, mode=mode)  # captures the graph
    torch.cuda.synchronize()
    reps = 3
    mp.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        mp.gemm_batched(fmt, As, Bs, Cs, mode=mode)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mp.profile_enable(False)
    _, gms = mp.profile_read()
    flops = float(np.sum(2.0 * m * n * k))
    gpu_ms = float(np.mean(gms))
    Ds = np.array([mp.num_slices(fmt, mode, int(kk)) for kk in k], dtype=np.float64)
    slice_flops = float(np.sum(Ds * (Ds + 1) / 2 * 2.0 * m * n * k))
    peak = INT8_MFMA_PEAK_TOPS if mode == "int8" else FP64_MFMA_PEAK_TFLOPS
    return {
        "products": count,
        "mode": mode,
        "sum_2mnk": flops,
        "launch_ms": round(gpu_ms, 3),
        "effective_gflops": round(flops / (gpu_ms * 1e-3) / 1e9, 1),
        "slice_gemm_tflops": round(slice_flops / (gpu_ms * 1e-3) / 1e12, 2),
        "mfma_frac": round(slice_flops / (gpu_ms * 1e-3) / 1e12 / peak, 4),
        "wall_ms_per_batch": round((t1 - t0) * 1e3 / reps, 3),
        "max_slices": mp.last_num_slices(),
    }


# ---------------------------------------------------------------------------
# sweeps (--sweep)
# ---------------------------------------------------------------------------

SWEEP_PEAK = {"float64": FP64_MFMA_PEAK_TFLOPS, "float32": FP32_MFMA_PEAK_TFLOPS, "int8": INT8_MFMA_PEAK_TOPS}


def _timed_calls(torch, mp, call, reps):
    """Median split and GEMM milliseconds of `reps` calls (library events)."""
    call()
    torch.cuda.synchronize()
    mp.profile_enable(True)
    for _ in range(reps):
        call()
    torch.cuda.synchronize()
    mp.profile_enable(False)
    sp, gm = mp.profile_read()
    return float(np.median(sp)), float(np.median(gm))


def _event_ms(torch, call, reps):
    """Median milliseconds of `reps` calls, HIP events on the current stream."""
    call()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        call()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return float(np.median(out))


def sweep_grid(torch, mp, sizes, reps):
    import workload as W
    cases = [(f, n, E, "float") for n in sizes for f in ("dd", "td", "qd") for E in (0, 16)]
    big = max(sizes)
    cases += [("ts", big, E, "float") for E in (0, 16)]
    cases += [(f, big, E, "int8") for f in ("dd", "td", "qd") for E in (0, 16)]
    for fmt, n, E, mode in cases:
        A, B = W.gen_pair(fmt, n, n, n, E=E, seed=n + E)
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        del A, B
        C = torch.empty((W.FORMATS[fmt][0], n, n), dtype=dA.dtype, device="cuda")
        split_ms, gemm_ms = _timed_calls(torch, mp, lambda: mp.gemm(fmt, dA, dB, C, mode=mode), reps)
        D = mp.last_num_slices()
        ops = D * (D + 1) / 2 * 2.0 * n ** 3
        kind = "int8" if mode == "int8" else ("float32" if fmt == "ts" else "float64")
        rate = ops / (gemm_ms * 1e-3) / 1e12
        print(json.dumps({
            "fmt": fmt, "n": n, "E": E, "mode": mode, "D": D,
            "split_ms": round(split_ms, 3), "gemm_ms": round(gemm_ms, 3),
            "effective_gflops": round(2.0 * n ** 3 / ((split_ms + gemm_ms) * 1e-3) / 1e9, 1),
            "slice_rate": round(rate, 2), "slice_rate_unit": "TOP/s" if mode == "int8" else "TFLOP/s",
            "peak_frac": round(rate / SWEEP_PEAK[kind], 4)}), flush=True)
        del dA, dB, C


def sweep_nd(torch, mp, sizes, reps, E=16):
    import workload as W
    for n in sizes:
        for c in (4, 5, 6, 8, 10, 12, 14):
            fmt = f"{c}d" if c > 4 else {2: "dd", 3: "td", 4: "qd"}[c]
            A, B = W.gen_pair(fmt, n, n, n, E=E, seed=n + c)
            dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
            del A, B
            C = torch.empty((c, n, n), dtype=torch.float64, device="cuda")
            split_ms, gemm_ms = _timed_calls(torch, mp, lambda: mp.gemm_nd(dA, dB, C), reps)
            D = mp.nd_num_slices(c, n)
            ops = D * (D + 1) / 2 * 2.0 * n ** 3
            print(json.dumps({
                "components": c, "bits": 53 * c, "n": n, "E": E, "mode": "int8", "D": D,
                "split_ms": round(split_ms, 3), "gemm_ms": round(gemm_ms, 3),
                "effective_gflops": round(2.0 * n ** 3 / ((split_ms + gemm_ms) * 1e-3) / 1e9, 1),
                "slice_rate": round(ops / (gemm_ms * 1e-3) / 1e12, 2), "slice_rate_unit": "TOP/s",
                "peak_frac": round(ops / (gemm_ms * 1e-3) / 1e12 / INT8_MFMA_PEAK_TOPS, 4)}), flush=True)
            del dA, dB, C


def sweep_simple(torch, mp, sizes, reps, E=16):
    """Section 4.4's GPU comparison at square n: the simple in-format products
    of DD, TS and D+S with and without LDS staging, and the Ozaki products of
    the same inputs (DD and TS with binary64 / binary32 slices, DD with INT8
    slices, D+S through the DD product), milliseconds per call (HIP events)."""
    import workload as W
    for n in sizes:
        rows = []
        for fmt in ("dd", "ts"):
            A, B = W.gen_pair(fmt, n, n, n, E=E, seed=n + E)
            dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
            del A, B
            C = torch.empty((W.FORMATS[fmt][0], n, n), dtype=dA.dtype, device="cuda")
            for staging in (1, 0):
                ms = _event_ms(torch, lambda: mp.simple(fmt, dA, dB, C, staging=staging), reps)
                rows.append({"fmt": fmt, "method": "simple", "lds": bool(staging), "ms": ms})
            ms = _event_ms(torch, lambda: mp.gemm(fmt, dA, dB, C, mode="float"), reps)
            rows.append({"fmt": fmt, "method": "ozaki", "mode": "float", "D": mp.last_num_slices(), "ms": ms})
            if fmt == "dd":
                ms = _event_ms(torch, lambda: mp.gemm(fmt, dA, dB, C, mode="int8"), reps)
                rows.append({"fmt": fmt, "method": "ozaki", "mode": "int8", "D": mp.last_num_slices(), "ms": ms})
            del dA, dB, C
        Ahi, Alo = W.gen_ds(n, n, E=E, seed=n + E, operand="A")
        Bhi, Blo = W.gen_ds(n, n, E=E, seed=n + E, operand="B")
        d = [torch.from_numpy(x).cuda() for x in (Ahi, Alo, Bhi, Blo)]
        Chi = torch.empty((1, n, n), dtype=torch.float64, device="cuda")
        Clo = torch.empty((1, n, n), dtype=torch.float32, device="cuda")
        for staging in (1, 0):
            ms = _event_ms(torch, lambda: mp.ds_simple(*d, Chi, Clo, staging=staging), reps)
            rows.append({"fmt": "ds", "method": "simple", "lds": bool(staging), "ms": ms})
        ms = _event_ms(torch, lambda: mp.ds_gemm(*d, Chi, Clo), reps)
        rows.append({"fmt": "ds", "method": "ozaki", "mode": "float", "D": mp.last_num_slices(), "ms": ms})
        del d, Chi, Clo
        for r in rows:
            r["n"] = n
            r["ms"] = round(r["ms"], 3)
            r["effective_gflops"] = round(2.0 * n ** 3 / (r["ms"] * 1e-3) / 1e9, 1)
            print(json.dumps(r), flush=True)


# ---------------------------------------------------------------------------
# HBM traffic from rocprofv3 counters (--traffic)
# ---------------------------------------------------------------------------

COPY_KERNEL = "copyBuffer"
GIB_KIB = 1 << 20


def counter_values(folder, counter):
    """{kernel name: [counter value per dispatch]} from every counter CSV below `folder`."""
    import csv
    import glob
    per = {}
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                key = (r["Kernel_Name"], r["Dispatch_Id"])
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (name, _), v in per.items():
        out.setdefault(name, []).append(v)
    return out


def traffic_summary(fetch_dir, write_dir, kernel, algorithmic_bytes, source, label, commands=()):
    """HBM bytes per launch of `kernel`: each counter's mean per dispatch,
    scaled by 1 GiB over what the counter reads for a plain 1 GiB copy."""
    def mean_of(values, sub):
        vals = [v for name, vs in values.items() if sub in name for v in vs]
        if not vals:
            raise SystemExit(f"no dispatch of a kernel matching {sub!r}")
        return sum(vals) / len(vals)

    def copy_reading(values):
        vals = [v for name, vs in values.items() if COPY_KERNEL in name for v in vs if v >= GIB_KIB / 4]
        if not vals:
            raise SystemExit("no 1 GiB copy dispatch found (run the command with --copy-calibration)")
        return sum(vals) / len(vals)

    fv, wv = counter_values(fetch_dir, "FETCH_SIZE"), counter_values(write_dir, "WRITE_SIZE")
    fk, wk = mean_of(fv, kernel), mean_of(wv, kernel)
    cf, cw = copy_reading(fv), copy_reading(wv)
    ff, wf = GIB_KIB / cf, GIB_KIB / cw
    fb, wb = fk * 1024 * ff, wk * 1024 * wf
    return {
        "kernel": label, "kernel_match": kernel, "source_sha256_16": source_hash(source),
        "fetch_kib_counter": fk, "write_kib_counter": wk,
        "copy_fetch_kib_per_gib": cf, "copy_write_kib_per_gib": cw,
        "fetch_factor": ff, "write_factor": wf, "fetch_bytes": fb, "write_bytes": wb,
        "bytes_per_launch": fb + wb, "algorithmic_bytes": algorithmic_bytes, "commands": list(commands),
    }


def run_mixed_batch(mp, torch, pool, mode="float", seed=31):
    """256 DD and 256 QD products (the first and second halves of the seeded
    shape sequence), as two graph launches on one stream: sum of 2mnk over
    the wall time of both."""
    from paper_2301_09960_amd import serve
    Ad, Bd, md, nd, kd = serve.batch_operands(pool, "dd", 256, seed)
    Aq, Bq, mq, nq, kq = serve.batch_operands(pool, "qd", 256, seed, first=256)
    Cd = mp.gemm_batched("dd", Ad, Bd, mode=mode)
    Cq = mp.gemm_batched("qd", Aq, Bq, mode=mode)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        mp.gemm_batched("dd", Ad, Bd, Cd, mode=mode)
        mp.gemm_batched("qd", Aq, Bq, Cq, mode=mode)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    flops = float(np.sum(2.0 * md * nd * kd) + np.sum(2.0 * mq * nq * kq))
    return {"products": "256 dd + 256 qd", "mode": mode, "sum_2mnk": flops, "wall_ms_per_batch": round(ms, 3),
            "effective_gflops": round(flops / (ms * 1e-3) / 1e9, 1)}


def main():
    args = parse()
    if args.traffic:
        if not (args.fetch and args.write and args.kernel and args.source and args.algorithmic_bytes):
            raise SystemExit("--traffic needs --fetch, --write, --kernel, --algorithmic-bytes and --source")
        summ = traffic_summary(args.fetch, args.write, args.kernel, args.algorithmic_bytes, args.source,
                               args.label or args.kernel, args.command)
        text = json.dumps(summ, indent=1)
        if args.out:
            with open(args.out, "w") as f:
                f.write(text + "\n")
        print(text)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2301_09960_amd as mp
    import workload as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    mp.lib()
    torch.cuda.set_device(0)
    if args.sweep:
        default = {"grid": "1024,2048,4096", "nd": "1024,2048", "simple": "512,1024,1536,2048,2560,3072,3584,4096"}
        sizes = [int(x) for x in (args.sizes or default[args.sweep]).split(",")]
        {"grid": sweep_grid, "nd": sweep_nd, "simple": sweep_simple}[args.sweep](torch, mp, sizes, args.reps)
        return
    n = args.n
    fmts = args.formats.split(",")
    log(f"generating inputs n={n} formats={fmts}")
    inputs = {}
    for f in fmts:
        A, B = W.gen_pair(f, n, n, n, E=args.E, seed=4096)
        inputs[f] = (torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
        del A, B
    outs = {f: torch.empty((W.FORMATS[f][0], n, n), dtype=inputs[f][0].dtype, device="cuda") for f in fmts}
    slices = {f: mp.num_slices(f, "float", n) for f in fmts}
    torch.cuda.synchronize()

    def timed(mode):
        for w in range(args.warmup):
            for f in fmts:
                mp.gemm(f, *inputs[f], outs[f], mode=mode)
            torch.cuda.synchronize()
            log(f"{mode}: warmup step {w + 1}/{args.warmup} done")
        mp.profile_enable(True)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            for f in fmts:
                mp.gemm(f, *inputs[f], outs[f], mode=mode)
        torch.cuda.synchronize()
        t_end = time.perf_counter()
        mp.profile_enable(False)
        sp, gm = mp.profile_read()
        log(f"{mode}: timed {args.steps} steps in {t_end - t_start:.3f} s")
        return t_start, t_end, sp, gm

    t0, t1, split_ms, gemm_ms = timed("float")
    useful = 2.0 * n ** 3 * len(fmts) * args.steps
    value = useful / (t1 - t0) / 1e9
    stages = {}
    for idx, f in enumerate(fmts):
        sp = split_ms[idx::len(fmts)]
        gm = gemm_ms[idx::len(fmts)]
        D = slices[f]
        slice_flops = D * (D + 1) / 2 * 2.0 * n ** 3
        peak = FP32_MFMA_PEAK_TFLOPS if f == "ts" else FP64_MFMA_PEAK_TFLOPS
        g_avg = float(np.mean(gm))
        c, w = W.FORMATS[f][0], (4 if f == "ts" else 8)
        split_bytes = (c * w + D * w) * 2.0 * n * n  # read A and B once, write D slices of each
        stages[f] = {
            "D": D,
            "split_ms": round(float(np.mean(sp)), 3),
            "split_gbs_algorithmic": round(split_bytes / (float(np.mean(sp)) * 1e-3) / 1e9, 1),
            "gemm_kernel_ms": round(g_avg, 3),
            "effective_gflops": round(2.0 * n ** 3 / ((float(np.mean(sp)) + g_avg) * 1e-3) / 1e9, 1),
            "slice_gemm_tflops": round(slice_flops / (g_avg * 1e-3) / 1e12, 2),
            "mfma_frac": round(slice_flops / (g_avg * 1e-3) / 1e12 / peak, 4),
        }
    dom = max(fmts, key=lambda f: stages[f]["gemm_kernel_ms"])
    D = slices[dom]
    peak = FP32_MFMA_PEAK_TFLOPS if dom == "ts" else FP64_MFMA_PEAK_TFLOPS
    achieved = D * (D + 1) / 2 * 2.0 * n ** 3 / (stages[dom]["gemm_kernel_ms"] * 1e-3) / 1e12
    kernel_key = f"k_gemm_plain<{'float' if dom == 'ts' else 'double'},{W.FORMATS[dom][0]}> n={n}"
    roofline = {
        "bound": "mfma",
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": traffic_for(kernel_key),
        "kernel": kernel_key,
    }

    int8 = None
    if not args.no_int8 and all(f != "ts" for f in fmts):
        i0, i1, isp, igm = timed("int8")
        int8 = {"wall_speedup": round((t1 - t0) / (i1 - i0), 3)}
        for idx, f in enumerate(fmts):
            D8 = mp.num_slices(f, "int8", n)
            call_ms = float(np.mean(isp[idx::len(fmts)])) + float(np.mean(igm[idx::len(fmts)]))
            gemm8 = float(np.mean(igm[idx::len(fmts)]))
            ops = D8 * (D8 + 1) / 2 * 2.0 * n ** 3
            split8 = float(np.mean(isp[idx::len(fmts)]))
            int8[f] = {
                "D": D8,
                "split_ms": round(split8, 3),
                "split_gbs_algorithmic": round((W.FORMATS[f][0] * 8 + D8) * 2.0 * n * n / (split8 * 1e-3) / 1e9, 1),
                "gemm_and_combine_ms": round(gemm8, 3),
                "effective_gflops": round(2.0 * n ** 3 / (call_ms * 1e-3) / 1e9, 1),
                "int8_tops": round(ops / (gemm8 * 1e-3) / 1e12, 1),
                "int8_mfma_frac": round(ops / (gemm8 * 1e-3) / 1e12 / INT8_MFMA_PEAK_TOPS, 4),
                "speedup_vs_float_slices": round(
                    (stages[f]["split_ms"] + stages[f]["gemm_kernel_ms"]) / call_ms, 3),
            }
            if not args.no_certify:
                # equal accuracy: the certificate of the INT8 result (one
                # untimed call), and the smallest digit count whose certificate
                # meets 2^-t with its time and speedup (the certificate takes
                # every left-out pair at its largest, so it can ask for a digit
                # more than the exact error does)
                _, _, worst8 = mp.certify(f, *inputs[f], outs[f], mode="int8")
                torch.cuda.synchronize()
                int8[f]["log2_worst_bound_ratio"] = round(float(np.log2(float(worst8.cpu()[0]))), 2)
                _, _, wc, Dc = mp.certify_adaptive(f, *inputs[f], outs[f], mode="int8", d_first=D8, d_last=D8 + 3)
                torch.cuda.synchronize()
                mp.gemm(f, *inputs[f], outs[f], mode="int8", slices=Dc)
                torch.cuda.synchronize()
                mp.profile_enable(True)
                for _ in range(3):
                    mp.gemm(f, *inputs[f], outs[f], mode="int8", slices=Dc)
                torch.cuda.synchronize()
                mp.profile_enable(False)
                csp, cgm = mp.profile_read()
                cms = float(np.mean(csp)) + float(np.mean(cgm))
                int8[f]["certified"] = {
                    "D": Dc,
                    "log2_worst_bound_ratio": round(float(np.log2(float(wc.cpu()[0]))), 2),
                    "call_ms": round(cms, 3),
                    "speedup_vs_float_slices": round(
                        (stages[f]["split_ms"] + stages[f]["gemm_kernel_ms"]) / cms, 3),
                }
                log(f"int8 {f} certified: {int8[f]['certified']}")

    certify = None
    if not args.no_certify:
        # the same products with the a-posteriori certificate (one call each,
        # after a warm call), against the plain call's split + GEMM time
        certify = {}
        for f in fmts:
            mp.certify(f, *inputs[f], outs[f])
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            _, _, worst = mp.certify(f, *inputs[f], outs[f])
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            plain = stages[f]["split_ms"] + stages[f]["gemm_kernel_ms"]
            certify[f] = {
                "certify_call_ms": round(ms, 3),
                "plain_call_ms": round(plain, 3),
                "overhead_frac": round(ms / plain - 1.0, 4),
                "log2_worst_bound_ratio": round(float(np.log2(float(worst.cpu()[0]))), 2),
            }
            log(f"certify {f}: {certify[f]}")

    data = None
    if not args.no_data and all(f != "ts" for f in fmts):
        # the same products with the slice products chosen from the data
        # (16 slices, per-tile pair sets, certified by construction): call
        # time, pairs formed against the automatic triangle, and the
        # certificate of the result
        data = {}
        for f in fmts:
            sets = mp.debug_pair_sets(f, *inputs[f]).cpu().numpy().astype(np.int64)
            mp.set_num_slices(f, "float", -1)
            try:
                mp.gemm(f, *inputs[f], outs[f])
                torch.cuda.synchronize()
                mp.profile_enable(True)
                for _ in range(2):
                    mp.gemm(f, *inputs[f], outs[f])
                torch.cuda.synchronize()
                mp.profile_enable(False)
                sp, gm = mp.profile_read()
                _, _, worst = mp.certify(f, *inputs[f], outs[f])
                torch.cuda.synchronize()
            finally:
                mp.set_num_slices(f, "float", 0)
            D = slices[f]
            pairs = float(sets.sum(axis=2).mean())
            data[f] = {
                "split_and_selection_ms": round(float(np.mean(sp)), 3),
                "gemm_kernel_ms": round(float(np.mean(gm)), 3),
                "call_ms": round(float(np.mean(sp)) + float(np.mean(gm)), 3),
                "automatic_call_ms": round(stages[f]["split_ms"] + stages[f]["gemm_kernel_ms"], 3),
                "pairs_per_tile_mean": round(pairs, 2),
                "automatic_pairs": D * (D + 1) // 2,
                "log2_worst_bound_ratio": round(float(np.log2(float(worst.cpu()[0]))), 2),
            }
            log(f"data-chosen pairs {f}: {data[f]}")

    batched = None
    pool = None
    if not args.no_batched or not args.no_serving:
        from paper_2301_09960_amd import serve
        pool = serve.DevicePool(elements=1 << 24, seed=99)
    if not args.no_batched:
        batched = {}
        for f in ("dd", "qd"):
            batched[f] = run_batched(mp, torch, pool, f)
            log(f"batched {f}: {batched[f]}")
        batched["mixed"] = run_mixed_batch(mp, torch, pool)
        log(f"batched mixed: {batched['mixed']}")
        if not args.no_int8:
            batched["int8"] = {}
            for f in ("dd", "qd"):
                batched["int8"][f] = run_batched(mp, torch, pool, f, mode="int8")
                log(f"batched int8 {f}: {batched['int8'][f]}")
            batched["int8"]["mixed"] = run_mixed_batch(mp, torch, pool, mode="int8")
            log(f"batched int8 mixed: {batched['int8']['mixed']}")
        mp.batched_cache_clear()

    serving = None
    if not args.no_serving:
        from paper_2301_09960_amd import serve

        def serve_at(mode):
            cap = serve.capacity(pool, count=200, mode=mode)
            nreq = args.serve_requests
            reqs = serve.make_requests(nreq + nreq // 10, rate=0.75 * cap, seed=1, pool=pool.elements)
            st = serve.Server(pool, budget_gb=64, streams=8, mode=mode).run(reqs, warmup=nreq // 10)
            return {
                "capacity_req_per_s": round(cap, 1),
                "offered_fraction": 0.75,
                "requests": st.requests,
                "p50_ms": round(st.p50_ms, 3),
                "p99_ms": round(st.p99_ms, 3),
                "throughput_gflops": round(st.throughput_gflops, 1),
                "max_inflight": st.max_inflight,
                "peak_ledger_gb": round(st.peak_ledger_gb, 3),
                "budget_gb": 64,
            }

        serving = serve_at("float")
        if not args.no_int8:
            serving["int8"] = serve_at("int8")
        log(f"serving: {serving}")
    del pool

    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration done (3 x 1 GiB device copies)")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        cpu = cpu_baseline(n, args.E, args.cpu_rows)

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s (effective 2n^3/s)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((t1 - t0) * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"Ozaki GEMM {'+'.join(x.upper() for x in fmts)} m=n=k={n}, e~U{{0..{args.E}}}, "
                        f"binary64 slices on FP64 matrix cores",
            "n": n,
            "formats": fmts,
            "slices": slices,
            "mode": "float",
        },
        "stages": stages,
        "int8": int8,
        "certify": certify,
        "data_chosen_pairs": data,
        "batched": batched,
        "serving": serving,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
