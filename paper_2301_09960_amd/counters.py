"""HBM traffic of one kernel from two `rocprofv3 --pmc` runs.

`FETCH_SIZE` and `WRITE_SIZE` (KiB per dispatch) are taken in separate runs
of the same command, which also performs plain 1 GiB device-to-device copies
(`bench.py --copy-calibration`). What each counter reads for such a copy, against
the 1 GiB it really moves, gives the factor that turns the kernel's reading into
bytes:

    python -m paper_2301_09960_amd.counters --fetch DIR1 --write DIR2 \
        --kernel "k_gemm_plain<double, 4, 2>" --algorithmic-bytes 3489660928 \
        --source paper_2301_09960_amd/csrc/gemm_fp.hip --out traffic.json

DIR1 and DIR2 are the `-d` output folders of the two runs. The summary keeps a
hash of the kernel source, so readers can tell whether it is current.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

COPY_KERNEL = "copyBuffer"
GIB_KIB = 1 << 20


def dispatch_values(folder: str, counter: str) -> dict:
    """{kernel name: [counter value per dispatch]} from every counter CSV below `folder`."""
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


def kernel_mean(values: dict, sub: str) -> float:
    vals = [v for name, vs in values.items() if sub in name for v in vs]
    if not vals:
        raise SystemExit(f"no dispatch of a kernel matching {sub!r}")
    return sum(vals) / len(vals)


def copy_kib_per_gib(values: dict) -> float:
    """Counter reading of one 1 GiB copy: the copy dispatches that moved at least
    a quarter of a GiB by the counter (smaller runtime copies are ignored)."""
    vals = [v for name, vs in values.items() if COPY_KERNEL in name for v in vs if v >= GIB_KIB / 4]
    if not vals:
        raise SystemExit("no 1 GiB copy dispatch found (run the command with --copy-calibration)")
    return sum(vals) / len(vals)


def source_hash(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def summarize(fetch_dir, write_dir, kernel, algorithmic_bytes, source, label, commands=()):
    fv = dispatch_values(fetch_dir, "FETCH_SIZE")
    wv = dispatch_values(write_dir, "WRITE_SIZE")
    fk, wk = kernel_mean(fv, kernel), kernel_mean(wv, kernel)
    cf, cw = copy_kib_per_gib(fv), copy_kib_per_gib(wv)
    ff, wf = GIB_KIB / cf, GIB_KIB / cw
    fb, wb = fk * 1024 * ff, wk * 1024 * wf
    return {
        "kernel": label,
        "kernel_match": kernel,
        "source_sha256_16": source_hash(source),
        "fetch_kib_counter": fk,
        "write_kib_counter": wk,
        "copy_fetch_kib_per_gib": cf,
        "copy_write_kib_per_gib": cw,
        "fetch_factor": ff,
        "write_factor": wf,
        "fetch_bytes": fb,
        "write_bytes": wb,
        "bytes_per_launch": fb + wb,
        "algorithmic_bytes": algorithmic_bytes,
        "commands": list(commands),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True, help="rocprofv3 -d folder of the FETCH_SIZE run")
    ap.add_argument("--write", required=True, help="rocprofv3 -d folder of the WRITE_SIZE run")
    ap.add_argument("--kernel", required=True, help="substring of the kernel's name")
    ap.add_argument("--label", default="", help="name written into the summary (default: --kernel)")
    ap.add_argument("--algorithmic-bytes", type=float, required=True)
    ap.add_argument("--source", required=True, help="the kernel's source file (hashed)")
    ap.add_argument("--command", action="append", default=[], help="command of a run, recorded as given")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    s = summarize(a.fetch, a.write, a.kernel, a.algorithmic_bytes, a.source, a.label or a.kernel, a.command)
    text = json.dumps(s, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text)


if __name__ == "__main__":
    main()
