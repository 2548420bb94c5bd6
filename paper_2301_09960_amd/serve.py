"""Serving loop for multi-component GEMM requests (continuous batching).

Requests (format uniform over DD/TD/QD, m, n, k log-uniform in [lo, hi],
entries with exponent spread e ~ U{0..8}) arrive by a seeded Poisson process.
The server admits a waiting request as soon as a stream slot is free and its
device memory fits the HBM budget.  Admitted requests run concurrently, one
per HIP stream, so work of requests that arrive while others are on the GPU
overlaps on the device.  Latency is measured from arrival to the completion
event and includes staging the operands.

Device memory and the ledger:
* Operands come from a device pool of synthetic values generated once (the
  requests' source data, outside the budget).  At admission a request's
  operands are copied out of the pool and its output allocated, on its
  stream; they are charged to the ledger at an upper bound of what the
  caching allocator holds for them (512-byte units plus a block's possible
  slack) and released at completion.  Its slices and the product's other
  temporaries live in the stream slot's workspace.
* Each stream slot owns a library workspace sized for the largest request of
  the run, allocated when the run starts and charged to the ledger, as
  allocated, for the whole run (a stream-ordered allocation inside the library could otherwise
  wait for the other streams under load).
So the device memory the server holds beyond the pool never exceeds the
ledger, and the ledger never exceeds the budget (a test checks
torch.cuda.memory_allocated against it at every admission and completion).

Run a rate sweep: ``python -m paper_2301_09960_amd.serve --sweep``.
"""
from __future__ import annotations

import argparse
import json
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import COMPONENTS, gemm, set_workspace, workspace_bytes

FMTS = ("dd", "td", "qd")
GB = 1 << 30


@dataclass
class Request:
    rid: int
    fmt: str
    m: int
    n: int
    k: int
    arrival: float  # seconds from the start of the run
    a_off: int = 0
    b_off: int = 0
    start: float = math.nan
    done: float = math.nan
    bytes: int = 0
    A: object = None
    B: object = None
    C: object = None
    kept: object = None  # the result, when the run keeps results
    event: object = None
    stream_slot: int = -1

    @property
    def flops(self) -> float:
        return 2.0 * self.m * self.n * self.k


@dataclass
class ServeStats:
    rate: float
    requests: int
    p50_ms: float
    p99_ms: float
    mean_ms: float
    throughput_gflops: float
    max_inflight: int
    peak_ledger_gb: float
    wall_s: float
    extra: dict = field(default_factory=dict)


def make_requests(count: int, rate: float, seed: int = 0, lo: int = 64, hi: int = 2048, pool: int = 1 << 24):
    """Seeded request stream: Poisson arrivals at ``rate`` per second."""
    from workload import log_uniform_sizes, uniform01, uniform_int
    m = log_uniform_sizes(seed, count, lo, hi, draw=0)
    n = log_uniform_sizes(seed, count, lo, hi, draw=1)
    k = log_uniform_sizes(seed, count, lo, hi, draw=2)
    f = uniform_int(seed, 4, 0, count, 0, len(FMTS) - 1)
    gaps = -np.log1p(-uniform01(seed, 4, 1, count)) / rate
    t = np.cumsum(gaps)
    ao = uniform_int(seed, 4, 2, count, 0, pool - 1)
    bo = uniform_int(seed, 4, 3, count, 0, pool - 1)
    out = []
    for i in range(count):
        r = Request(i, FMTS[f[i]], int(m[i]), int(n[i]), int(k[i]), float(t[i]))
        r.a_off = int(ao[i]) % max(1, pool - r.m * r.k)
        r.b_off = int(bo[i]) % max(1, pool - r.k * r.n)
        out.append(r)
    return out


class DevicePool:
    """Synthetic component planes on the device (one pool per format), from
    which request operands are sliced."""

    def __init__(self, elements: int = 1 << 24, seed: int = 99):
        import torch

        from workload import gen_matrix
        self.elements = elements
        self.planes = {}
        for fmt in FMTS:
            X = gen_matrix(fmt, elements, 1, E=8, seed=seed, operand="A")  # (c, 1, elements)
            self.planes[fmt] = torch.from_numpy(np.ascontiguousarray(X[:, 0, :])).cuda()

    def operand(self, fmt, rows, cols, offset):
        P = self.planes[fmt]
        return P[:, offset:offset + rows * cols].reshape(P.shape[0], cols, rows).contiguous()


def batch_operands(pool: DevicePool, fmt: str, count: int = 512, seed: int = 31, lo: int = 64, hi: int = 1024,
                   first: int = 0):
    """Operands of a batch of ``count`` independent products with m, n, k each
    log-uniform in [lo, hi] (seeded), sliced out of the pool at seeded
    offsets.  Products ``first .. first + count - 1`` of the seed's sequence.
    Returns ``(As, Bs, m, n, k)`` (device tensors and integer arrays)."""
    from workload import log_uniform_sizes, uniform_int
    total = first + count
    m = log_uniform_sizes(seed, total, lo, hi, draw=0)[first:]
    n = log_uniform_sizes(seed, total, lo, hi, draw=1)[first:]
    k = log_uniform_sizes(seed, total, lo, hi, draw=2)[first:]
    offs = uniform_int(seed, 5, 0, 2 * total, 0, pool.elements - 1)[2 * first:]
    As, Bs = [], []
    for i in range(count):
        ao = int(offs[2 * i]) % (pool.elements - int(m[i] * k[i]))
        bo = int(offs[2 * i + 1]) % (pool.elements - int(k[i] * n[i]))
        As.append(pool.operand(fmt, int(m[i]), int(k[i]), ao))
        Bs.append(pool.operand(fmt, int(k[i]), int(n[i]), bo))
    return As, Bs, m, n, k


class Server:
    """Admits requests under an HBM budget onto a fixed set of streams."""

    UNIT = 512  # allocation granularity of torch's caching allocator
    LARGE = 1 << 20  # a block of the allocator's large pool can carry up to this much unsplit slack

    def __init__(self, pool: DevicePool, budget_gb: float = 64.0, streams: int = 8, mode: str = "float"):
        import torch
        self.pool = pool
        self.mode = mode  # slice form of every request: "float" (binary64 slices) or "int8"
        self.budget = int(budget_gb * GB)
        self.ledger = 0
        self.peak = 0
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.free_slots = deque(range(streams))
        self.ws = [None] * streams  # per-slot library workspace
        self.ws_charge = [0] * streams
        self.on_change = None  # called with the server after every admission and completion

    @classmethod
    def units(cls, nbytes: int) -> int:
        """An upper bound of the device memory torch's caching allocator holds
        for one tensor of nbytes: rounded to 512 bytes, plus the remainder of
        a cached block it may hand out unsplit (below 512 bytes in the small
        pool, below 1 MiB in the large one)."""
        n = -(-max(int(nbytes), 1) // cls.UNIT) * cls.UNIT
        return n + (cls.LARGE if n > cls.LARGE else cls.UNIT)

    def cost(self, r: Request) -> int:
        """Bytes a request holds while admitted: its operand copies and output."""
        c = COMPONENTS[r.fmt]
        return self.units(8 * c * r.m * r.k) + self.units(8 * c * r.k * r.n) + self.units(8 * c * r.m * r.n)

    def reserve(self, reqs):
        """One workspace per stream slot, for the largest request of the run,
        charged to the ledger for the whole run."""
        import torch
        need = max(workspace_bytes(r.fmt, self.mode, r.m, r.n, r.k) for r in reqs)
        if self.ledger + len(self.ws) * self.units(need) > self.budget:
            raise ValueError(f"slot workspaces of {len(self.ws) * need / GB:.2f} GB exceed the budget")
        for i in range(len(self.ws)):
            before = torch.cuda.memory_allocated()
            self.ws[i] = torch.empty(need, dtype=torch.uint8, device="cuda")
            # charged as allocated (the allocator rounds and may add a block's slack)
            self.ws_charge[i] = torch.cuda.memory_allocated() - before
            self.ledger += self.ws_charge[i]
        if self.ledger > self.budget:
            raise ValueError(f"slot workspaces of {self.ledger / GB:.2f} GB exceed the budget")
        self.peak = max(self.peak, self.ledger)

    def stage(self, r: Request):
        """Operands (compact copies out of the pool) and output in HBM, on the
        current stream."""
        import torch
        r.A = self.pool.operand(r.fmt, r.m, r.k, r.a_off)
        r.B = self.pool.operand(r.fmt, r.k, r.n, r.b_off)
        r.C = torch.empty((COMPONENTS[r.fmt], r.n, r.m), dtype=r.A.dtype, device=r.A.device)

    def launch(self, r: Request, now: float):
        import torch
        slot = self.free_slots.popleft()
        st = self.streams[slot]
        r.stream_slot = slot
        r.start = now
        self.ledger += r.bytes
        self.peak = max(self.peak, self.ledger)
        with torch.cuda.stream(st):
            self.stage(r)
            set_workspace(self.ws[slot])
            try:
                gemm(r.fmt, r.A, r.B, r.C, mode=self.mode, stream=st)
            finally:
                set_workspace(None)
        r.event = torch.cuda.Event()
        r.event.record(st)
        if self.on_change:
            self.on_change(self)

    def run(self, reqs, warmup: int = 0, keep_results: bool = False) -> ServeStats:
        """Replays the arrival trace in real time; returns latency statistics of
        the requests after the first ``warmup``."""
        import torch
        self.reserve(reqs)
        for r in reqs:
            r.bytes = self.cost(r)
            if self.ledger + r.bytes > self.budget:
                raise ValueError(f"request {r.rid} needs {r.bytes / GB:.1f} GB beside the slot workspaces, "
                                 f"above the budget")
        waiting = deque()
        inflight = []
        pending = deque(reqs)
        max_inflight = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admit in arrival order while a slot and memory are free
            while waiting and self.free_slots and self.ledger + waiting[0].bytes <= self.budget:
                r = waiting.popleft()
                self.launch(r, now)
                inflight.append(r)
            max_inflight = max(max_inflight, len(inflight))
            still = []
            for r in inflight:
                if r.event.query():
                    r.done = time.perf_counter() - t0
                    self.free_slots.append(r.stream_slot)
                    r.A = r.B = None
                    if keep_results:
                        r.kept = r.C  # held by the caller from here on, outside the ledger
                    r.C = None
                    self.ledger -= r.bytes
                    if self.on_change:
                        self.on_change(self)
                else:
                    still.append(r)
            inflight = still
            if not inflight and not waiting and pending:
                time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.001)))
        wall = time.perf_counter() - t0
        for i in range(len(self.ws)):  # the run's reservation ends with it
            self.ledger -= self.ws_charge[i]
            self.ws[i] = None
            self.ws_charge[i] = 0
        meas = reqs[warmup:]
        lat = np.array([(r.done - r.arrival) * 1e3 for r in meas])
        span = max(r.done for r in meas) - min(r.arrival for r in meas)
        return ServeStats(
            rate=float(len(reqs) / max(reqs[-1].arrival, 1e-9)),
            requests=len(meas),
            p50_ms=float(np.percentile(lat, 50)),
            p99_ms=float(np.percentile(lat, 99)),
            mean_ms=float(lat.mean()),
            throughput_gflops=float(sum(r.flops for r in meas) / span / 1e9),
            max_inflight=max_inflight,
            peak_ledger_gb=self.peak / GB,
            wall_s=wall,
        )


def capacity(pool: DevicePool, count: int = 200, seed: int = 5, streams: int = 8, mode: str = "float") -> float:
    """Requests per second the server completes with every request present at t = 0."""
    reqs = make_requests(count, rate=1e9, seed=seed, pool=pool.elements)
    for r in reqs:
        r.arrival = 0.0
    st = Server(pool, streams=streams, mode=mode).run(reqs)
    return count / st.wall_s


def sweep(fractions=(0.25, 0.5, 0.75, 0.9, 1.0, 1.2), requests: int = 2000, warmup: int = 200, seed: int = 1,
          streams: int = 8, mode: str = "float"):
    pool = DevicePool()
    cap = capacity(pool, streams=streams, mode=mode)
    out = {"capacity_req_per_s": cap, "mode": mode, "points": []}
    for fr in fractions:
        reqs = make_requests(requests + warmup, rate=fr * cap, seed=seed, pool=pool.elements)
        st = Server(pool, streams=streams, mode=mode).run(reqs, warmup=warmup)
        st.extra["mode"] = mode
        st.extra["fraction_of_capacity"] = fr
        out["points"].append(st.__dict__)
        print(json.dumps({k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.__dict__.items()}),
              flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--streams", type=int, default=8)
    ap.add_argument("--mode", default="float", choices=("float", "int8"))
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    res = sweep(requests=args.requests, warmup=args.warmup, streams=args.streams, mode=args.mode)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
