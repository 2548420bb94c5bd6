"""GPU parity on the square benchmark grid, at full size, in the launch path
the benchmark times.

Cells: n in {1024, 2048, 4096} x {DD, TD, QD} x exponent spread E in {0, 16}
with binary64 slices, TS at n = 4096 with binary32 slices, and the INT8-slice
form of DD, TD and QD at n = 4096.  C is compared with the oracle's exact
product on sampled rows x all columns: at n = 4096 for DD and QD (the
benchmark's two formats, E = 16, the benchmark's inputs) one row in every
64-row tile, so every tile of C of both slice kernels (64 x 64 binary64 tiles,
256 x 256 INT8 tiles) is checked, in both forms against one exact product;
elsewhere one to three rows per cell.  The bound is |C - AB| <= 2^-t (|A||B|)
elementwise (t = 100 / 150 / 200 / 66 for DD / TD / QD / TS), the automatic D.
"""
import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu

T_BITS = {"dd": 100, "td": 150, "qd": 200, "ts": 66}
SEED = 4096  # the benchmark's inputs at n = 4096


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_09960_amd as mp
    mp.lib()
    assert mp.check_device() == 0
    return mp


def say(*a):
    print(*a, flush=True)


def tile_rows(n, tile=64):
    """One row in every tile of `tile` rows, at a varying offset; the first and
    last rows of C included."""
    rows = [t * tile + (37 * t + 11) % tile for t in range(n // tile)]
    rows[0], rows[-1] = 0, n - 1
    return rows


_cache = {}


def products(mp, fmt, n, E, modes):
    """Inputs (host) and the results of the listed slice forms for one cell;
    only the most recent cell is kept (the n = 4096 QD operands are 1 GB)."""
    import torch
    key = (fmt, n, E)
    if key not in _cache:
        _cache.clear()
        seed = SEED if n == 4096 else n + E
        A, B = W.gen_pair(fmt, n, n, n, E=E, seed=seed)
        _cache[key] = {"A": A, "B": B, "C": {}}
    cell = _cache[key]
    todo = [md for md in modes if md not in cell["C"]]
    if todo:
        dA, dB = torch.from_numpy(cell["A"]).cuda(), torch.from_numpy(cell["B"]).cuda()
        for md in todo:
            C = mp.gemm(fmt, dA, dB, mode=md)
            torch.cuda.synchronize()
            cell["C"][md] = (C.cpu().numpy(), mp.last_num_slices())
            del C
        del dA, dB
    return cell["A"], cell["B"], [cell["C"][md] for md in modes]


def check(orc, fmt, A, B, results, modes, rows, label):
    diffs, absab, _ = orc.exact_check_many(A, B, [C for C, _ in results], rows=rows)
    for (C, D), md, diff in zip(results, modes, diffs):
        ok, worst = orc.bound_report(diff, absab, T_BITS[fmt])
        say(f"  {label} {md}: D={D} worst log2(|C-AB|/|A||B|) = {worst:.1f} (bound -{T_BITS[fmt]})")
        assert ok, (label, md, worst)


# (fmt, n, E, rows): the binary64-slice cells other than the two tiled ones
GRID = []
for _n in (1024, 2048, 4096):
    for _fmt in ("dd", "td", "qd"):
        for _E in (0, 16):
            if _n == 4096 and _fmt in ("dd", "qd") and _E == 16:
                continue  # every tile below
            GRID.append((_fmt, _n, _E, [0, (_n * 2) // 3 + 5, _n - 1] if _n < 4096 else [1, _n - 2]))
GRID += [("ts", 4096, 0, [100, 4095]), ("ts", 4096, 16, [17, 2222])]


@pytest.mark.parametrize("fmt,n,E,rows", GRID, ids=[f"{f}-n{n}-E{E}" for f, n, E, _ in GRID])
def test_grid_cell(mp, orc, fmt, n, E, rows):
    say(f"grid {fmt} n={n} E={E} rows={rows}")
    modes = ["float"] + (["int8"] if (n == 4096 and fmt != "ts") else [])
    A, B, res = products(mp, fmt, n, E, modes)
    check(orc, fmt, A, B, res, modes, rows, f"{fmt} n={n} E={E}")


# every 64-row tile at n = 4096, E = 16 (the benchmark's products), both
# slice forms against one exact product; rows in chunks so each test stays short
TILED = [("dd", 0, 2), ("dd", 1, 2), ("qd", 0, 4), ("qd", 1, 4), ("qd", 2, 4), ("qd", 3, 4)]


@pytest.mark.parametrize("fmt,chunk,chunks", TILED, ids=[f"{f}-{c + 1}of{n}" for f, c, n in TILED])
def test_every_tile_n4096(mp, orc, fmt, chunk, chunks):
    n = 4096
    rows = tile_rows(n)
    part = rows[chunk * len(rows) // chunks:(chunk + 1) * len(rows) // chunks]
    say(f"tiles {fmt} n={n} E=16 rows {part[0]}..{part[-1]} ({len(part)} rows)")
    modes = ["float", "int8"]
    A, B, res = products(mp, fmt, n, 16, modes)
    check(orc, fmt, A, B, res, modes, part, f"{fmt} n={n} E=16")
