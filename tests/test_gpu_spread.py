"""Wide exponent spreads and the slice counts chosen from the data.

* The automatic D meets the bound on inputs whose exponents spread over 32 and
  60 bits (e ~ U{0..E}), both slice forms, k = 1024 and 4096.
* Rows of A and columns of B with one entry 2^40 above the rest: the grid of
  every slice is set by that entry, so the automatic D misses the bound.  The
  certificate reports it, and the data-chosen pair sets
  (mpgemm_set_num_slices(fmt, FLOAT, MPGEMM_SLICES_DATA)) meet it, certified
  and checked against the exact product.
* The data-chosen pair sets on the benchmark-like inputs of every format and
  on ragged shapes: C within the bound, certificate within it and above the
  exact error entry by entry; the sets are staircases, larger than the
  automatic triangle where outliers need it, and much smaller where the data
  carry fewer bits than the format (lower components zero).
"""
import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu

T_BITS = {"dd": 100, "td": 150, "qd": 200, "ts": 66}
SLICES_DATA = -1


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_09960_amd as mp
    mp.lib()
    assert mp.check_device() == 0
    return mp


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def say(*a):
    print(*a, flush=True)


def bound(orc, fmt, A, B, C):
    diff, absab, _ = orc.exact_check(A, B, C)
    ok, worst = orc.bound_report(diff, absab, T_BITS[fmt])
    return ok, worst, diff


def with_outliers(A, B, seed):
    """One entry of every row of A and of every column of B scaled by 2^40."""
    A, B = A.copy(), B.copy()
    rng = np.random.default_rng(seed)
    _, k, m = A.shape
    n = B.shape[1]
    for i, p in enumerate(rng.integers(0, k, m)):
        A[:, p, i] *= 2.0 ** 40
    for j, p in enumerate(rng.integers(0, k, n)):
        B[:, j, p] *= 2.0 ** 40
    return A, B


class data_slices:
    """The thread's slice count for (fmt, float) set to the data-chosen mode."""

    def __init__(self, mp, fmt):
        self.mp, self.fmt = mp, fmt

    def __enter__(self):
        self.mp.set_num_slices(self.fmt, "float", SLICES_DATA)

    def __exit__(self, *exc):
        self.mp.set_num_slices(self.fmt, "float", 0)


@pytest.mark.parametrize("fmt", ["dd", "qd"])
@pytest.mark.parametrize("mode", ["float", "int8"])
@pytest.mark.parametrize("k", [1024, 4096])
@pytest.mark.parametrize("E", [32, 60])
def test_wide_spread_automatic_slices(mp, orc, fmt, mode, k, E):
    m, n = 48, 40
    A, B = W.gen_pair(fmt, m, n, k, E=E, seed=E + k)
    C = mp.gemm(fmt, dev(A), dev(B), mode=mode).cpu().numpy()
    ok, worst, _ = bound(orc, fmt, A, B, C)
    say(f"spread {fmt} {mode} k={k} E={E}: D={mp.last_num_slices()} worst {worst:.1f} (bound -{T_BITS[fmt]})")
    assert ok


@pytest.mark.parametrize("fmt", ["dd", "qd"])
def test_outliers_need_the_data_chosen_pairs(mp, orc, fmt):
    import torch
    m, n, k = 48, 40, 1024
    A, B = with_outliers(*W.gen_pair(fmt, m, n, k, E=8, seed=3), seed=4)
    dA, dB = dev(A), dev(B)
    t = T_BITS[fmt]
    # the automatic D: the bound is missed, and the certificate says so
    C, cert, worst = mp.certify(fmt, dA, dB)
    torch.cuda.synchronize()
    ok, w_auto, _ = bound(orc, fmt, A, B, C.cpu().numpy())
    say(f"outliers {fmt}: automatic D={mp.last_num_slices()} worst {w_auto:.1f}, "
        f"certificate {np.log2(float(worst.cpu()[0])):.1f} (bound -{t})")
    assert not ok and float(worst.cpu()[0]) > 2.0 ** -t
    # the data-chosen pairs: certified and within the bound
    with data_slices(mp, fmt):
        C2 = mp.gemm(fmt, dA, dB)
        C3, cert3, worst3 = mp.certify(fmt, dA, dB)
    torch.cuda.synchronize()
    assert torch.equal(C2, C3)
    ok, w_data, diff = bound(orc, fmt, A, B, C2.cpu().numpy())
    w_cert = float(worst3.cpu()[0])
    say(f"  data-chosen pairs: worst {w_data:.1f}, certificate {np.log2(w_cert):.1f}")
    assert ok and w_cert <= 2.0 ** -t
    assert np.all(diff <= cert3.cpu().numpy()[0])
    sets = mp.debug_pair_sets(fmt, dA, dB).cpu().numpy().astype(np.int64)
    D = mp.num_slices(fmt, "float", k)
    pairs = sets.sum(axis=2)
    say(f"  pairs per tile {pairs.min()} .. {pairs.max()} (automatic triangle {D * (D + 1) // 2})")
    assert pairs.min() > D * (D + 1) // 2
    # the adaptive certified product finds a D that meets it too
    _, _, worst4, D4 = mp.certify_adaptive(fmt, dA, dB, d_first=mp.num_slices(fmt, "float", k), d_last=16)
    say(f"  adaptive: D={D4} certificate {np.log2(float(worst4.cpu()[0])):.1f}")
    assert float(worst4.cpu()[0]) <= 2.0 ** -t


@pytest.mark.parametrize("fmt", ["dd", "td", "qd", "ts"])
@pytest.mark.parametrize("m,n,k,E", [(200, 150, 333, 16), (130, 70, 1000, 0), (1, 77, 5, 8), (65, 1, 4097, 16)])
def test_data_chosen_pairs_meet_the_bound(mp, orc, fmt, m, n, k, E):
    import torch
    A, B = W.gen_pair(fmt, m, n, k, E=E, seed=m + n + k)
    dA, dB = dev(A), dev(B)
    with data_slices(mp, fmt):
        C, cert, worst = mp.certify(fmt, dA, dB)
    torch.cuda.synchronize()
    ok, w, diff = bound(orc, fmt, A, B, C.cpu().numpy())
    wc = float(worst.cpu()[0])
    say(f"data pairs {fmt} {m}x{n}x{k} E={E}: worst {w:.1f}, certificate "
        f"{np.log2(wc) if wc > 0 else float('-inf'):.1f} (bound -{T_BITS[fmt]})")
    assert ok and wc <= 2.0 ** -T_BITS[fmt]
    assert np.all(diff <= cert.cpu().numpy()[0])
    sets = mp.debug_pair_sets(fmt, dA, dB).cpu().numpy().astype(np.int64)
    assert sets.shape == ((n + 63) // 64, (m + 63) // 64, 16)
    assert np.all((sets >= 0) & (sets <= 16)) and np.all(np.diff(sets, axis=2) <= 0)
    D = mp.num_slices(fmt, "float", k)
    say(f"  pairs per tile {sets.sum(axis=2).min()} .. {sets.sum(axis=2).max()} "
        f"(automatic triangle {D * (D + 1) // 2})")


@pytest.mark.parametrize("fmt,nonzero,most", [("dd", 1, 0.5), ("qd", 2, 0.7)])
def test_data_chosen_pairs_fewer_on_short_data(mp, orc, fmt, nonzero, most):
    """Values with fewer significant bits than the format (DD holding binary64
    values, QD holding DD values: the lower components zero) run out of
    slices early: their later slices are exactly zero, so the data-chosen
    sets form far fewer slice products than the automatic triangle (DD: 9
    pairs against 21; QD: 43 against 66, the exponent spread within rows
    keeping a few more slices nonzero), still certified and within the
    bound."""
    import torch
    m, n, k = 256, 192, 1024
    A, B = W.gen_pair(fmt, m, n, k, E=8, seed=77)
    A[nonzero:] = 0.0
    B[nonzero:] = 0.0
    dA, dB = dev(A), dev(B)
    sets = mp.debug_pair_sets(fmt, dA, dB).cpu().numpy().astype(np.int64)
    D = mp.num_slices(fmt, "float", k)
    mean = sets.sum(axis=2).mean()
    say(f"short data {fmt} ({nonzero} nonzero components): pairs per tile {mean:.1f} "
        f"(automatic triangle {D * (D + 1) // 2})")
    assert mean <= most * (D * (D + 1) // 2)
    with data_slices(mp, fmt):
        C, cert, worst = mp.certify(fmt, dA, dB)
    torch.cuda.synchronize()
    ok, w, _ = bound(orc, fmt, A, B, C.cpu().numpy())
    say(f"  worst {w:.1f}, certificate {np.log2(float(worst.cpu()[0])):.1f} (bound -{T_BITS[fmt]})")
    assert ok and float(worst.cpu()[0]) <= 2.0 ** -T_BITS[fmt]


def test_data_chosen_pairs_zero_rows_and_workspace(mp, orc):
    """Zero rows and columns give exact zeros; an attached workspace of the
    data-mode size suffices and one a little smaller is refused."""
    import torch
    m, n, k = 70, 66, 200
    A, B = W.gen_pair("dd", m, n, k, E=8, seed=9)
    A[:, :, 3] = 0.0
    B[:, 5, :] = 0.0
    dA, dB = dev(A), dev(B)
    with data_slices(mp, "dd"):
        need = mp.workspace_bytes("dd", "float", m, n, k)
        assert need == mp.workspace_bytes("dd", "float", m, n, k, D=SLICES_DATA) > mp.workspace_bytes(
            "dd", "float", m, n, k, D=6)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        mp.set_workspace(ws)
        try:
            C = mp.gemm("dd", dA, dB)
            torch.cuda.synchronize()
            mp.set_workspace(ws[: need - 4096])
            with pytest.raises(mp.MpgemmError) as ei:
                mp.gemm("dd", dA, dB)
            assert ei.value.status == 2
        finally:
            mp.set_workspace(None)
    Ch = C.cpu().numpy()
    assert np.all(Ch[:, :, 3] == 0) and np.all(Ch[:, 5, :] == 0)
    ok, w, _ = bound(orc, "dd", A, B, Ch)
    assert ok
