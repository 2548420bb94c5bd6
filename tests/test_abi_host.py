"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every function the header declares, and its argument checks, slice policy and
workspace sizing behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpgemm.h")


@pytest.fixture(scope="module")
def L():
    import paper_2301_09960_amd as mp
    if not os.path.exists(mp.LIB_PATH):
        from paper_2301_09960_amd import build
        build.build()
    return mp.lib()


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpgemm_\w+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = declared()
    assert len(names) >= 16
    for name in names:
        assert hasattr(L, name), name


def test_argument_codes(L):
    P = ctypes.c_void_p
    x = P(16)  # never dereferenced: the checks fail before any work
    f = L.mpgemm_dd
    assert f(-1, 4, 4, x, 4, x, 4, x, 4, None) == -1
    assert f(4, -1, 4, x, 4, x, 4, x, 4, None) == -2
    assert f(4, 4, -1, x, 4, x, 4, x, 4, None) == -3
    assert f(4, 4, 4, None, 4, x, 4, x, 4, None) == -4
    assert f(4, 4, 4, x, 3, x, 4, x, 4, None) == -5
    assert f(4, 4, 4, x, 4, None, 4, x, 4, None) == -6
    assert f(4, 4, 4, x, 4, x, 3, x, 4, None) == -7
    assert f(4, 4, 4, x, 4, x, 4, None, 4, None) == -8
    assert f(4, 4, 4, x, 4, x, 4, x, 3, None) == -9
    assert L.mpgemm_ts(4, 4, 4, x, 4, x, 4, x, 2, None) == -9
    assert f(1 << 21, 4, 4, x, 1 << 21, x, 4, x, 1 << 21, None) == 5  # beyond the size limit
    # allocation-free DD product: the codes of mpgemm_dd
    assert L.mpgemm_dd_noalloc(4, 4, 4, x, 3, x, 4, x, 4, None) == -5
    # simple in-format product: fmt, staging, then the product's codes shifted by two
    sp = L.mpgemm_simple
    assert sp(9, 1, 4, 4, 4, x, 4, x, 4, x, 4, None) == -1
    assert sp(0, 2, 4, 4, 4, x, 4, x, 4, x, 4, None) == -2
    assert sp(0, 1, -1, 4, 4, x, 4, x, 4, x, 4, None) == -3
    assert sp(3, 0, 4, 4, 4, x, 4, x, 3, x, 4, None) == -9
    assert sp(1, 1, 4, 4, 4, x, 4, x, 4, x, 3, None) == -11
    # D+S: (m, n, k, Ahi, Alo, lda, Bhi, Blo, ldb, Chi, Clo, ldc); the simple form takes staging first
    ds = L.mpgemm_ds
    assert ds(-1, 4, 4, x, x, 4, x, x, 4, x, x, 4, None) == -1
    assert ds(4, 4, 4, x, None, 4, x, x, 4, x, x, 4, None) == -5
    assert ds(4, 4, 4, x, x, 3, x, x, 4, x, x, 4, None) == -6
    assert ds(4, 4, 4, x, x, 4, x, None, 4, x, x, 4, None) == -8
    assert ds(4, 4, 4, x, x, 4, x, x, 4, x, None, 4, None) == -11
    assert ds(4, 4, 4, x, x, 4, x, x, 4, x, x, 3, None) == -12
    dss = L.mpgemm_ds_simple
    assert dss(3, 4, 4, 4, x, x, 4, x, x, 4, x, x, 4, None) == -1
    assert dss(0, 4, -1, 4, x, x, 4, x, x, 4, x, x, 4, None) == -3
    assert dss(1, 4, 4, 4, x, x, 4, x, x, 3, x, x, 4, None) == -10
    # certified product: fmt first, then the product's codes shifted by one
    c = L.mpgemm_certify
    assert c(7, 4, 4, 4, x, 4, x, 4, x, 4, x, x, None) == -1
    assert c(0, -1, 4, 4, x, 4, x, 4, x, 4, x, x, None) == -2
    assert c(0, 4, 4, 4, x, 3, x, 4, x, 4, x, x, None) == -6
    assert c(0, 4, 4, 4, x, 4, x, 4, x, 4, None, x, None) == -11
    assert c(0, 4, 4, 4, x, 4, x, 4, x, 4, x, None, None) == -12
    # adaptive certified product: the certify codes, then the D range and d_used
    ca = L.mpgemm_certify_adaptive
    assert ca(7, 4, 4, 4, x, 4, x, 4, x, 4, x, x, 2, 4, x, None) == -1
    assert ca(0, 4, 4, 4, x, 3, x, 4, x, 4, x, x, 2, 4, x, None) == -6
    assert ca(0, 4, 4, 4, x, 4, x, 4, x, 4, None, x, 2, 4, x, None) == -11
    assert ca(0, 4, 4, 4, x, 4, x, 4, x, 4, x, None, 2, 4, x, None) == -12
    assert ca(0, 4, 4, 4, x, 4, x, 4, x, 4, x, x, 0, 4, x, None) == -13
    assert ca(0, 4, 4, 4, x, 4, x, 4, x, 4, x, x, 17, 17, x, None) == -13  # beyond the binary64 form's 16
    assert ca(0, 4, 4, 4, x, 4, x, 4, x, 4, x, x, 5, 4, x, None) == -14
    assert ca(0, 4, 4, 4, x, 4, x, 4, x, 4, x, x, 5, 17, x, None) == -14
    assert ca(0, 4, 4, 4, x, 4, x, 4, x, 4, x, x, 2, 4, None, None) == -15
    # DD LU and its solve
    assert L.mpgemm_dd_lu(-1, x, 1, 8, None) == -1
    assert L.mpgemm_dd_lu(4, None, 4, 8, None) == -2
    assert L.mpgemm_dd_lu(4, x, 3, 8, None) == -3
    assert L.mpgemm_dd_lu(4, x, 4, 0, None) == -4
    assert L.mpgemm_dd_lu_solve(-1, x, 1, x, None) == -1
    assert L.mpgemm_dd_lu_solve(4, x, 4, None, None) == -4
    assert L.mpgemm_td_lu(4, x, 4, 0, None) == -4
    nc = L.mpgemm_nd_certify
    assert nc(1, 0, 4, 4, 4, x, 4, x, 4, x, 4, x, x, None) == -1
    assert nc(6, -1, 4, 4, 4, x, 4, x, 4, x, 4, x, x, None) == -2
    assert nc(6, 0, 4, 4, 4, x, 4, x, 4, x, 4, None, x, None) == -12
    assert nc(6, 0, 4, 4, 4, x, 4, x, 4, x, 4, x, None, None) == -13
    assert L.mpgemm_td_lu_solve(4, None, 4, x, None) == -2


def test_options_and_policy(L):
    import paper_2301_09960_amd as mp
    # the automatic slice counts at k = 4096 (binary64 slices carry 20 bits there)
    assert [mp.num_slices(f, "float", 4096) for f in ("dd", "td", "qd", "ts")] == [6, 8, 11, 13]
    assert [mp.num_slices(f, "int8", 4096) for f in ("dd", "td", "qd")] == [16, 23, 30]
    assert [mp.num_slices(f, "int8", 128) for f in ("dd", "td", "qd")] == [17, 24, 31]
    with pytest.raises(mp.MpgemmError):
        mp.set_mode("ts", "int8")
    mp.set_num_slices("dd", "float", 9)
    assert mp.num_slices("dd", "float", 4096) == 9
    mp.set_num_slices("dd", "float", 0)
    assert mp.num_slices("dd", "float", 4096) == 6
    with pytest.raises(mp.MpgemmError):
        mp.set_num_slices("dd", "float", 17)
    assert L.mpgemm_status_string(2) == b"workspace too small or allocation failed"
    # split kernel switch: 0 fused where the vectors fit, 1 one launch per pass
    assert mp.split_kernel() == 0
    mp.set_split_kernel(1)
    assert mp.split_kernel() == 1
    mp.set_split_kernel(0)
    with pytest.raises(mp.MpgemmError):
        mp.set_split_kernel(2)
    assert mp.split_kernel() == 0
    # last slice of the split: extracted (default) or Algorithm 1's remainder
    assert mp.last_slice() == "extract"
    mp.set_last_slice("remainder")
    assert mp.last_slice() == "remainder"
    mp.set_last_slice("extract")
    assert L.mpgemm_set_last_slice(2) == -1
    assert mp.last_slice() == "extract"


def test_workspace_bytes(L):
    import paper_2301_09960_amd as mp
    # DD, D = 6, 4096^3: residuals 2 x 2 x 4096^2 x 8 B, packed slices 2 x 6 x 4096^2 x 8 B, plus small arrays
    b = mp.workspace_bytes("dd", "float", 4096, 4096, 4096)
    big = 2 * 2 * 4096 * 4096 * 8 + 2 * 6 * 4096 * 4096 * 8
    assert big <= b <= big + 2 * 6 * 4096 * 8 * 2 + 4096
    # ragged sizes are padded to 64 rows/columns and 32 in k
    assert mp.workspace_bytes("ts", "float", 65, 1, 33, 1) >= 1 * 128 * 64 * 4 + 1 * 64 * 64 * 4


def test_tuning_file_tables(L, tmp_path):
    import paper_2301_09960_amd as mp
    f = tmp_path / "tune.txt"
    f.write_text("# tuned\nqd 3\nslices dd float 1024 5\nslices dd float 4096 7\nslices qd int8 256 29\n")
    try:
        mp.load_tune_file(f)
        assert mp.num_slices("dd", "float", 512) == 5
        assert mp.num_slices("dd", "float", 2048) == 7
        assert mp.num_slices("dd", "float", 8192) == 6  # beyond the table: the formula
        assert mp.num_slices("qd", "int8", 200) == 29 and mp.num_slices("qd", "int8", 300) == 31
        assert mp.num_slices("td", "float", 512) == 8
        assert mp.tile_layout("qd") == 3
        mp.set_num_slices("dd", "float", 9)  # per-thread settings take precedence
        assert mp.num_slices("dd", "float", 512) == 9
        mp.set_num_slices("dd", "float", 0)
        bad = tmp_path / "bad.txt"
        bad.write_text("slices dd float 100 99\n")  # D beyond the limit: rejected, tables kept
        with pytest.raises(mp.MpgemmError):
            mp.load_tune_file(bad)
        assert mp.num_slices("dd", "float", 512) == 5
        with pytest.raises(OSError):
            mp.load_tune_file(tmp_path / "missing.txt")
    finally:
        mp.load_tune_file(None)
    assert mp.num_slices("dd", "float", 512) == 6 and mp.tile_layout("qd") == 2


def test_long_expansion_entry_points(L):
    P = ctypes.c_void_p
    x = P(16)
    f = L.mpgemm_nd
    assert f(1, 0, 4, 4, 4, x, 4, x, 4, x, 4, None) == -1
    assert f(15, 0, 4, 4, 4, x, 4, x, 4, x, 4, None) == -1
    assert f(8, -1, 4, 4, 4, x, 4, x, 4, x, 4, None) == -2
    assert f(8, 113, 4, 4, 4, x, 4, x, 4, x, 4, None) == -2
    assert f(8, 0, -1, 4, 4, x, 4, x, 4, x, 4, None) == -3
    assert f(8, 0, 4, 4, 4, x, 3, x, 4, x, 4, None) == -7
    assert f(8, 0, 4, 4, 4, x, 4, x, 4, x, 3, None) == -11
    # automatic digit slices: the INT8 policy with t = 50 c (c = 2, 3, 4 as DD, TD, QD)
    assert [L.mpgemm_nd_num_slices(c, 128) for c in (2, 3, 4)] == [17, 24, 31]
    assert [L.mpgemm_nd_num_slices(c, 4096) for c in (2, 3, 4)] == [16, 23, 30]
    assert L.mpgemm_nd_num_slices(14, 128) == 102 and L.mpgemm_nd_num_slices(8, 4096) == 59
    assert L.mpgemm_nd_num_slices(1, 128) == -1
    assert L.mpgemm_nd_workspace_bytes(8, 0, 0, 5, 5) == 0
    assert L.mpgemm_nd_workspace_bytes(8, 0, 100, 100, 100) > 59 * 2 * 128 * 128


def test_batched_argument_codes(L):
    IA = ctypes.c_int * 1
    PA = ctypes.c_void_p * 1
    x = PA(16)
    assert L.mpgemm_dd_batched(-1, None, None, None, None, None, None, None, None, None, None) == -1
    assert L.mpgemm_dd_batched(1, None, IA(1), IA(1), x, IA(1), x, IA(1), x, IA(1), None) == -2
    assert L.mpgemm_dd_batched(1, IA(4), IA(4), IA(4), x, IA(3), x, IA(4), x, IA(4), None) == -6
    assert L.mpgemm_qd_batched(1, IA(4), IA(4), IA(4), x, IA(4), x, IA(4), x, IA(2), None) == -10


ENV_PROBE = r"""
import ctypes, json, sys
sys.path.insert(0, sys.argv[1])
import paper_2301_09960_amd as mp
L = mp.lib()
L.mpgemm_workspace_bytes.restype = ctypes.c_size_t
out = {"mode": [L.mpgemm_get_mode(f) for f in range(4)],
       "float": [L.mpgemm_num_slices(f, 0, 1024) for f in range(4)],
       "int8": [L.mpgemm_num_slices(f, 1, 1024) for f in range(3)],
       "ws0": L.mpgemm_workspace_bytes(0, 0, 100, 90, 80, 0),
       "wsdata": L.mpgemm_workspace_bytes(0, 0, 100, 90, 80, -1)}
L.mpgemm_set_mode(0, 0)
out["after_set"] = L.mpgemm_get_mode(0)
print(json.dumps(out))
"""


def env_probe(**env):
    import json
    import subprocess
    import sys
    e = dict(os.environ)
    for k in ("MPGEMM_MODE", "MPGEMM_SLICES"):
        e.pop(k, None)
    e.update(env)
    r = subprocess.run([sys.executable, "-c", ENV_PROBE, ROOT], env=e, capture_output=True, text=True, check=True)
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_environment_defaults(L):
    """MPGEMM_MODE and MPGEMM_SLICES set the starting options of every host
    thread; the setters override them; bad values are ignored."""
    base = env_probe()
    assert base["mode"] == [0, 0, 0, 0]
    p = env_probe(MPGEMM_MODE="int8", MPGEMM_SLICES="7")
    assert p["mode"] == [1, 1, 1, 0]  # TS has no INT8 form
    assert p["float"] == [7, 7, 7, 7] and p["int8"] == [7, 7, 7]
    assert p["after_set"] == 0
    p = env_probe(MPGEMM_SLICES="30")  # beyond the FLOAT range: automatic there
    assert p["float"] == base["float"] and p["int8"] == [30, 30, 30]
    p = env_probe(MPGEMM_SLICES="data")
    assert p["float"] == base["float"] and p["int8"] == base["int8"]
    assert p["ws0"] == p["wsdata"] != base["ws0"]
    p = env_probe(MPGEMM_MODE="fast", MPGEMM_SLICES="7x")
    assert p == base
