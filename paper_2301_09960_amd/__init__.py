"""Ozaki-scheme multi-component GEMM on AMD MI355X (gfx950): Python binding.

This module only marshals arguments to ``libmpgemm.so`` (the C-ABI declared
in ``include/mpgemm.h``); every step of the computation runs in the HIP
kernels.  PyTorch provides device memory and streams.  If the library has not
been built, importing succeeds but every call raises ``RuntimeError`` -- there
is no fallback path.

Tensor conventions (component-planar, column-major planes):
    A (m x k)  -> tensor of shape (c, k, m)
    B (k x n)  -> tensor of shape (c, n, k)
    C (m x n)  -> tensor of shape (c, n, m)
with c = 2 (DD), 3 (TD), 4 (QD) float64 components, or 3 float32 (TS).
``gemm``, ``certify`` and ``gemm_batched`` also take views ``X[:, :, :rows]``
of a (c, cols, ld) buffer: the buffer's ld is passed as the leading dimension
(planes ld * cols elements apart), and C's rows beyond m are left untouched.
Row-major users get C^T = B^T A^T by swapping operands.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpgemm.so")

FORMATS = {"dd": 0, "td": 1, "qd": 2, "ts": 3}
COMPONENTS = {"dd": 2, "td": 3, "qd": 4, "ts": 3}
BOUND_BITS = {"dd": 100, "td": 150, "qd": 200, "ts": 66}
MODES = {"float": 0, "int8": 1}
ZERO_EXP = -(2 ** 31)

_lib = None
_lock = threading.Lock()

_P = ctypes.c_void_p
_I = ctypes.c_int


class MpgemmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: status {status} ({_status_string(status)})")


def lib():
    """The loaded HIP library; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2301_09960_amd.build`")
                # torch first: it brings its own HIP runtime, and the library must
                # bind to that same runtime (loaded first, the library would pull in
                # the system one and torch's device memory would be foreign to it)
                import torch  # noqa: F401
                L = ctypes.CDLL(LIB_PATH)
                for name in ("mpgemm_dd", "mpgemm_td", "mpgemm_qd", "mpgemm_ts"):
                    f = getattr(L, name)
                    f.restype = _I
                    f.argtypes = [_I, _I, _I, _P, _I, _P, _I, _P, _I, _P]
                for name in ("mpgemm_dd_batched", "mpgemm_td_batched", "mpgemm_qd_batched", "mpgemm_ts_batched"):
                    f = getattr(L, name)
                    f.restype = _I
                    f.argtypes = [_I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
                L.mpgemm_set_tile_layout.argtypes = [_I, _I]
                L.mpgemm_tile_layout.argtypes = [_I]
                L.mpgemm_set_int8_tile.argtypes = [_I]
                L.mpgemm_set_split_kernel.argtypes = [_I]
                L.mpgemm_split_kernel.argtypes = []
                L.mpgemm_set_last_slice.argtypes = [_I]
                L.mpgemm_last_slice.argtypes = []
                L.mpgemm_set_mode.argtypes = [_I, _I]
                L.mpgemm_get_mode.argtypes = [_I]
                L.mpgemm_set_num_slices.argtypes = [_I, _I, _I]
                L.mpgemm_num_slices.argtypes = [_I, _I, _I]
                L.mpgemm_workspace_bytes.restype = ctypes.c_size_t
                L.mpgemm_workspace_bytes.argtypes = [_I, _I, _I, _I, _I, _I]
                L.mpgemm_set_workspace.argtypes = [_P, ctypes.c_size_t]
                L.mpgemm_debug_split.argtypes = [_I, _I, _I, _I, _I, _P, _I, _I, _P, _P, _P]
                L.mpgemm_debug_products.argtypes = [_I, _I, _I, _I, _I, _P, _I, _P, _I, _I, _I, _I, _P, _I, _P]
                L.mpgemm_certify.argtypes = [_I, _I, _I, _I, _P, _I, _P, _I, _P, _I, _P, _P, _P]
                L.mpgemm_certify_adaptive.argtypes = [_I, _I, _I, _I, _P, _I, _P, _I, _P, _I, _P, _P, _I, _I, _P,
                                                      _P]
                for name in ("mpgemm_dd_lu", "mpgemm_td_lu"):
                    getattr(L, name).argtypes = [_I, _P, _I, _I, _P]
                for name in ("mpgemm_dd_lu_solve", "mpgemm_td_lu_solve"):
                    getattr(L, name).argtypes = [_I, _P, _I, _P, _P]
                L.mpgemm_profile_enable.argtypes = [_I]
                L.mpgemm_profile_read.argtypes = [_P, _P, _I]
                L.mpgemm_load_tune_file.argtypes = [ctypes.c_char_p]
                L.mpgemm_nd.restype = _I
                L.mpgemm_nd.argtypes = [_I, _I, _I, _I, _I, _P, _I, _P, _I, _P, _I, _P]
                L.mpgemm_nd_certify.argtypes = [_I, _I, _I, _I, _I, _P, _I, _P, _I, _P, _I, _P, _P, _P]
                L.mpgemm_nd_num_slices.argtypes = [_I, _I]
                L.mpgemm_nd_workspace_bytes.restype = ctypes.c_size_t
                L.mpgemm_nd_workspace_bytes.argtypes = [_I, _I, _I, _I, _I]
                L.mpgemm_nd_debug_split.argtypes = [_I, _I, _I, _I, _P, _I, _I, _P, _P, _P]
                L.mpgemm_nd_debug_products.argtypes = [_I, _I, _I, _I, _P, _I, _P, _I, _I, _I, _P, _I, _P]
                L.mpgemm_simple.argtypes = [_I, _I, _I, _I, _I, _P, _I, _P, _I, _P, _I, _P]
                L.mpgemm_ds_simple.argtypes = [_I, _I, _I, _I, _P, _P, _I, _P, _P, _I, _P, _P, _I, _P]
                L.mpgemm_ds.argtypes = [_I, _I, _I, _P, _P, _I, _P, _P, _I, _P, _P, _I, _P]
                L.mpgemm_dd_noalloc.argtypes = [_I, _I, _I, _P, _I, _P, _I, _P, _I, _P]
                L.mpgemm_debug_pair_sets.argtypes = [_I, _I, _I, _I, _P, _I, _P, _I, _P, _P]
                L.mpgemm_status_string.restype = ctypes.c_char_p
                L.mpgemm_status_string.argtypes = [_I]
                _lib = L
    return _lib


def _status_string(status: int) -> str:
    try:
        return lib().mpgemm_status_string(status).decode()
    except Exception:  # library missing while formatting an error
        return "?"


def _check(status: int, what: str):
    if status != 0:
        raise MpgemmError(status, what)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _fmt(fmt) -> int:
    return FORMATS[fmt] if isinstance(fmt, str) else int(fmt)


def _mode(mode) -> int:
    return MODES[mode] if isinstance(mode, str) else int(mode)


def _check_tensor(t, c, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dim() != 3 or t.shape[0] != c:
        raise ValueError(f"{name} must have shape (c={c}, cols, rows), got {tuple(t.shape)}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _planes_ld(t, c, dtype, name) -> int:
    """Leading dimension of a (c, cols, rows) tensor of column-major component
    planes: a contiguous tensor has ld = rows; a view ``X[:, :, :rows]`` of a
    contiguous (c, cols, ld) buffer (strides (ld * cols, ld, 1), ld >= rows)
    passes its buffer's ld, as the C-ABI's plane addressing expects."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dim() != 3 or t.shape[0] != c:
        raise ValueError(f"{name} must have shape (c={c}, cols, rows), got {tuple(t.shape)}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    cols, rows = t.shape[1], t.shape[2]
    if t.is_contiguous():
        return max(1, rows)
    s0, s1, s2 = t.stride()
    if s2 != 1 or s1 < max(1, rows) or (c > 1 and s0 != s1 * cols):
        raise ValueError(f"{name}: planes must be column-major with plane stride ld * cols "
                         f"(strides (ld * {cols}, ld, 1)), got strides {t.stride()}")
    return s1


def set_mode(fmt, mode):
    _check(lib().mpgemm_set_mode(_fmt(fmt), _mode(mode)), "set_mode")


def get_mode(fmt) -> str:
    m = lib().mpgemm_get_mode(_fmt(fmt))
    return {0: "float", 1: "int8"}[m]


def set_tile_layout(fmt, layout: int):
    """Wavefront layout of the slice-product kernel (0 = tuned default, 1..3)."""
    _check(lib().mpgemm_set_tile_layout(_fmt(fmt), int(layout)), "set_tile_layout")


def set_split_kernel(kind: int):
    """Kernel of the binary64/binary32 split, this thread: 0 = fused where the
    rows of A / columns of B fit one workgroup (else one launch per pass),
    1 = one launch per pass always.  Both give the same slices."""
    _check(lib().mpgemm_set_split_kernel(int(kind)), "set_split_kernel")


def split_kernel() -> int:
    return int(lib().mpgemm_split_kernel())


def set_last_slice(last: str):
    """Last slice of the binary64/binary32 split, this thread: ``"extract"``
    (default; every slice product exact) or ``"remainder"`` (Algorithm 1 as
    printed: the residual's leading component after D - 1 passes)."""
    if last not in ("extract", "remainder"):
        raise ValueError(last)
    _check(lib().mpgemm_set_last_slice(1 if last == "remainder" else 0), "set_last_slice")


def last_slice() -> str:
    return "remainder" if lib().mpgemm_last_slice() == 1 else "extract"


def set_int8_tile(cfg: int):
    """INT8-form tile configuration (0 = automatic, 1..3)."""
    _check(lib().mpgemm_set_int8_tile(int(cfg)), "set_int8_tile")


def tile_layout(fmt) -> int:
    return lib().mpgemm_tile_layout(_fmt(fmt))


def set_num_slices(fmt, mode, D: int):
    _check(lib().mpgemm_set_num_slices(_fmt(fmt), _mode(mode), int(D)), "set_num_slices")


def load_tune_file(path=None) -> None:
    """Replace the process-wide tuned tables (wave layouts, slice counts) by a
    tuning file's; None restores the compiled-in tables."""
    st = lib().mpgemm_load_tune_file(None if path is None else str(path).encode())
    if st == -1:
        raise OSError(f"cannot read tuning file {path}")
    _check(st, "load_tune_file")


def num_slices(fmt, mode, k: int) -> int:
    return lib().mpgemm_num_slices(_fmt(fmt), _mode(mode), int(k))


def last_num_slices() -> int:
    return lib().mpgemm_last_num_slices()


def workspace_bytes(fmt, mode, m, n, k, D=0) -> int:
    return lib().mpgemm_workspace_bytes(_fmt(fmt), _mode(mode), m, n, k, D)


def set_workspace(tensor=None):
    """Attach a caller-owned device buffer (a torch tensor) as this thread's workspace; None detaches."""
    if tensor is None:
        _check(lib().mpgemm_set_workspace(None, 0), "set_workspace")
    else:
        _check(lib().mpgemm_set_workspace(ctypes.c_void_p(tensor.data_ptr()), tensor.numel() * tensor.element_size()),
               "set_workspace")


def profile_enable(on: bool = True):
    """Record stage timings (split, fused GEMM kernel) of this thread's later calls."""
    lib().mpgemm_profile_enable(1 if on else 0)


def profile_read(max_calls: int = 4096):
    """Per-call ``(split_ms, gemm_ms)`` lists of the recorded calls, oldest first (waits for the events)."""
    s = (ctypes.c_double * max_calls)()
    g = (ctypes.c_double * max_calls)()
    n = lib().mpgemm_profile_read(s, g, max_calls)
    if n < 0:
        raise MpgemmError(-n, "profile_read")
    return list(s[:n]), list(g[:n])


def check_device() -> int:
    return lib().mpgemm_check_device()


class _options:
    """Temporarily set (mode, slices) for one call on this thread."""

    def __init__(self, fmt, mode, slices):
        self.fmt, self.mode, self.slices = fmt, mode, slices

    def __enter__(self):
        L = lib()
        self.old_mode = L.mpgemm_get_mode(self.fmt)
        if self.mode is not None:
            _check(L.mpgemm_set_mode(self.fmt, self.mode), "set_mode")
        m = L.mpgemm_get_mode(self.fmt)
        self.mode_used = m
        if self.slices is not None:
            _check(L.mpgemm_set_num_slices(self.fmt, m, int(self.slices)), "set_num_slices")
        return self

    def __exit__(self, *exc):
        L = lib()
        if self.slices is not None:
            L.mpgemm_set_num_slices(self.fmt, self.mode_used, 0)
        L.mpgemm_set_mode(self.fmt, self.old_mode)
        return False


def gemm(fmt, A, B, C=None, *, mode=None, slices=None, stream=None):
    """C = A B (Ozaki scheme) for torch tensors in the conventions above.

    ``mode``: 'float' (binary64/binary32 slices) or 'int8'; ``slices``: D
    (None/0 = automatic).  Enqueued on ``stream`` (default: the current
    stream); returns C without synchronizing.
    """
    import torch
    f = _fmt(fmt)
    name = [k for k, v in FORMATS.items() if v == f][0]
    c = COMPONENTS[name]
    dtype = torch.float32 if name == "ts" else torch.float64
    lda = _planes_ld(A, c, dtype, "A")
    ldb = _planes_ld(B, c, dtype, "B")
    k, m = A.shape[1], A.shape[2]
    n, kb = B.shape[1], B.shape[2]
    if kb != k:
        raise ValueError(f"inner dimensions differ: A has k={k}, B has k={kb}")
    if C is None:
        C = torch.empty((c, n, m), dtype=dtype, device=A.device)
    if tuple(C.shape) != (c, n, m):
        raise ValueError(f"C must have shape {(c, n, m)}")
    ldc = _planes_ld(C, c, dtype, "C")
    fn = getattr(lib(), "mpgemm_" + name)
    with _options(f, None if mode is None else _mode(mode), slices):
        st = fn(m, n, k, _P(A.data_ptr()), lda, _P(B.data_ptr()), ldb, _P(C.data_ptr()), ldc, _stream(stream))
    _check(st, "mpgemm_" + name)
    return C


def simple(fmt, A, B, C=None, *, staging: int = 1, stream=None):
    """C = A B by the simple triple loop in the format's own arithmetic (the
    non-Ozaki comparison of Section 4.4), tensors as in ``gemm``.
    ``staging``: 1 stages operand panels through LDS, 0 reads them from
    global memory (same C bit for bit)."""
    import torch
    f = _fmt(fmt)
    name = [k for k, v in FORMATS.items() if v == f][0]
    c = COMPONENTS[name]
    dtype = torch.float32 if name == "ts" else torch.float64
    lda = _planes_ld(A, c, dtype, "A")
    ldb = _planes_ld(B, c, dtype, "B")
    k, m = A.shape[1], A.shape[2]
    n, kb = B.shape[1], B.shape[2]
    if kb != k:
        raise ValueError(f"inner dimensions differ: A has k={k}, B has k={kb}")
    if C is None:
        C = torch.empty((c, n, m), dtype=dtype, device=A.device)
    if tuple(C.shape) != (c, n, m):
        raise ValueError(f"C must have shape {(c, n, m)}")
    ldc = _planes_ld(C, c, dtype, "C")
    _check(lib().mpgemm_simple(f, int(staging), m, n, k, _P(A.data_ptr()), lda, _P(B.data_ptr()), ldb,
                               _P(C.data_ptr()), ldc, _stream(stream)), "mpgemm_simple")
    return C


def _ds_args(Ahi, Alo, Bhi, Blo, Chi, Clo):
    import torch
    for X, dt, nm in ((Ahi, torch.float64, "Ahi"), (Alo, torch.float32, "Alo"), (Bhi, torch.float64, "Bhi"),
                      (Blo, torch.float32, "Blo")):
        if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dtype != dt or X.dim() != 3 or X.shape[0] != 1 \
                or not X.is_contiguous():
            raise ValueError(f"{nm} must be a contiguous CUDA {dt} tensor of shape (1, cols, rows)")
    if Alo.shape != Ahi.shape or Blo.shape != Bhi.shape:
        raise ValueError("hi and lo planes must have one shape")
    k, m = Ahi.shape[1], Ahi.shape[2]
    n, kb = Bhi.shape[1], Bhi.shape[2]
    if kb != k:
        raise ValueError(f"inner dimensions differ: A has k={k}, B has k={kb}")
    if Chi is None:
        Chi = torch.empty((1, n, m), dtype=torch.float64, device=Ahi.device)
    if Clo is None:
        Clo = torch.empty((1, n, m), dtype=torch.float32, device=Ahi.device)
    if tuple(Chi.shape) != (1, n, m) or tuple(Clo.shape) != (1, n, m) or not Chi.is_contiguous() \
            or not Clo.is_contiguous():
        raise ValueError(f"C planes must be contiguous of shape {(1, n, m)}")
    return m, n, k, Chi, Clo


def ds_gemm(Ahi, Alo, Bhi, Blo, Chi=None, Clo=None, *, mode=None, slices=None, stream=None):
    """D+S product through the DD Ozaki product (``mpgemm_ds``): operands as
    (hi, lo) planes of shapes (1, k, m) float64 / float32 and (1, n, k);
    returns ``(Chi, Clo)`` of shape (1, n, m).  ``mode`` / ``slices`` as for DD."""
    m, n, k, Chi, Clo = _ds_args(Ahi, Alo, Bhi, Blo, Chi, Clo)
    with _options(FORMATS["dd"], None if mode is None else _mode(mode), slices):
        st = lib().mpgemm_ds(m, n, k, _P(Ahi.data_ptr()), _P(Alo.data_ptr()), max(1, m), _P(Bhi.data_ptr()),
                             _P(Blo.data_ptr()), max(1, k), _P(Chi.data_ptr()), _P(Clo.data_ptr()), max(1, m),
                             _stream(stream))
    _check(st, "mpgemm_ds")
    return Chi, Clo


def ds_simple(Ahi, Alo, Bhi, Blo, Chi=None, Clo=None, *, staging: int = 1, stream=None):
    """D+S product by the simple triple loop (``mpgemm_ds_simple``)."""
    m, n, k, Chi, Clo = _ds_args(Ahi, Alo, Bhi, Blo, Chi, Clo)
    _check(lib().mpgemm_ds_simple(int(staging), m, n, k, _P(Ahi.data_ptr()), _P(Alo.data_ptr()), max(1, m),
                                  _P(Bhi.data_ptr()), _P(Blo.data_ptr()), max(1, k), _P(Chi.data_ptr()),
                                  _P(Clo.data_ptr()), max(1, m), _stream(stream)), "mpgemm_ds_simple")
    return Chi, Clo


def certify(fmt, A, B, C=None, *, mode="float", slices=None, stream=None):
    """C = A B in the given slice form with its a-posteriori certificate.

    Returns ``(C, cert, worst)``: cert ``(2, n, m)`` float64 holding, per entry,
    an upper bound of |C - AB| (plane 0) and a lower bound of (|A||B|)_ij (plane
    1); worst a one-element float64 tensor with the largest ratio of the two
    (the result meets 2^-t |A||B| everywhere when worst <= 2^-t).  Enqueued on
    ``stream`` without synchronizing.
    """
    import torch
    f = _fmt(fmt)
    name = [k for k, v in FORMATS.items() if v == f][0]
    c = COMPONENTS[name]
    dtype = torch.float32 if name == "ts" else torch.float64
    lda = _planes_ld(A, c, dtype, "A")
    ldb = _planes_ld(B, c, dtype, "B")
    k, m = A.shape[1], A.shape[2]
    n, kb = B.shape[1], B.shape[2]
    if kb != k:
        raise ValueError(f"inner dimensions differ: A has k={k}, B has k={kb}")
    if C is None:
        C = torch.empty((c, n, m), dtype=dtype, device=A.device)
    if tuple(C.shape) != (c, n, m):
        raise ValueError(f"C must have shape {(c, n, m)}")
    ldc = _planes_ld(C, c, dtype, "C")
    cert = torch.empty((2, n, m), dtype=torch.float64, device=A.device)
    worst = torch.empty((1,), dtype=torch.float64, device=A.device)
    with _options(f, _mode(mode), slices):
        st = lib().mpgemm_certify(f, m, n, k, _P(A.data_ptr()), lda, _P(B.data_ptr()), ldb,
                                  _P(C.data_ptr()), ldc, _P(cert.data_ptr()), _P(worst.data_ptr()),
                                  _stream(stream))
    _check(st, "mpgemm_certify")
    return C, cert, worst


def certify_adaptive(fmt, A, B, C=None, *, d_first: int, d_last: int, mode="float", stream=None):
    """``certify`` with the slice count found from the data: the certified
    product at D = d_first, d_first + 1, ... d_last, stopping at the first D
    whose worst ratio meets 2^-t.  Returns ``(C, cert, worst, D)`` for that
    attempt (the d_last attempt's if none is certified: see ``worst``).
    Synchronizes ``stream`` after each attempt."""
    import torch
    f = _fmt(fmt)
    name = [k for k, v in FORMATS.items() if v == f][0]
    c = COMPONENTS[name]
    dtype = torch.float32 if name == "ts" else torch.float64
    _check_tensor(A, c, dtype, "A")
    _check_tensor(B, c, dtype, "B")
    k, m = A.shape[1], A.shape[2]
    n, kb = B.shape[1], B.shape[2]
    if kb != k:
        raise ValueError(f"inner dimensions differ: A has k={k}, B has k={kb}")
    if C is None:
        C = torch.empty((c, n, m), dtype=dtype, device=A.device)
    cert = torch.empty((2, n, m), dtype=torch.float64, device=A.device)
    worst = torch.empty((1,), dtype=torch.float64, device=A.device)
    used = ctypes.c_int(0)
    with _options(f, _mode(mode), None):
        st = lib().mpgemm_certify_adaptive(f, m, n, k, _P(A.data_ptr()), max(1, m), _P(B.data_ptr()), max(1, k),
                                           _P(C.data_ptr()), max(1, m), _P(cert.data_ptr()), _P(worst.data_ptr()),
                                           int(d_first), int(d_last), ctypes.byref(used), _stream(stream))
    _check(st, "mpgemm_certify_adaptive")
    return C, cert, worst, used.value


def lu(fmt, A, K: int, *, mode=None, stream=None):
    """In-place blocked LU (no pivoting, Section 4.6) of a DD or TD matrix ``A``
    of shape ``(c, n, n)`` (component planes, column-major: A[r, j, i] is
    component r of a_ij) with block width K; Schur updates by the library's
    product in ``mode`` ('float' or 'int8', default the thread's).  Returns A
    (now L and U)."""
    import torch
    name = {0: "dd", 1: "td"}.get(_fmt(fmt))
    if name is None:
        raise ValueError("lu: DD or TD only")
    c = COMPONENTS[name]
    _check_tensor(A, c, torch.float64, "A")
    n = A.shape[2]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    with _options(FORMATS[name], None if mode is None else _mode(mode), None):
        st = getattr(lib(), f"mpgemm_{name}_lu")(n, _P(A.data_ptr()), max(1, n), int(K), _stream(stream))
    _check(st, f"mpgemm_{name}_lu")
    return A


def lu_solve(fmt, LU, b, *, stream=None):
    """Solve L U x = b with the factors from ``lu``; b is ``(c, n)`` float64
    (component planes).  Returns x as a new ``(c, n)`` tensor."""
    import torch
    name = {0: "dd", 1: "td"}.get(_fmt(fmt))
    if name is None:
        raise ValueError("lu_solve: DD or TD only")
    c = COMPONENTS[name]
    _check_tensor(LU, c, torch.float64, "LU")
    n = LU.shape[2]
    x = b.detach().clone().contiguous()
    if tuple(x.shape) != (c, n) or x.dtype != torch.float64 or x.device != LU.device:
        raise ValueError(f"b must be a float64 tensor of shape ({c}, {n}) on the device of LU")
    _check(getattr(lib(), f"mpgemm_{name}_lu_solve")(n, _P(LU.data_ptr()), max(1, n), _P(x.data_ptr()),
                                                      _stream(stream)), f"mpgemm_{name}_lu_solve")
    return x


def dd_lu(A, K: int, *, mode=None, stream=None):
    """``lu('dd', ...)``."""
    return lu("dd", A, K, mode=mode, stream=stream)


def dd_lu_solve(LU, b, *, stream=None):
    """``lu_solve('dd', ...)``."""
    return lu_solve("dd", LU, b, stream=stream)


def gemm_batched(fmt, As, Bs, Cs=None, *, mode=None, slices=None, stream=None):
    """C_i = A_i B_i for lists of tensors (conventions as in ``gemm``), as one
    batched launch (graph-captured per batch shape).  ``mode``: 'float' or
    'int8' (DD/TD/QD).  Returns the list of C."""
    import torch
    f = _fmt(fmt)
    name = [k for k, v in FORMATS.items() if v == f][0]
    c = COMPONENTS[name]
    dtype = torch.float32 if name == "ts" else torch.float64
    count = len(As)
    if len(Bs) != count or (Cs is not None and len(Cs) != count):
        raise ValueError("As, Bs and Cs must have the same length")
    ms, ns, ks, ldas, ldbs, ldcs = [], [], [], [], [], []
    for i, (A, B) in enumerate(zip(As, Bs)):
        ldas.append(_planes_ld(A, c, dtype, f"A[{i}]"))
        ldbs.append(_planes_ld(B, c, dtype, f"B[{i}]"))
        if B.shape[2] != A.shape[1]:
            raise ValueError(f"product {i}: inner dimensions differ")
        ms.append(A.shape[2])
        ks.append(A.shape[1])
        ns.append(B.shape[1])
    if Cs is None:
        Cs = [torch.empty((c, n, m), dtype=dtype, device=A.device) for A, m, n in zip(As, ms, ns)]
    for i, Cm in enumerate(Cs):
        if tuple(Cm.shape) != (c, ns[i], ms[i]):
            raise ValueError(f"C[{i}] must have shape {(c, ns[i], ms[i])}")
        ldcs.append(_planes_ld(Cm, c, dtype, f"C[{i}]"))
    IA = ctypes.c_int * max(count, 1)
    PA = ctypes.c_void_p * max(count, 1)
    fn = getattr(lib(), f"mpgemm_{name}_batched")
    with _options(f, None if mode is None else _mode(mode), slices):
        st = fn(count, IA(*ms), IA(*ns), IA(*ks), PA(*[A.data_ptr() for A in As]), IA(*ldas),
                PA(*[B.data_ptr() for B in Bs]), IA(*ldbs), PA(*[Cm.data_ptr() for Cm in Cs]), IA(*ldcs),
                _stream(stream))
    _check(st, f"mpgemm_{name}_batched")
    return Cs


def batched_cache_clear():
    _check(lib().mpgemm_batched_cache_clear(), "batched_cache_clear")


def debug_split(fmt, X, operand: int, D: int = 0, mode="float", stream=None):
    """Slices and exponents of one operand as the GEMM computes them.

    ``operand=0``: X is A ``(c, k, m)`` split by rows; ``operand=1``: X is B
    ``(c, n, k)`` split by columns.  Returns ``(slices, exps)`` with slices
    ``(D, cols, rows)`` (float64 / float32 / int8) and exps ``(D, nvec)`` int32
    (FLOAT) or ``(nvec,)`` (INT8).
    """
    import torch
    f = _fmt(fmt)
    md = _mode(mode)
    name = [k for k, v in FORMATS.items() if v == f][0]
    c = COMPONENTS[name]
    dtype = torch.float32 if name == "ts" else torch.float64
    _check_tensor(X, c, dtype, "X")
    cols, rows = X.shape[1], X.shape[2]
    k = cols if operand == 0 else rows
    if D == 0:
        D = num_slices(f, md, k)
    nvec = rows if operand == 0 else cols
    sdt = torch.int8 if md == 1 else dtype
    slices = torch.zeros((D, cols, rows), dtype=sdt, device=X.device)
    exps = torch.zeros((D, nvec) if md == 0 else (nvec,), dtype=torch.int32, device=X.device)
    _check(lib().mpgemm_debug_split(f, md, operand, rows, cols, _P(X.data_ptr()), max(1, rows), D,
                                    _P(slices.data_ptr()), _P(exps.data_ptr()), _stream(stream)), "debug_split")
    return slices, exps


def _check_nd(X, name):
    import torch
    if X.dim() != 3 or X.dtype != torch.float64 or not X.is_cuda or not X.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape (c, cols, rows)")
    if not 2 <= X.shape[0] <= 14:
        raise ValueError(f"{name}: 2 to 14 components, got {X.shape[0]}")


def gemm_nd(A, B, C=None, *, slices: int = 0, stream=None):
    """C = A B for binary64 expansions of c = 2..14 components (A ``(c, k, m)``,
    B ``(c, n, k)``, C ``(c, n, m)``), INT8-slice form with ``slices`` digit
    slices (0 = automatic: 2^-(50 c) (|A||B|))."""
    import torch
    _check_nd(A, "A")
    _check_nd(B, "B")
    c = A.shape[0]
    if B.shape[0] != c:
        raise ValueError("A and B must have the same number of components")
    k, m = A.shape[1], A.shape[2]
    n, kb = B.shape[1], B.shape[2]
    if kb != k:
        raise ValueError(f"inner dimensions differ: A has k={k}, B has k={kb}")
    if C is None:
        C = torch.empty((c, n, m), dtype=torch.float64, device=A.device)
    elif tuple(C.shape) != (c, n, m) or C.dtype != torch.float64 or not C.is_contiguous():
        raise ValueError(f"C must be a contiguous float64 tensor of shape {(c, n, m)}")
    _check(lib().mpgemm_nd(c, int(slices), m, n, k, _P(A.data_ptr()), max(1, m), _P(B.data_ptr()), max(1, k),
                           _P(C.data_ptr()), max(1, m), _stream(stream)), "mpgemm_nd")
    return C


def nd_certify(A, B, C=None, *, slices: int = 0, stream=None):
    """``gemm_nd`` with its a-posteriori certificate: returns ``(C, cert,
    worst)`` as ``certify`` does (the result meets 2^-(50 c) |A||B| wherever
    cert[0] <= 2^-(50 c) cert[1], everywhere when worst <= 2^-(50 c))."""
    import torch
    _check_nd(A, "A")
    _check_nd(B, "B")
    c = A.shape[0]
    if B.shape[0] != c:
        raise ValueError("A and B must have the same number of components")
    k, m = A.shape[1], A.shape[2]
    n, kb = B.shape[1], B.shape[2]
    if kb != k:
        raise ValueError(f"inner dimensions differ: A has k={k}, B has k={kb}")
    if C is None:
        C = torch.empty((c, n, m), dtype=torch.float64, device=A.device)
    cert = torch.empty((2, n, m), dtype=torch.float64, device=A.device)
    worst = torch.empty((1,), dtype=torch.float64, device=A.device)
    _check(lib().mpgemm_nd_certify(c, int(slices), m, n, k, _P(A.data_ptr()), max(1, m), _P(B.data_ptr()),
                                   max(1, k), _P(C.data_ptr()), max(1, m), _P(cert.data_ptr()),
                                   _P(worst.data_ptr()), _stream(stream)), "mpgemm_nd_certify")
    return C, cert, worst


def nd_num_slices(c: int, k: int) -> int:
    return lib().mpgemm_nd_num_slices(int(c), int(k))


def nd_workspace_bytes(c: int, m: int, n: int, k: int, D: int = 0) -> int:
    return lib().mpgemm_nd_workspace_bytes(int(c), int(D), int(m), int(n), int(k))


def nd_debug_split(X, operand: int, D: int = 0, stream=None):
    """INT8 digits ``(D, cols, rows)`` and exponents ``(nvec,)`` of one operand of gemm_nd."""
    import torch
    _check_nd(X, "X")
    c, cols, rows = X.shape
    k = cols if operand == 0 else rows
    if D == 0:
        D = nd_num_slices(c, k)
    nvec = rows if operand == 0 else cols
    digits = torch.zeros((D, cols, rows), dtype=torch.int8, device=X.device)
    exps = torch.zeros((nvec,), dtype=torch.int32, device=X.device)
    _check(lib().mpgemm_nd_debug_split(c, operand, rows, cols, _P(X.data_ptr()), max(1, rows), D,
                                       _P(digits.data_ptr()), _P(exps.data_ptr()), _stream(stream)), "nd_debug_split")
    return digits, exps


def nd_debug_products(A, B, g: int, D: int = 0, stream=None):
    """The INT8 diagonal sum S_g of gemm_nd, ``(n, m)`` int64."""
    import torch
    _check_nd(A, "A")
    _check_nd(B, "B")
    c, k, m = A.shape
    n = B.shape[1]
    out = torch.zeros((n, m), dtype=torch.int64, device=A.device)
    _check(lib().mpgemm_nd_debug_products(c, m, n, k, _P(A.data_ptr()), max(1, m), _P(B.data_ptr()), max(1, k),
                                          int(D), int(g), _P(out.data_ptr()), max(1, m), _stream(stream)),
           "nd_debug_products")
    return out


def debug_pair_sets(fmt, A, B, stream=None):
    """The pair sets of the data-chosen slice mode for C = A B: an int8 tensor
    ``(tiles_n, tiles_m, 16)``; entry ``[tn, tm, a]`` is how many slices of B
    pair with slice a of A in that 64 x 64 tile of C."""
    import torch
    f = _fmt(fmt)
    name = [k for k, v in FORMATS.items() if v == f][0]
    c = COMPONENTS[name]
    dtype = torch.float32 if name == "ts" else torch.float64
    _check_tensor(A, c, dtype, "A")
    _check_tensor(B, c, dtype, "B")
    k, m = A.shape[1], A.shape[2]
    n = B.shape[1]
    tm, tn = (m + 63) // 64, (n + 63) // 64
    out = torch.zeros((tn, tm, 16), dtype=torch.int8, device=A.device)
    _check(lib().mpgemm_debug_pair_sets(f, m, n, k, _P(A.data_ptr()), max(1, m), _P(B.data_ptr()), max(1, k),
                                        _P(out.data_ptr()), _stream(stream)), "debug_pair_sets")
    return out


def debug_products(fmt, A, B, a: int, b: int = 0, D: int = 0, mode="float", stream=None):
    """FLOAT: the exact slice product C_ab (1-based), ``(n, m)`` float64.
    INT8: the diagonal sum S_g for g = a, ``(n, m)`` int64."""
    import torch
    f = _fmt(fmt)
    md = _mode(mode)
    name = [k for k, v in FORMATS.items() if v == f][0]
    c = COMPONENTS[name]
    dtype = torch.float32 if name == "ts" else torch.float64
    _check_tensor(A, c, dtype, "A")
    _check_tensor(B, c, dtype, "B")
    k, m = A.shape[1], A.shape[2]
    n = B.shape[1]
    out = torch.zeros((n, m), dtype=torch.int64 if md == 1 else torch.float64, device=A.device)
    _check(lib().mpgemm_debug_products(f, md, m, n, k, _P(A.data_ptr()), max(1, m), _P(B.data_ptr()), max(1, k), D,
                                       a, b, _P(out.data_ptr()), max(1, m), _stream(stream)), "debug_products")
    return out
