"""ctypes binding of libspmv (include/spmv.h): argument marshalling only.

Every function here checks Python-side types, turns arrays and tensors into
pointers and sizes, and calls the C entry point of the same name; all the work
of the path runs in the library's C++ runtime and gfx950 kernels.  Host arrays
are numpy arrays; device vectors are torch tensors on the GPU (torch provides
device memory and streams, nothing else).  A failing call raises SpmvError
with the library's status and message.

There is no fallback: if libspmv.so has not been built, the first call raises
ImportError.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# SPMV_LIBRARY selects another build of the library (for example one with
# host sanitizers); by default the in-tree libspmv.so is loaded.
LIB_PATH = os.environ.get("SPMV_LIBRARY") or os.path.join(_PKG, "libspmv.so")

# status codes
SPMV_OK = 0
SPMV_ERR_INVALID_ARG = -1
SPMV_ERR_INVALID_MATRIX = -2
SPMV_ERR_ALLOC = -3
SPMV_ERR_HIP = -4
SPMV_ERR_UNSUPPORTED = -5
SPMV_ERR_STATE = -6

# precision modes
PREC = {"f64": 0, "f32": 1, "bf16": 2, "f32f64": 3}
PREC_NAMES = {v: k for k, v in PREC.items()}
# element type of B and C per mode
VEC_DTYPE = {"f64": "float64", "f32": "float32", "bf16": "float32", "f32f64": "float64"}
# storage type of val per mode (bf16 as uint16 codes)
VAL_DTYPE = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16, "f32f64": np.float32}

SPMV_FLAG_ALLOW_PAGEABLE_HALO = 0x1
SPMV_FLAG_NO_TUNE_CACHE = 0x2

SPMV_KERNEL_STREAM = 1
SPMV_KERNEL_VECTOR = 2
SPMV_KERNEL_TILE_GRID = 3
SPMV_KERNEL_STAGED = 4
SPMV_KERNEL_FUSED_PANELS = 5
SPMV_KERNEL_SORTED_BLOCKS = 6
SPMV_PART_MAIN = 0
SPMV_PART_NONLOCAL = 1

SPMV_KIND_PLAIN = 0
SPMV_KIND_SPLIT = 1
SPMV_KIND_BATCH = 2
SPMV_KIND_SYMMETRIC = 3

SPMV_ARR_ROW_PTR = 0
SPMV_ARR_COL = 1
SPMV_ARR_VAL = 2
SPMV_ARR_NL_ROWS = 3
SPMV_ARR_NL_PTR = 4
SPMV_ARR_NL_COL = 5
SPMV_ARR_NL_VAL = 6
SPMV_ARR_SEND_IDX = 7
SPMV_ARR_TILES = 8
SPMV_ARR_RUNS = 9

SPMV_SCHEDULE_OVERLAP = 0
SPMV_SCHEDULE_SERIAL = 1
SPMV_SCHEDULE_BATCH_GRAPH = 0
SPMV_SCHEDULE_BATCH_DIRECT = 2
SPMV_SCHEDULE_BATCH_FLAT = 3
SPMV_SCHEDULE_OVERLAP_NONLOCAL = 4
SPMV_SCHEDULE_OVERLAP_MERGED = 5

EXPORTED = [
    "spmv_create_crs", "spmv_create_sym_crs", "spmv_split_local_nonlocal", "spmv_run",
    "spmv_run_block",
    "spmv_destroy", "spmv_last_error", "spmv_create_batch", "spmv_get_plan",
    "spmv_set_plan", "spmv_tune", "spmv_get_info", "spmv_export", "spmv_probe_copy",
    "spmv_probe_triad", "spmv_probe_read", "spmv_probe_spin", "spmv_set_schedule",
    "spmv_set_send_list", "spmv_send_list_symmetric", "spmv_run_exchange", "spmv_probe_atomic",
    "spmv_kpm_moments", "spmv_set_phase_timing", "spmv_phase_times", "spmv_lanczos",
    "spmv_get_block_plan", "spmv_lanczos_noalloc", "spmv_probe_gather",
    "spmv_probe_gather_sums_needed",
]


class SpmvError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libspmv status {status}: {message}")
        self.status = status
        self.message = message


class spmv_plan_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("kernel", "tile_items", "lanes", "nontemporal", "xcd_remap", "block_kt",
                 "tiles_per_group", "panels")]


class spmv_info_t(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("halo_begin", ctypes.c_int64), ("nnz_local", ctypes.c_int64),
        ("nnz_nonlocal", ctypes.c_int64), ("n_nonlocal_rows", ctypes.c_int64),
        ("batch_count", ctypes.c_int32), ("n_tiles", ctypes.c_int64),
        ("row_len_mean", ctypes.c_double), ("row_len_cv", ctypes.c_double),
        ("row_len_max", ctypes.c_int64), ("n_send", ctypes.c_int64),
        ("n_staged_tiles", ctypes.c_int64),
    ]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def load():
    """Load libspmv.so (raises ImportError if it has not been built).

    PyTorch is imported first when it is installed: the library then binds
    to the HIP runtime torch carries (both name the same shared object), so
    the process has one runtime and torch's streams and buffers are the
    library's.  Loaded the other way round, torch cannot bring up its own
    copy of the runtime afterwards."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1106_5908_amd.build")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "spmv_create_crs": [_i64, _i64, _i64, _vp, _vp, _vp, _i32, _i32, ctypes.c_uint32, _vp],
        "spmv_create_sym_crs": [_i64, _i64, _vp, _vp, _vp, _i32, _i32, ctypes.c_uint32, _vp],
        "spmv_split_local_nonlocal": [_vp, _i64, _vp],
        "spmv_run": [_vp, _vp, _vp, _vp, _vp],
        "spmv_run_block": [_vp, _i32, _vp, _i64, _vp, _i64, _vp],
        "spmv_destroy": [_vp],
        "spmv_create_batch": [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32, ctypes.c_uint32, _vp],
        "spmv_get_plan": [_vp, _i32, _vp],
        "spmv_set_plan": [_vp, _i32, _vp],
        "spmv_tune": [_vp, _i32, _vp],
        "spmv_get_info": [_vp, _vp],
        "spmv_export": [_vp, _i32, _vp, _i64, _vp],
        "spmv_probe_copy": [_vp, _vp, _i64, _vp],
        "spmv_probe_triad": [_vp, _vp, _vp, ctypes.c_double, _i64, _vp],
        "spmv_probe_spin": [_i64, _vp],
        "spmv_probe_read": [_vp, _i64, _vp, _i64, _vp],
        "spmv_set_schedule": [_vp, _i32],
        "spmv_set_send_list": [_vp, _vp, _i64],
        "spmv_send_list_symmetric": [_vp, _vp],
        "spmv_run_exchange": [_vp, _vp, _vp, _vp, _vp, _vp],
        "spmv_probe_atomic": [_vp, _i64, _i32, _i32, _vp],
        "spmv_kpm_moments": [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp],
        "spmv_set_phase_timing": [_vp, _i32],
        "spmv_phase_times": [_vp, _vp],
        "spmv_lanczos": [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp],
        "spmv_get_block_plan": [_vp, _i32, _vp],
        "spmv_lanczos_noalloc": [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp],
        "spmv_probe_gather": [_vp, _i64, _i32, _vp, _i64, _i32, _vp, _i64, _vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.spmv_probe_gather_sums_needed.argtypes = [_i64, _i32]
    lib.spmv_probe_gather_sums_needed.restype = _i64
    lib.spmv_last_error.argtypes = []
    lib.spmv_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != SPMV_OK:
        msg = load().spmv_last_error().decode(errors="replace")
        raise SpmvError(status, msg)


def spmv_last_error() -> str:
    return load().spmv_last_error().decode(errors="replace")


class Handle:
    """Owns one spmv_handle_t; destroyed by spmv_destroy() or when collected."""

    def __init__(self, ptr: int, prec: str, kind: int):
        self.ptr = ptr
        self.prec = prec
        self.kind = kind
        info = spmv_get_info(self)
        self.n_rows = info["n_rows"]
        self.n_cols = info["n_cols"]
        self.halo_begin = info["halo_begin"]

    @property
    def vec_dtype(self) -> str:
        return VEC_DTYPE[self.prec]

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            try:
                _lib.spmv_destroy(ctypes.c_void_p(self.ptr))
            except Exception:
                pass
            self.ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        spmv_destroy(self)


def _hp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def _as(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _prec(prec) -> str:
    if isinstance(prec, int):
        return PREC_NAMES[prec]
    if prec not in PREC:
        raise ValueError(f"unknown precision {prec!r}")
    return prec


def spmv_create_crs(row_ptr, col_idx, val, n_cols: int, index_base: int = 0,
                    prec: str = "f64", flags: int = 0, n_rows: Optional[int] = None,
                    nnz: Optional[int] = None) -> Handle:
    """spmv_create_crs: host CRS arrays (int32 / int32 / float64)."""
    prec = _prec(prec)
    rp = _as(row_ptr, np.int32)
    ci = _as(col_idx, np.int32)
    v = _as(val, np.float64)
    n_rows = rp.size - 1 if n_rows is None else n_rows
    nnz = ci.size if nnz is None else nnz
    out = ctypes.c_void_p()
    _check(load().spmv_create_crs(n_rows, n_cols, nnz, _hp(rp) if rp.size else rp.ctypes.data,
                                  _hp(ci), _hp(v), index_base, PREC[prec], flags,
                                  ctypes.byref(out)))
    return Handle(out.value, prec, SPMV_KIND_PLAIN)


def spmv_create_sym_crs(row_ptr, col_idx, val, index_base: int = 0, prec: str = "f64",
                        flags: int = 0) -> Handle:
    """spmv_create_sym_crs: the upper triangle (col >= row) of a symmetric
    matrix in host CRS arrays; spmv_run then applies the whole matrix."""
    prec = _prec(prec)
    rp = _as(row_ptr, np.int32)
    ci = _as(col_idx, np.int32)
    v = _as(val, np.float64)
    out = ctypes.c_void_p()
    _check(load().spmv_create_sym_crs(rp.size - 1, ci.size, _hp(rp) if rp.size else rp.ctypes.data,
                                      _hp(ci), _hp(v), index_base, PREC[prec], flags,
                                      ctypes.byref(out)))
    return Handle(out.value, prec, SPMV_KIND_SYMMETRIC)


def spmv_split_local_nonlocal(h: Handle, halo_begin_col: int) -> Handle:
    out = ctypes.c_void_p()
    _check(load().spmv_split_local_nonlocal(_ptr(h), halo_begin_col, ctypes.byref(out)))
    return Handle(out.value, h.prec, SPMV_KIND_SPLIT)


def spmv_create_batch(members: Sequence, index_base: int = 0, prec: str = "f64",
                      flags: int = 0) -> Handle:
    """spmv_create_batch: members are (row_ptr, col_idx, val, n_cols) tuples."""
    prec = _prec(prec)
    count = len(members)
    keep = []
    n_rows = np.empty(count, np.int64)
    n_cols = np.empty(count, np.int64)
    nnz = np.empty(count, np.int64)
    rps = (ctypes.c_void_p * count)()
    cis = (ctypes.c_void_p * count)()
    vs = (ctypes.c_void_p * count)()
    for m, (rp, ci, v, nc) in enumerate(members):
        rp = _as(rp, np.int32)
        ci = _as(ci, np.int32)
        v = _as(v, np.float64)
        keep += [rp, ci, v]
        n_rows[m] = rp.size - 1
        n_cols[m] = nc
        nnz[m] = ci.size
        rps[m] = rp.ctypes.data
        cis[m] = ci.ctypes.data if ci.size else None
        vs[m] = v.ctypes.data if v.size else None
    out = ctypes.c_void_p()
    _check(load().spmv_create_batch(count, _hp(n_rows), _hp(n_cols), _hp(nnz), rps, cis, vs,
                                    index_base, PREC[prec], flags, ctypes.byref(out)))
    del keep
    return Handle(out.value, prec, SPMV_KIND_BATCH)


def _ptr(h: Handle):
    if not isinstance(h, Handle):
        raise TypeError("expected a Handle")
    return ctypes.c_void_p(h.ptr) if h.ptr else None


def _dev(t, dtype: str, name: str):
    import torch

    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if str(t.dtype) != "torch." + dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else None


def _stream(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def spmv_run(h: Handle, B, C, B_halo_host=None, stream=None) -> None:
    """spmv_run: C = C + A*B on `stream` (default: torch's current stream).

    B_halo_host (split handles only) is a CPU torch tensor, preferably pinned."""
    bp, cp, hp = _check_vectors(h, B, C, B_halo_host)
    _check(load().spmv_run(_ptr(h), bp, cp, hp, _stream(stream)))


def _check_vectors(h: Handle, B, C, B_halo_host):
    """Pointers of B, C and the optional halo tensor after the size checks the
    C side cannot make for device buffers."""
    dt = h.vec_dtype
    bp = _dev(B, dt, "B")
    cp = _dev(C, dt, "C")
    if B is None or B.numel() != h.n_cols or not B.is_contiguous():
        raise ValueError(f"B must be a contiguous tensor of {h.n_cols} elements")
    if C is None or C.numel() != h.n_rows or not C.is_contiguous():
        raise ValueError(f"C must be a contiguous tensor of {h.n_rows} elements")
    hp = None
    if B_halo_host is not None:
        if B_halo_host.is_cuda or str(B_halo_host.dtype) != "torch." + dt or not B_halo_host.is_contiguous():
            raise TypeError(f"B_halo_host must be a contiguous CPU tensor of dtype {dt}")
        if B_halo_host.numel() != h.n_cols - h.halo_begin:
            raise ValueError(f"B_halo_host must hold {h.n_cols - h.halo_begin} elements")
        hp = ctypes.c_void_p(B_halo_host.data_ptr()) if B_halo_host.numel() else None
    return bp, cp, hp


def spmv_set_send_list(h: Handle, send_idx) -> None:
    """spmv_set_send_list: positions in B (all below the halo start) whose
    elements spmv_run_exchange sends, in send order."""
    a = np.ascontiguousarray(send_idx, dtype=np.int32)
    _check(load().spmv_set_send_list(_ptr(h), _hp(a), a.size))


def spmv_send_list_symmetric(h: Handle) -> int:
    """spmv_send_list_symmetric: send list of a structurally symmetric matrix;
    returns its length."""
    n = ctypes.c_int64()
    _check(load().spmv_send_list_symmetric(_ptr(h), ctypes.byref(n)))
    return n.value


def spmv_run_exchange(h: Handle, B, C, B_halo_host=None, send_host=None, stream=None) -> None:
    """spmv_run_exchange: pack and send B[send list] into send_host (a pinned
    CPU tensor of the vector dtype), receive the halo, C = C + A*B."""
    bp, cp, hp = _check_vectors(h, B, C, B_halo_host)
    n_send = spmv_get_info(h)["n_send"]
    sp = None
    if send_host is not None:
        dt = h.vec_dtype
        if send_host.is_cuda or str(send_host.dtype) != "torch." + dt or not send_host.is_contiguous():
            raise TypeError(f"send_host must be a contiguous CPU tensor of dtype {dt}")
        if send_host.numel() != n_send:
            raise ValueError(f"send_host must hold {n_send} elements")
        sp = ctypes.c_void_p(send_host.data_ptr()) if send_host.numel() else None
    _check(load().spmv_run_exchange(_ptr(h), bp, cp, hp, sp, _stream(stream)))


PHASES = ("copy", "local", "nonlocal", "send")


def spmv_set_phase_timing(h: Handle, on: bool = True) -> None:
    _check(load().spmv_set_phase_timing(_ptr(h), int(bool(on))))


def spmv_phase_times(h: Handle) -> dict:
    """{phase: (start_ms, end_ms) or None} of the last timed call, from its start."""
    t = (ctypes.c_double * 8)()
    _check(load().spmv_phase_times(_ptr(h), t))
    return {p: (None if t[2 * i] < 0 else (t[2 * i], t[2 * i + 1])) for i, p in enumerate(PHASES)}


def spmv_run_block(h: Handle, B, C, stream=None) -> None:
    """spmv_run_block: B [n_cols x k], C [n_rows x k], row-major (unit column stride)."""
    dt = h.vec_dtype
    if B.dim() != 2 or C.dim() != 2 or B.shape[1] != C.shape[1]:
        raise ValueError("B and C must be 2-D with the same number of columns")
    if B.stride(1) != 1 or C.stride(1) != 1:
        raise ValueError("B and C must be row-major with unit column stride")
    k = B.shape[1]
    if B.shape[0] != h.n_cols or C.shape[0] != h.n_rows:
        raise ValueError(f"B must have {h.n_cols} rows and C {h.n_rows} rows")
    _check(load().spmv_run_block(_ptr(h), k, _dev(B, dt, "B"), B.stride(0), _dev(C, dt, "C"),
                                 C.stride(0), _stream(stream)))


def spmv_kpm_moments(h: Handle, V0, M: int, W1=None, W2=None, stream=None):
    """spmv_kpm_moments: Chebyshev moments mu[m, r] = v0_r . T_m(H) v0_r for
    the columns of V0 (a CUDA float64 tensor [n_rows x R], row-major).  Work
    blocks are allocated when not given.  Returns mu as a CUDA tensor [M x R]."""
    import torch

    if V0.dim() != 2 or V0.shape[0] != h.n_rows or not V0.is_contiguous():
        raise ValueError(f"V0 must be a contiguous [{h.n_rows} x R] tensor")
    R = V0.shape[1]
    W1 = torch.empty_like(V0) if W1 is None else W1
    W2 = torch.empty_like(V0) if W2 is None else W2
    for name, W in (("W1", W1), ("W2", W2)):
        if W.shape != V0.shape or not W.is_contiguous():
            raise ValueError(f"{name} must be a contiguous tensor shaped like V0")
    mu = torch.empty((M, R), dtype=torch.float64, device=V0.device)
    _check(load().spmv_kpm_moments(_ptr(h), R, M, _dev(V0, "float64", "V0"), _dev(W1, "float64", "W1"),
                                   _dev(W2, "float64", "W2"), _dev(mu, "float64", "mu"),
                                   _stream(stream)))
    return mu


def spmv_lanczos(h: Handle, q, m: int, V1=None, V2=None, stream=None):
    """spmv_lanczos: m plain Lanczos steps from q (a CUDA float64 vector of
    n_rows); returns (alpha, beta) as CUDA tensors of m elements."""
    import torch

    if q.dim() != 1 or q.numel() != h.n_rows or not q.is_contiguous():
        raise ValueError(f"q must be a contiguous vector of {h.n_rows} elements")
    V1 = torch.empty_like(q) if V1 is None else V1
    V2 = torch.empty_like(q) if V2 is None else V2
    for name, V in (("V1", V1), ("V2", V2)):
        if V.shape != q.shape or not V.is_contiguous():
            raise ValueError(f"{name} must be a contiguous vector shaped like q")
    alpha = torch.empty(m, dtype=torch.float64, device=q.device)
    beta = torch.empty(m, dtype=torch.float64, device=q.device)
    _check(load().spmv_lanczos(_ptr(h), m, _dev(q, "float64", "q"), _dev(V1, "float64", "V1"),
                               _dev(V2, "float64", "V2"), _dev(alpha, "float64", "alpha"),
                               _dev(beta, "float64", "beta"), _stream(stream)))
    return alpha, beta


def spmv_lanczos_noalloc(h: Handle, q, m: int, V1, V2, alpha, beta, stream=None) -> None:
    """spmv_lanczos_noalloc: as spmv_lanczos, into caller-provided buffers
    (V1, V2 like q; alpha, beta of at least m float64 elements on the same
    device); neither this wrapper nor the library allocates."""
    if q.dim() != 1 or q.numel() != h.n_rows or not q.is_contiguous():
        raise ValueError(f"q must be a contiguous vector of {h.n_rows} elements")
    for name, V in (("V1", V1), ("V2", V2)):
        if V.shape != q.shape or not V.is_contiguous():
            raise ValueError(f"{name} must be a contiguous vector shaped like q")
    for name, a in (("alpha", alpha), ("beta", beta)):
        if a.dim() != 1 or a.numel() < m or not a.is_contiguous():
            raise ValueError(f"{name} must be a contiguous vector of at least {m} elements")
    _check(load().spmv_lanczos_noalloc(_ptr(h), m, _dev(q, "float64", "q"),
                                       _dev(V1, "float64", "V1"), _dev(V2, "float64", "V2"),
                                       _dev(alpha, "float64", "alpha"),
                                       _dev(beta, "float64", "beta"), _stream(stream)))


def spmv_destroy(h: Handle) -> None:
    if h is None or not h.ptr:
        return
    p = h.ptr
    h.ptr = None
    _check(load().spmv_destroy(ctypes.c_void_p(p)))


def spmv_get_plan(h: Handle, part: int = SPMV_PART_MAIN) -> dict:
    p = spmv_plan_t()
    _check(load().spmv_get_plan(_ptr(h), part, ctypes.byref(p)))
    return {n: getattr(p, n) for n, _ in spmv_plan_t._fields_}


def spmv_get_block_plan(h: Handle, k: int) -> dict:
    """The plan spmv_run_block uses for blocks of k columns on this handle."""
    p = spmv_plan_t()
    _check(load().spmv_get_block_plan(_ptr(h), k, ctypes.byref(p)))
    return {n: getattr(p, n) for n, _ in spmv_plan_t._fields_}


def spmv_set_plan(h: Handle, part: int = SPMV_PART_MAIN, **fields) -> None:
    cur = spmv_get_plan(h, part)
    cur.update(fields)
    p = spmv_plan_t(**cur)
    _check(load().spmv_set_plan(_ptr(h), part, ctypes.byref(p)))


def spmv_tune(h: Handle, k: int = 1, stream=None) -> None:
    _check(load().spmv_tune(_ptr(h), k, _stream(stream)))


def spmv_get_info(h: Handle) -> dict:
    i = spmv_info_t()
    _check(load().spmv_get_info(_ptr(h), ctypes.byref(i)))
    return {n: getattr(i, n) for n, _ in spmv_info_t._fields_}


_EXPORT_DTYPE = {SPMV_ARR_ROW_PTR: np.int32, SPMV_ARR_COL: np.int32, SPMV_ARR_NL_ROWS: np.int32,
                 SPMV_ARR_NL_PTR: np.int32, SPMV_ARR_NL_COL: np.int32, SPMV_ARR_SEND_IDX: np.int32,
                 SPMV_ARR_TILES: np.int32, SPMV_ARR_RUNS: np.int32}


def spmv_export(h: Handle, which: int) -> np.ndarray:
    """Copy one device array of the handle back to the host."""
    size = ctypes.c_int64()
    lib = load()
    _check(lib.spmv_export(_ptr(h), which, None, 0, ctypes.byref(size)))
    dt = _EXPORT_DTYPE.get(which, VAL_DTYPE[h.prec])
    out = np.empty(size.value // np.dtype(dt).itemsize, dtype=dt)
    _check(lib.spmv_export(_ptr(h), which, _hp(out), size.value, ctypes.byref(size)))
    if which == SPMV_ARR_TILES:
        return out.reshape(-1, 2)  # (first row, first entry) per tile start
    if which == SPMV_ARR_RUNS:
        return out.reshape(-1, 12)
    return out


def spmv_set_schedule(h: Handle, schedule: int) -> None:
    _check(load().spmv_set_schedule(_ptr(h), schedule))


def spmv_probe_copy(dst, src, stream=None) -> None:
    if dst.numel() < src.numel():
        raise ValueError("dst is shorter than src")
    _check(load().spmv_probe_copy(_dev(dst, "float64", "dst"), _dev(src, "float64", "src"),
                                  src.numel(), _stream(stream)))


def spmv_probe_triad(a, b, c, s: float, stream=None) -> None:
    if not (a.numel() == b.numel() == c.numel()):
        raise ValueError("triad operands differ in length")
    _check(load().spmv_probe_triad(_dev(a, "float64", "a"), _dev(b, "float64", "b"),
                                   _dev(c, "float64", "c"), s, a.numel(), _stream(stream)))


def spmv_probe_read(src, sums, stream=None) -> None:
    """Read-only stream over src (float64); per-workgroup sums into sums."""
    _check(load().spmv_probe_read(_dev(src, "float64", "src"), src.numel(),
                                  _dev(sums, "float64", "sums"), sums.numel(), _stream(stream)))


def read_sums_needed(n: int) -> int:
    return (n // 2 + 1023) // 1024 + 1


ATOMIC_THREADS = 2048 * 256


def spmv_probe_atomic(C, scattered: bool, iters: int, stream=None) -> int:
    """FP64 atomic adds of 1.0 into C (float64, power-of-two length); returns
    how many were made (ATOMIC_THREADS * iters)."""
    _check(load().spmv_probe_atomic(_dev(C, "float64", "C"), C.numel(), int(bool(scattered)),
                                    int(iters), _stream(stream)))
    return ATOMIC_THREADS * int(iters)


def gather_sums_needed(n: int, width: int) -> int:
    v = int(load().spmv_probe_gather_sums_needed(int(n), int(width)))
    if v < 0:
        raise ValueError("bad n or width")
    return v


def spmv_probe_gather(src, idx, width: int = 1, xcd_remap: bool = True, sums=None,
                      stream=None):
    """Gather probe: `width` doubles of row idx[k] of src (float64, viewed as
    rows of width doubles) for every index of idx (int32); returns the
    per-workgroup sums (float64 CUDA tensor)."""
    import torch

    if src.numel() % width:
        raise ValueError("src length must be a multiple of width")
    if idx.dtype != torch.int32 or not idx.is_contiguous():
        raise ValueError("idx must be a contiguous int32 tensor")
    need = gather_sums_needed(idx.numel(), width)
    if sums is None:
        sums = torch.empty(max(need, 1), dtype=torch.float64, device=src.device)
    _check(load().spmv_probe_gather(_dev(src, "float64", "src"), src.numel() // width, int(width),
                                    ctypes.c_void_p(idx.data_ptr()), idx.numel(),
                                    int(bool(xcd_remap)), _dev(sums, "float64", "sums"),
                                    sums.numel(), _stream(stream)))
    return sums


def spmv_probe_spin(nanoseconds: int, stream=None) -> None:
    _check(load().spmv_probe_spin(int(nanoseconds), _stream(stream)))
