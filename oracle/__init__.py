"""ctypes wrapper of ``spmv_oracle.c``, the plain sequential FP64 reference.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the package smoke
check and by the benchmark's CPU-baseline leg.  The GPU library never imports,
links or calls anything in this directory, and this directory imports nothing
from the GPU library.

What each function computes is documented in ``spmv_oracle.c`` with the
passage of the paper it follows (Listing 1 for the kernel, Sect. 3.4 for the
local / nonlocal split, Sect. 3.3 for the send buffer).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spmv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra", "-shared", "-fPIC"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_p = ctypes.c_void_p

_SIGNATURES = {
    "oracle_spmv": [_i64, _p, _p, _p, _i32, _p, _p],
    "oracle_spmv_rows": [_i64, _p, _p, _p, _p, _i32, _p, _p],
    "oracle_spmv_block": [_i64, _p, _p, _p, _i32, _i32, _p, _i64, _p, _i64],
    "oracle_abs_spmv": [_i64, _p, _p, _p, _i32, _p, _p, _p],
    "oracle_split_count": [_i64, _p, _p, _i32, _i64, _p, _p, _p],
    "oracle_split_fill": [_i64, _p, _p, _p, _i32, _i64, _p, _p, _p, _p, _p, _p, _p],
    "oracle_spmv_split": [_i64, _p, _p, _p, _i64, _p, _p, _p, _p, _p, _p],
    "oracle_kpm_moments": [_i64, _p, _p, _p, _i32, _i32, _i32, _p, _p],
    "oracle_lanczos": [_i64, _p, _p, _p, _i32, _i32, _p, _p, _p],
    "oracle_pack": [_i64, _p, _p, _p],
    "oracle_send_list_symmetric": [_i64, _p, _p, _i32, _i64, _p, _p],
    "oracle_round_f32": [_i64, _p, _p],
    "oracle_round_bf16": [_i64, _p, _p],
    "oracle_bf16_to_f64": [_i64, _p, _p],
}


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Oracle:
    """The oracle functions bound to one compiled copy of spmv_oracle.c.

    The module-level functions use the copy built from this directory; the
    test suite also binds copies built from deliberately altered sources to
    show that its pins reject them."""

    def __init__(self, libpath: str):
        lib = ctypes.CDLL(libpath)
        for name, args in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = None
        lib.oracle_kpm_moments.restype = ctypes.c_int
        lib.oracle_lanczos.restype = ctypes.c_int
        self._lib = lib

    def spmv(self, row_ptr, col_idx, val, B, C0=None, base: int = 0) -> np.ndarray:
        """C = C0 + A*B by Listing 1 (C0 defaults to zeros); returns a new array."""
        row_ptr = _c(row_ptr, np.int32)
        col_idx = _c(col_idx, np.int32)
        val = _c(val, np.float64)
        B = _c(B, np.float64)
        n = row_ptr.size - 1
        C = np.zeros(n) if C0 is None else np.array(C0, dtype=np.float64, copy=True)
        assert C.size == n
        self._lib.oracle_spmv(n, _ptr(row_ptr), _ptr(col_idx), _ptr(val), base, _ptr(B), _ptr(C))
        return C

    def spmv_rows(self, rows, row_ptr, col_idx, val, B, C0_sel=None, base: int = 0) -> np.ndarray:
        """Entries ``rows`` of C0 + A*B, each computed by the Listing 1 loop."""
        rows = _c(rows, np.int64)
        row_ptr = _c(row_ptr, np.int32)
        col_idx = _c(col_idx, np.int32)
        val = _c(val, np.float64)
        B = _c(B, np.float64)
        n = row_ptr.size - 1
        if rows.size and (rows.min() < 0 or rows.max() >= n):
            raise IndexError("row out of range")
        out = np.zeros(rows.size) if C0_sel is None else np.array(C0_sel, dtype=np.float64, copy=True)
        self._lib.oracle_spmv_rows(rows.size, _ptr(rows), _ptr(row_ptr), _ptr(col_idx), _ptr(val),
                                 base, _ptr(B), _ptr(out))
        return out

    def spmv_block(self, row_ptr, col_idx, val, B, C0=None, base: int = 0) -> np.ndarray:
        """C = C0 + A*B for a row-major block B [n_cols x k]; returns [n_rows x k]."""
        row_ptr = _c(row_ptr, np.int32)
        col_idx = _c(col_idx, np.int32)
        val = _c(val, np.float64)
        B = _c(B, np.float64)
        assert B.ndim == 2
        k = B.shape[1]
        n = row_ptr.size - 1
        C = np.zeros((n, k)) if C0 is None else np.array(C0, dtype=np.float64, copy=True, order="C")
        assert C.shape == (n, k)
        self._lib.oracle_spmv_block(n, _ptr(row_ptr), _ptr(col_idx), _ptr(val), base, k,
                                  _ptr(B), k, _ptr(C), k)
        return C

    def abs_spmv(self, row_ptr, col_idx, val, B, C0=None, base: int = 0) -> np.ndarray:
        """Per-row |C0| + sum |a_ij| |b_j|: the denominator of the normalised error."""
        row_ptr = _c(row_ptr, np.int32)
        col_idx = _c(col_idx, np.int32)
        val = _c(val, np.float64)
        B = _c(B, np.float64)
        n = row_ptr.size - 1
        C0 = np.zeros(n) if C0 is None else _c(C0, np.float64)
        D = np.empty(n)
        self._lib.oracle_abs_spmv(n, _ptr(row_ptr), _ptr(col_idx), _ptr(val), base, _ptr(B),
                                _ptr(C0), _ptr(D))
        return D

    def split(self, row_ptr, col_idx, val, h: int, base: int = 0) -> dict:
        """Local (columns < h) / nonlocal (columns >= h) parts, Sect. 3.4."""
        row_ptr = _c(row_ptr, np.int32)
        col_idx = _c(col_idx, np.int32)
        val = _c(val, np.float64)
        n = row_ptr.size - 1
        lib = self._lib
        cnt = [ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()]
        lib.oracle_split_count(n, _ptr(row_ptr), _ptr(col_idx), base, h,
                               *(ctypes.byref(c) for c in cnt))
        nnz_loc, nnz_nl, R = (c.value for c in cnt)
        out = {
            "loc_row_ptr": np.empty(n + 1, np.int32),
            "loc_col": np.empty(nnz_loc, np.int32),
            "loc_val": np.empty(nnz_loc, np.float64),
            "nl_rows": np.empty(R, np.int32),
            "nl_ptr": np.empty(R + 1, np.int32),
            "nl_col": np.empty(nnz_nl, np.int32),
            "nl_val": np.empty(nnz_nl, np.float64),
        }
        lib.oracle_split_fill(n, _ptr(row_ptr), _ptr(col_idx), _ptr(val), base, h,
                              *(_ptr(out[k]) for k in ("loc_row_ptr", "loc_col", "loc_val", "nl_rows",
                                                       "nl_ptr", "nl_col", "nl_val")))
        return out

    def spmv_split(self, parts: dict, B, C0=None) -> np.ndarray:
        """Local part then nonlocal part (Sect. 3.4) on the arrays from split()."""
        B = _c(B, np.float64)
        n = parts["loc_row_ptr"].size - 1
        C = np.zeros(n) if C0 is None else np.array(C0, dtype=np.float64, copy=True)
        self._lib.oracle_spmv_split(n, _ptr(parts["loc_row_ptr"]), _ptr(parts["loc_col"]),
                                  _ptr(parts["loc_val"]), parts["nl_rows"].size,
                                  _ptr(parts["nl_rows"]), _ptr(parts["nl_ptr"]),
                                  _ptr(parts["nl_col"]), _ptr(parts["nl_val"]), _ptr(B), _ptr(C))
        return C

    def kpm_moments(self, row_ptr, col_idx, val, V0, M: int, base: int = 0) -> np.ndarray:
        """Chebyshev moments mu[m, r] = V0[:, r] . T_m(H) V0[:, r] by the plain
        recursion (Sect. 1.3 applications); V0 is [n_rows x R]."""
        row_ptr = _c(row_ptr, np.int32)
        col_idx = _c(col_idx, np.int32)
        val = _c(val, np.float64)
        V0 = _c(V0, np.float64)
        n = row_ptr.size - 1
        assert V0.ndim == 2 and V0.shape[0] == n
        R = V0.shape[1]
        mu = np.empty((M, R), np.float64)
        if self._lib.oracle_kpm_moments(n, _ptr(row_ptr), _ptr(col_idx), _ptr(val), base, R, M,
                                        _ptr(V0), _ptr(mu)) != 0:
            raise MemoryError("oracle_kpm_moments")
        return mu

    def lanczos(self, row_ptr, col_idx, val, q, m: int, base: int = 0):
        """m plain Lanczos steps from q (Sect. 1.3 applications): returns
        (alpha[m], beta[m])."""
        row_ptr = _c(row_ptr, np.int32)
        col_idx = _c(col_idx, np.int32)
        val = _c(val, np.float64)
        q = _c(q, np.float64)
        n = row_ptr.size - 1
        assert q.size == n
        alpha = np.empty(m, np.float64)
        beta = np.empty(m, np.float64)
        if self._lib.oracle_lanczos(n, _ptr(row_ptr), _ptr(col_idx), _ptr(val), base, m, _ptr(q),
                                    _ptr(alpha), _ptr(beta)) != 0:
            raise MemoryError("oracle_lanczos")
        return alpha, beta

    def pack(self, idx, B) -> np.ndarray:
        """Send buffer B[idx] (Sect. 3.3)."""
        idx = _c(idx, np.int32)
        B = _c(B, np.float64)
        if idx.size and (idx.min() < 0 or idx.max() >= B.size):
            raise IndexError("send index out of range")
        out = np.empty(idx.size, np.float64)
        self._lib.oracle_pack(idx.size, _ptr(idx), _ptr(B), _ptr(out))
        return out

    def send_list_symmetric(self, row_ptr, col_idx, h: int, base: int = 0) -> np.ndarray:
        """Rows i < h with an entry in a column >= h (send list of a
        structurally symmetric matrix split at h)."""
        row_ptr = _c(row_ptr, np.int32)
        col_idx = _c(col_idx, np.int32)
        n = row_ptr.size - 1
        out = np.empty(max(n, 1), np.int32)
        cnt = ctypes.c_int64()
        self._lib.oracle_send_list_symmetric(n, _ptr(row_ptr), _ptr(col_idx), base, h, _ptr(out),
                                             ctypes.byref(cnt))
        return out[:cnt.value].copy()

    def round_f32(self, x) -> np.ndarray:
        x = _c(x, np.float64)
        out = np.empty(x.size, np.float32)
        self._lib.oracle_round_f32(x.size, _ptr(x), _ptr(out))
        return out.reshape(x.shape)

    def round_bf16(self, x) -> np.ndarray:
        """bfloat16 codes (uint16) of binary64 inputs, single rounding, RNE."""
        x = _c(x, np.float64)
        out = np.empty(x.size, np.uint16)
        self._lib.oracle_round_bf16(x.size, _ptr(x), _ptr(out))
        return out.reshape(x.shape)

    def bf16_to_f64(self, codes) -> np.ndarray:
        codes = _c(codes, np.uint16)
        out = np.empty(codes.size, np.float64)
        self._lib.oracle_bf16_to_f64(codes.size, _ptr(codes), _ptr(out))
        return out.reshape(codes.shape)


_default = None


def default() -> Oracle:
    """The oracle built from spmv_oracle.c in this directory."""
    global _default
    if _default is None:
        _default = Oracle(build())
    return _default


def spmv(*args, **kwargs):
    return default().spmv(*args, **kwargs)


def spmv_rows(*args, **kwargs):
    return default().spmv_rows(*args, **kwargs)


def spmv_block(*args, **kwargs):
    return default().spmv_block(*args, **kwargs)


def abs_spmv(*args, **kwargs):
    return default().abs_spmv(*args, **kwargs)


def split(*args, **kwargs):
    return default().split(*args, **kwargs)


def spmv_split(*args, **kwargs):
    return default().spmv_split(*args, **kwargs)


def kpm_moments(*args, **kwargs):
    return default().kpm_moments(*args, **kwargs)


def lanczos(*args, **kwargs):
    return default().lanczos(*args, **kwargs)


def pack(*args, **kwargs):
    return default().pack(*args, **kwargs)


def send_list_symmetric(*args, **kwargs):
    return default().send_list_symmetric(*args, **kwargs)


def round_f32(*args, **kwargs):
    return default().round_f32(*args, **kwargs)


def round_bf16(*args, **kwargs):
    return default().round_bf16(*args, **kwargs)


def bf16_to_f64(*args, **kwargs):
    return default().bf16_to_f64(*args, **kwargs)


def normalized_error(c, c_ref, denom) -> np.ndarray:
    """|c - c_ref| / denom, with 0/0 := 0 and x/0 := inf for x > 0."""
    c = np.asarray(c, dtype=np.float64)
    c_ref = np.asarray(c_ref, dtype=np.float64)
    denom = np.asarray(denom, dtype=np.float64)
    diff = np.abs(c - c_ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(denom > 0, diff / np.where(denom > 0, denom, 1.0),
                     np.where(diff == 0, 0.0, np.inf))
    return e
