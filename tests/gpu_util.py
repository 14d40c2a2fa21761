"""Helpers of the GPU parity tests: run the library through its binding and
compare with the oracle."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1106_5908_amd import spmv

U64 = 2.0 ** -53
U32 = 2.0 ** -24
U16 = 2.0 ** -8  # bfloat16 unit roundoff (8 significant bits)

FP64_TOL = 1e-12  # normalised componentwise error bound for FP64 parity


def torch_dtype(prec: str):
    import torch

    return torch.float64 if spmv.VEC_DTYPE[prec] == "float64" else torch.float32


def np_vec_dtype(prec: str):
    return np.float64 if spmv.VEC_DTYPE[prec] == "float64" else np.float32


def to_dev(a, prec: str):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np_vec_dtype(prec))).to("cuda")


def gpu_spmv(A, x, c0=None, prec="f64", plan=None, base=0, flags=spmv.SPMV_FLAG_NO_TUNE_CACHE,
             runs=1):
    """C0 + runs * (A x) computed by the library (one handle, `runs` calls)."""
    import torch

    h = spmv.spmv_create_crs(A.row_ptr + base, A.col_idx + base, A.val, A.n_cols,
                             index_base=base, prec=prec, flags=flags)
    try:
        if plan:
            spmv.spmv_set_plan(h, **plan)
        B = to_dev(x, prec)
        C = to_dev(np.zeros(A.n_rows) if c0 is None else c0, prec)
        for _ in range(runs):
            spmv.spmv_run(h, B, C)
        torch.cuda.synchronize()
        return C.cpu().numpy().astype(np.float64)
    finally:
        spmv.spmv_destroy(h)


def oracle_ref(A, x, c0=None):
    ref = oracle.spmv(A.row_ptr, A.col_idx, A.val, x, c0)
    den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, x, c0)
    return ref, den


def assert_close(got, ref, den, tol, what=""):
    e = oracle.normalized_error(got, ref, den)
    worst = int(np.argmax(e)) if e.size else -1
    assert e.size == 0 or e.max() <= tol, (
        f"{what}: max normalised error {e.max():.3e} > {tol:.1e} at row {worst} "
        f"(got {got[worst]!r}, oracle {ref[worst]!r})")
    return float(e.max()) if e.size else 0.0


def rounded_inputs(A, x, prec):
    """val and x as the library sees them, widened exactly to FP64."""
    if prec == "f64":
        return A.val, x
    if prec == "bf16":
        v = oracle.bf16_to_f64(oracle.round_bf16(A.val))
    else:
        v = oracle.round_f32(A.val).astype(np.float64)
    xr = x if spmv.VEC_DTYPE[prec] == "float64" else oracle.round_f32(x).astype(np.float64)
    return v, xr


def prec_bounds(prec, n):
    """(bound vs the FP64 oracle on the original inputs, bound vs the oracle
    on the rounded inputs) for rows of at most n entries plus C0 (normalised,
    first order, with a 10% margin)."""
    if prec == "f64":
        return FP64_TOL, FP64_TOL
    if prec == "f32":
        return 1.1 * (n + 3) * U32, 1.1 * (n + 2) * U32
    if prec == "bf16":
        return 1.1 * (U16 + (n + 3) * U32), 1.1 * (n + 2) * U32
    return 1.1 * (U32 + (n + 2) * U64), max(1.1 * (n + 2) * U64, 1e-15)
