"""Symmetric storage (upper triangle, Sect. 1.3.1) against the oracle applied
to the whole symmetric matrix, through the C interface.  The additions into
C are atomic and unordered, so random data is compared to the FP64 bound and
integer data bit for bit (every partial sum is an exact integer)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import FP64_TOL, assert_close, oracle_ref, to_dev
from paper_1106_5908_amd import spmv
from workloads import gen

pytestmark = pytest.mark.gpu

NOTUNE = spmv.SPMV_FLAG_NO_TUNE_CACHE


def _mats():
    return {
        "irregular": gen.irregular_symmetric(100_000, 6_000, gen.rng_for(50, 0)),
        "27pt": gen.stencil_27pt_3d(30),
        "5pt": gen.laplace_5pt_2d(200),
    }


MATS = None


def mats():
    global MATS
    if MATS is None:
        MATS = _mats()
    return MATS


def sym_run(U, x, c0=None, plan=None, base=0, runs=1):
    import torch

    h = spmv.spmv_create_sym_crs(U.row_ptr + base, U.col_idx + base, U.val, index_base=base,
                                 flags=NOTUNE)
    try:
        if plan:
            spmv.spmv_set_plan(h, **plan)
        B = to_dev(x, "f64")
        C = to_dev(np.zeros(U.n_rows) if c0 is None else c0, "f64")
        for _ in range(runs):
            spmv.spmv_run(h, B, C)
        torch.cuda.synchronize()
        return C.cpu().numpy()
    finally:
        spmv.spmv_destroy(h)


PLANS = [dict(kernel=spmv.SPMV_KERNEL_VECTOR, lanes=l, nontemporal=nt)
         for l in (2, 4, 16, 64) for nt in (0, 1)]


def _pid(p):
    return "-".join(f"{k}{v}" for k, v in p.items())


@pytest.mark.parametrize("plan", PLANS, ids=_pid)
@pytest.mark.parametrize("name", ["irregular", "27pt", "5pt"])
def test_parity(name, plan):
    A = mats()[name]
    U = gen.upper_triangle(A)
    assert U.nnz < A.nnz
    x = gen.uniform_vector(A.n_cols, gen.rng_for(51, 1))
    c0 = gen.uniform_vector(A.n_rows, gen.rng_for(51, 2))
    ref, den = oracle_ref(A, x, c0)
    assert_close(sym_run(U, x, c0, plan=plan), ref, den, FP64_TOL, f"{name} {plan}")


@pytest.mark.parametrize("base", [0, 1])
def test_integer_exact_and_accumulate(base):
    A = gen.stencil_27pt_3d(25)  # 26 / -1: integer, symmetric
    U = gen.upper_triangle(A)
    rng = gen.rng_for(52, base)
    x = gen.integer_vector(A.n_cols, rng)
    c0 = gen.integer_vector(A.n_rows, rng)
    ref = oracle.spmv(A.row_ptr, A.col_idx, A.val, x, c0)
    assert np.array_equal(sym_run(U, x, c0, base=base), ref)
    ref2 = oracle.spmv(A.row_ptr, A.col_idx, A.val, x, ref)
    assert np.array_equal(sym_run(U, x, c0, base=base, runs=2), ref2)


def test_edges():
    rng = gen.rng_for(53, 0)
    # diagonal only
    d = rng.standard_normal(500)
    D = gen.CRS(500, 500, np.arange(501, dtype=np.int32), np.arange(500, dtype=np.int32), d)
    x = gen.uniform_vector(500, rng)
    ref, den = oracle_ref(D, x)
    assert_close(sym_run(D, x), ref, den, FP64_TOL, "diagonal")
    # empty rows, a repeated upper entry (the whole matrix then holds it twice
    # on each side) and an empty matrix
    rp = np.array([0, 3, 3, 5, 5, 6], np.int32)
    col = np.array([0, 2, 2, 2, 4, 4], np.int32)
    val = np.array([1.0, 2.0, 3.0, -1.0, 5.0, 7.0])
    U = gen.CRS(5, 5, rp, col, val)
    full = np.zeros((5, 5))
    for i in range(5):
        for j in range(rp[i], rp[i + 1]):
            full[i, col[j]] += val[j]
            if col[j] != i:
                full[col[j], i] += val[j]
    x = np.array([1.0, -2.0, 0.5, 3.0, -1.5])
    assert np.allclose(sym_run(U, x), full @ x, rtol=0, atol=1e-14)
    E = gen.CRS(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert sym_run(E, np.zeros(0)).size == 0


def test_validation_and_unsupported():
    import torch

    A = mats()["5pt"]
    with pytest.raises(spmv.SpmvError) as ei:  # the full matrix has entries below the diagonal
        spmv.spmv_create_sym_crs(A.row_ptr, A.col_idx, A.val)
    assert ei.value.status == spmv.SPMV_ERR_INVALID_MATRIX and "left of the diagonal" in ei.value.message
    U = gen.upper_triangle(A)
    with pytest.raises(spmv.SpmvError) as ei:
        spmv.spmv_create_sym_crs(U.row_ptr, U.col_idx, U.val, prec="f32")
    assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
    h = spmv.spmv_create_sym_crs(U.row_ptr, U.col_idx, U.val, flags=NOTUNE)
    try:
        assert spmv.spmv_get_info(h)["kind"] == spmv.SPMV_KIND_SYMMETRIC
        for bad in (dict(kernel=spmv.SPMV_KERNEL_STREAM), dict(kernel=spmv.SPMV_KERNEL_STAGED,
                                                               tile_items=16),
                    dict(kernel=spmv.SPMV_KERNEL_VECTOR, panels=2)):
            with pytest.raises(spmv.SpmvError) as ei:
                spmv.spmv_set_plan(h, **bad)
            assert ei.value.status in (spmv.SPMV_ERR_UNSUPPORTED, spmv.SPMV_ERR_INVALID_ARG)
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_split_local_nonlocal(h, A.n_cols // 2)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        B = torch.zeros((A.n_rows, 4), dtype=torch.float64, device="cuda")
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_run_block(h, B, torch.zeros_like(B))
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        # the tuner searches lanes and keeps a vector plan
        spmv.spmv_tune(h)
        assert spmv.spmv_get_plan(h)["kernel"] == spmv.SPMV_KERNEL_VECTOR
        x = gen.uniform_vector(A.n_cols, gen.rng_for(54, 0))
        C = to_dev(np.zeros(A.n_rows), "f64")
        spmv.spmv_run(h, to_dev(x, "f64"), C)
        torch.cuda.synchronize()
        ref, den = oracle_ref(A, x)
        assert_close(C.cpu().numpy(), ref, den, FP64_TOL, "tuned symmetric")
    finally:
        spmv.spmv_destroy(h)
