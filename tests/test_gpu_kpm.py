"""Chebyshev moments (kernel polynomial method) on the GPU against the oracle's
plain recursion, through the C interface.

Bound: the GPU takes two moments per product (mu_2n = 2 v_n.v_n - mu_0,
mu_2n+1 = 2 v_n+1.v_n - mu_1) and sums in another order than the oracle.
With the spectrum scaled into [-1, 1] every v_m has norm at most |v0|, a
rounding error made at step k reaches step m amplified at most (m - k + 1)
times (Chebyshev polynomials of the second kind are bounded by their degree
on [-1, 1]), and each step rounds at most (nnz_row + 3) operations per
entry; the dot products add N roundings.  So
    |mu_gpu - mu_oracle| <= (4 M^2 (nnz_row + 3) + 2 N) u |v0|^2,
u = 2^-53, which the tests use per column.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1106_5908_amd import spmv
from workloads import gen

pytestmark = pytest.mark.gpu

NOTUNE = spmv.SPMV_FLAG_NO_TUNE_CACHE
U = 2.0 ** -53


def scaled(A):
    """A / (1.01 * max absolute row sum): spectrum inside [-1, 1] (Gershgorin)."""
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    g = np.bincount(rows, weights=np.abs(A.val), minlength=A.n_rows).max()
    return A.val / (1.01 * g)


def gpu_moments(A, val, V0, M, **kw):
    import torch

    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, val, A.n_cols, flags=NOTUNE)
    try:
        mu = spmv.spmv_kpm_moments(h, torch.from_numpy(np.ascontiguousarray(V0)).to("cuda"), M, **kw)
        torch.cuda.synchronize()
        return mu.cpu().numpy()
    finally:
        spmv.spmv_destroy(h)


def check(A, val, V0, got, M):
    ref = oracle.kpm_moments(A.row_ptr, A.col_idx, val, V0, M)
    nmax = int(np.diff(A.row_ptr).max())
    tol = (4 * M * M * (nmax + 3) + 2 * A.n_rows) * U * np.sum(V0 * V0, axis=0)
    err = np.abs(got - ref)
    assert np.all(err <= tol[None, :]), (err.max(), tol.min())
    return float((err / tol[None, :]).max())


@pytest.mark.parametrize("R", [1, 4, 8, 64])
@pytest.mark.parametrize("M", [1, 2, 3, 50])
def test_laplacian_moments(R, M):
    A, _ = gen.workload_c1()  # 5-point 64^2
    val = scaled(A)
    V0 = gen.uniform_vector(A.n_rows * R, gen.rng_for(17, R)).reshape(A.n_rows, R)
    got = gpu_moments(A, val, V0, M)
    assert got.shape == (M, R)
    check(A, val, V0, got, M)


def test_irregular_moments_and_determinism():
    import torch

    A, _ = gen.workload_c3(N=100_000)
    val = scaled(A)
    R, M = 8, 33
    V0 = gen.uniform_vector(A.n_rows * R, gen.rng_for(18, 0)).reshape(A.n_rows, R)
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, val, A.n_cols, flags=NOTUNE)
    try:
        V = torch.from_numpy(V0).to("cuda")
        m1 = spmv.spmv_kpm_moments(h, V, M).cpu().numpy()
        m2 = spmv.spmv_kpm_moments(h, V, M).cpu().numpy()
        assert np.array_equal(m1.view(np.uint64), m2.view(np.uint64))
        spmv.spmv_tune(h, R)  # a tuned block plan gives the same moments to the bound
        m3 = spmv.spmv_kpm_moments(h, V, M).cpu().numpy()
        # V0 is read only: the recursion works in W1 and W2
        assert np.array_equal(V.cpu().numpy().view(np.uint64), V0.view(np.uint64))
    finally:
        spmv.spmv_destroy(h)
    check(A, val, V0, m1, M)
    check(A, val, V0, m3, M)


@pytest.mark.parametrize("kt", [4, 8])
def test_irregular_moments_sorted_block_plan(kt):
    """The block products in sorted blocks (values scaled by +-2 as they are
    loaded): the moments to the same bound."""
    import torch

    A, _ = gen.workload_c3(N=100_000)
    val = scaled(A)
    R, M = 8, 33
    V0 = gen.uniform_vector(A.n_rows * R, gen.rng_for(18, 1)).reshape(A.n_rows, R)
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, val, A.n_cols, flags=NOTUNE)
    try:
        spmv.spmv_set_plan(h, kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS, tile_items=2, block_kt=kt)
        assert spmv.spmv_get_block_plan(h, R)["kernel"] == spmv.SPMV_KERNEL_SORTED_BLOCKS
        got = spmv.spmv_kpm_moments(h, torch.from_numpy(V0).to("cuda"), M).cpu().numpy()
    finally:
        spmv.spmv_destroy(h)
    check(A, val, V0, got, M)


def test_integer_first_moments_exact():
    """With integer data the first two moments are exact sums: mu_0 = |v0|^2,
    mu_1 = v0.A v0 (no rounding anywhere below 2^53)."""
    A = gen.random_crs(300, 300, gen.rng_for(19, 0), max_len=9, integer_values=True)
    R = 4
    V0 = gen.integer_vector(300 * R, gen.rng_for(19, 1)).reshape(300, R).astype(np.float64)
    got = gpu_moments(A, A.val, V0, 2)
    ref = oracle.kpm_moments(A.row_ptr, A.col_idx, A.val, V0, 2)
    assert np.array_equal(got, ref)


def test_validation():
    import torch

    A, _ = gen.workload_c1()
    V = torch.zeros((A.n_rows, 4), dtype=torch.float64, device="cuda")
    lib = spmv.load()
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        W1, W2 = torch.empty_like(V), torch.empty_like(V)
        mu = torch.empty((4, 4), dtype=torch.float64, device="cuda")
        p = lambda t: spmv.ctypes.c_void_p(t.data_ptr())  # noqa: E731
        hp = spmv.ctypes.c_void_p(h.ptr)
        assert lib.spmv_kpm_moments(hp, 3, 4, p(V), p(W1), p(W2), p(mu), None) == spmv.SPMV_ERR_INVALID_ARG
        assert lib.spmv_kpm_moments(hp, 128, 4, p(V), p(W1), p(W2), p(mu), None) == spmv.SPMV_ERR_INVALID_ARG
        assert lib.spmv_kpm_moments(hp, 4, 0, p(V), p(W1), p(W2), p(mu), None) == spmv.SPMV_ERR_INVALID_ARG
        assert lib.spmv_kpm_moments(hp, 4, 4, p(V), p(V), p(W2), p(mu), None) == spmv.SPMV_ERR_INVALID_ARG
        assert lib.spmv_kpm_moments(hp, 4, 4, p(V), p(W1), p(W2), None, None) == spmv.SPMV_ERR_INVALID_ARG
        torch.cuda.synchronize()
    finally:
        spmv.spmv_destroy(h)
    h32 = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, prec="f32", flags=NOTUNE)
    try:
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_kpm_moments(h32, V, 4)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
    finally:
        spmv.spmv_destroy(h32)
    R = gen.random_crs(20, 30, gen.rng_for(19, 2), max_len=4)
    hr = spmv.spmv_create_crs(R.row_ptr, R.col_idx, R.val, R.n_cols, flags=NOTUNE)
    try:
        st = lib.spmv_kpm_moments(spmv.ctypes.c_void_p(hr.ptr), 1, 2, None, None, None,
                                  spmv.ctypes.c_void_p(V.data_ptr()), None)
        assert st == spmv.SPMV_ERR_INVALID_ARG and "square" in spmv.spmv_last_error()
    finally:
        spmv.spmv_destroy(hr)
