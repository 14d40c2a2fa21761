"""Lanczos on the GPU against the oracle's plain iteration, through the C
interface.

Bound: both run the same recursion with different summation orders.  Before a
Ritz value converges the three-term recursion is forward stable, so the
coefficients differ by a few roundings of the quantities involved; the tests
allow (j + 1) (4 (n_row + 5) + 2 N) u |H|_inf for step j (u = 2^-53, |H|_inf the
largest absolute row sum), checked for as many steps as stay before
convergence on each matrix.  Exactly representable cases are compared bit for
bit."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1106_5908_amd import spmv
from workloads import gen

pytestmark = pytest.mark.gpu

NOTUNE = spmv.SPMV_FLAG_NO_TUNE_CACHE
U = 2.0 ** -53


def gpu_lanczos(rp, ci, val, n_cols, q, m, tune=False):
    import torch

    h = spmv.spmv_create_crs(rp, ci, val, n_cols, flags=NOTUNE)
    try:
        if tune:
            spmv.spmv_tune(h, 1)
        a, b = spmv.spmv_lanczos(h, torch.from_numpy(np.ascontiguousarray(q, dtype=np.float64)).to("cuda"), m)
        torch.cuda.synchronize()
        return a.cpu().numpy(), b.cpu().numpy()
    finally:
        spmv.spmv_destroy(h)


def bound(rp, val, n, m):
    rows = np.repeat(np.arange(n), np.diff(rp))
    hinf = np.bincount(rows, weights=np.abs(val), minlength=n).max()
    nmax = int(np.diff(rp).max())
    return (np.arange(m) + 1) * (4 * (nmax + 5) + 2 * n) * U * hinf


def test_tridiagonal_is_its_own_lanczos_matrix():
    n = 5000
    rp, ci, vv = [0], [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                ci.append(j)
                vv.append(v)
        rp.append(len(ci))
    q = np.zeros(n)
    q[0] = 0.5
    a, b = gpu_lanczos(np.array(rp, np.int32), np.array(ci, np.int32), np.array(vv), n, q, 40)
    assert a.tolist() == [2.0] * 40 and b.tolist() == [1.0] * 40


@pytest.mark.parametrize("name,m", [("laplace64", 30), ("irregular", 25), ("27pt", 25)])
def test_coefficients_match_oracle(name, m):
    if name == "laplace64":
        A, _ = gen.workload_c1()
    elif name == "irregular":
        A, _ = gen.workload_c3(N=100_000)
    else:
        A, _ = gen.workload_c2(n=30)
        # symmetrise the perturbed stencil's values: (A + A^T) / 2 has the same structure
        import scipy.sparse as sp
        M = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_cols))
        M = ((M + M.T) * 0.5).tocsr()
        M.sort_indices()
        A.row_ptr, A.col_idx, A.val = M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data
    q = gen.uniform_vector(A.n_rows, gen.rng_for(41, m))
    a, b = gpu_lanczos(A.row_ptr, A.col_idx, A.val, A.n_cols, q, m)
    ra, rb = oracle.lanczos(A.row_ptr, A.col_idx, A.val, q, m)
    tol = bound(A.row_ptr, A.val, A.n_rows, m)
    assert np.all(np.abs(a - ra) <= tol), (np.abs(a - ra) / tol).max()
    assert np.all(np.abs(b - rb) <= tol), (np.abs(b - rb) / tol).max()


def test_deterministic_and_tuned_plan():
    A, _ = gen.workload_c3(N=100_000)
    q = gen.uniform_vector(A.n_rows, gen.rng_for(42, 0))
    a1, b1 = gpu_lanczos(A.row_ptr, A.col_idx, A.val, A.n_cols, q, 20)
    a2, b2 = gpu_lanczos(A.row_ptr, A.col_idx, A.val, A.n_cols, q, 20)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    a3, b3 = gpu_lanczos(A.row_ptr, A.col_idx, A.val, A.n_cols, q, 20, tune=True)
    ra, rb = oracle.lanczos(A.row_ptr, A.col_idx, A.val, q, 20)
    tol = bound(A.row_ptr, A.val, A.n_rows, 20)
    assert np.all(np.abs(a3 - ra) <= tol) and np.all(np.abs(b3 - rb) <= tol)


def test_invariant_subspace_terminates():
    """q in the span of 3 sine modes of the 64 x 64 Laplacian: beta_3 vanishes
    (to rounding) and the 3 x 3 Lanczos matrix has exactly those eigenvalues;
    q = 0 gives zeros throughout."""
    A, _ = gen.workload_c1()
    n = 64
    idx = np.arange(1, n + 1)
    S = np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(idx, idx) / (n + 1))
    lam = 2.0 - 2.0 * np.cos(idx * np.pi / (n + 1))
    modes = [(1, 1), (5, 9), (40, 2)]
    q = sum((t + 1.0) * np.outer(S[ky - 1], S[jx - 1]).reshape(-1) for t, (jx, ky) in enumerate(modes))
    a, b = gpu_lanczos(A.row_ptr, A.col_idx, A.val, A.n_cols, q, 3)
    assert abs(b[2]) <= 1e-12 * 8
    T = np.diag(a) + np.diag(b[:2], 1) + np.diag(b[:2], -1)
    assert np.allclose(np.linalg.eigvalsh(T), sorted(lam[jx - 1] + lam[ky - 1] for jx, ky in modes),
                       rtol=0, atol=1e-12)
    a0, b0 = gpu_lanczos(A.row_ptr, A.col_idx, A.val, A.n_cols, np.zeros(A.n_rows), 4)
    assert not a0.any() and not b0.any()


def test_validation():
    import torch

    A, _ = gen.workload_c1()
    lib = spmv.load()
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        q = torch.ones(A.n_rows, dtype=torch.float64, device="cuda")
        V = torch.empty_like(q)
        ab = torch.empty(4, dtype=torch.float64, device="cuda")
        p = lambda t: spmv.ctypes.c_void_p(t.data_ptr())  # noqa: E731
        hp = spmv.ctypes.c_void_p(h.ptr)
        assert lib.spmv_lanczos(hp, 0, p(q), p(V), p(ab), p(ab), p(ab), None) == spmv.SPMV_ERR_INVALID_ARG
        assert lib.spmv_lanczos(hp, 4, p(q), p(q), p(V), p(ab), p(ab), None) == spmv.SPMV_ERR_INVALID_ARG
        assert lib.spmv_lanczos(hp, 4, p(q), p(V), None, p(ab), p(ab), None) == spmv.SPMV_ERR_INVALID_ARG
        assert lib.spmv_lanczos(hp, 4, p(q), p(V), p(ab), None, p(ab), None) == spmv.SPMV_ERR_INVALID_ARG
        torch.cuda.synchronize()
    finally:
        spmv.spmv_destroy(h)
    h32 = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, prec="f32", flags=NOTUNE)
    try:
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_lanczos(h32, torch.ones(A.n_rows, dtype=torch.float64, device="cuda"), 2)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
    finally:
        spmv.spmv_destroy(h32)
