"""Invariants of the seeded input generators (host only)."""
import numpy as np

from workloads import gen


def _check_crs(A):
    rp = A.row_ptr.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == A.col_idx.size == A.val.size
    assert np.all(np.diff(rp) >= 0)
    if A.col_idx.size:
        assert A.col_idx.min() >= 0 and A.col_idx.max() < A.n_cols
    assert A.row_ptr.dtype == np.int32 and A.col_idx.dtype == np.int32 and A.val.dtype == np.float64


def test_c1_counts():
    A, x = gen.workload_c1()
    _check_crs(A)
    assert (A.n_rows, A.nnz) == (4096, 20224)  # 5*4096 - 4*64
    assert np.all(np.abs(x) <= 1) and x.size == 4096
    # deterministic
    A2, x2 = gen.workload_c1()
    assert np.array_equal(x, x2) and np.array_equal(A.col_idx, A2.col_idx)


def test_27pt_counts_and_perturbation():
    for n in (3, 5, 12):
        A = gen.stencil_27pt_3d(n)
        _check_crs(A)
        assert A.nnz == (3 * n - 2) ** 3
        assert np.all(np.diff(A.col_idx[A.row_ptr[0]:A.row_ptr[1]]) > 0)
    # full size formula for the 160^3 bandwidth case
    assert (3 * 160 - 2) ** 3 == 109_215_352
    A, x = gen.workload_c2(n=10)
    _check_crs(A)
    diag = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr)) == A.col_idx
    assert np.all(np.abs(A.val[diag] - 26) <= 0.01) and np.all(np.abs(A.val[~diag] + 1) <= 0.01)
    assert np.any(A.val[~diag] != -1)


def test_7pt_counts():
    for n in (2, 4, 9):
        A = gen.laplace_7pt_3d(n)
        _check_crs(A)
        assert A.nnz == 7 * n ** 3 - 6 * n ** 2


def test_irregular_symmetric():
    A, x = gen.workload_c3(N=100_000)
    _check_crs(A)
    st = A.stats()
    assert 12.0 <= st["mean"] <= 14.0 and st["max"] <= 64
    # exact symmetry: A == A^T, including values
    import scipy.sparse as sp
    M = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n_rows, A.n_cols))
    D = M - M.T
    assert D.count_nonzero() == 0
    # band: |i - j| <= N/16, diagonal present in every row
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    assert np.all(np.abs(rows - A.col_idx) <= A.n_rows // 16)
    assert np.all(M.diagonal() != 0)
    # sorted, unique columns per row
    d = np.diff(A.col_idx.astype(np.int64))
    starts = A.row_ptr[1:-1]
    mask = np.ones(d.size, bool)
    mask[starts[starts < d.size + 1] - 1] = False
    assert np.all(d[mask] > 0)


def test_halo_begin():
    assert gen.halo_begin(8_000_000) == 7_520_000
    assert gen.halo_begin(100) == 94


def test_batch_sizes_and_stencils():
    sizes, kinds = gen.batch_sizes()
    assert sizes.size == 512 and sizes.min() >= 1000 and sizes.max() <= 250_000
    assert 0.4 < kinds.mean() < 0.6
    for n, three_d in ((1000, False), (1000, True), (4097, True), (7777, False)):
        A = gen.truncated_stencil(n, three_d)
        _check_crs(A)
        assert A.n_rows == n
        rl = np.diff(A.row_ptr)
        assert rl.max() == (7 if three_d else 5)


def test_random_crs_edge_features():
    rng = gen.rng_for(99, 0)
    A = gen.random_crs(50, 20, rng, max_len=8)
    _check_crs(A)
    rl = np.diff(A.row_ptr)
    assert (rl == 0).any()
    dup = any(len(set(A.col_idx[a:b])) < b - a for a, b in zip(A.row_ptr[:-1], A.row_ptr[1:]))
    assert dup


def test_upper_triangle_expands_to_the_symmetric_matrix():
    """U + U^T - diag(U) rebuilt densely equals the symmetric input."""
    A = gen.irregular_symmetric(300, 40, gen.rng_for(55, 0))
    U = gen.upper_triangle(A)
    full = np.zeros((A.n_rows, A.n_cols))
    for i in range(A.n_rows):
        for j in range(A.row_ptr[i], A.row_ptr[i + 1]):
            full[i, A.col_idx[j]] += A.val[j]
    assert np.array_equal(full, full.T)
    rebuilt = np.zeros_like(full)
    for i in range(U.n_rows):
        for j in range(U.row_ptr[i], U.row_ptr[i + 1]):
            c = U.col_idx[j]
            assert c >= i
            rebuilt[i, c] += U.val[j]
            if c != i:
                rebuilt[c, i] += U.val[j]
    assert np.array_equal(rebuilt, full)
