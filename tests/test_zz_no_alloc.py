"""spmv_lanczos_noalloc (the Lanczos loop for callers that cannot allocate)
against spmv_lanczos, through the C interface.

Both run the same kernels with the same reduction order, so their
coefficients and final vectors must agree bit for bit; the noalloc call
keeps its partial sums in the library's per-GPU scratch array.  Two calls in
a row, the second on a smaller matrix with fewer steps, check that the
shared array carries nothing over from one call to the next.  The first
call's coefficients are also checked against the oracle's plain iteration
within the bound of the Lanczos tests."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
from paper_1106_5908_amd import spmv
from workloads import gen

pytestmark = pytest.mark.gpu

NOTUNE = spmv.SPMV_FLAG_NO_TUNE_CACHE
U = 2.0 ** -53


def bound(rp, val, n, m):
    rows = np.repeat(np.arange(n), np.diff(rp))
    hinf = np.bincount(rows, weights=np.abs(val), minlength=n).max()
    nmax = int(np.diff(rp).max())
    return (np.arange(m) + 1) * (4 * (nmax + 5) + 2 * n) * U * hinf


def run_both(A, q, m, plan=None):
    """(noalloc alpha, beta, V1, V2), (spmv_lanczos alpha, beta, V1, V2) on one handle."""
    import torch

    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        if plan:
            spmv.spmv_set_plan(h, **plan)
        qd = torch.from_numpy(np.ascontiguousarray(q, dtype=np.float64)).to("cuda")
        V1, V2 = torch.empty_like(qd), torch.empty_like(qd)
        a = torch.full((m,), float("nan"), dtype=torch.float64, device="cuda")
        b = torch.full((m,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        print(f"noalloc: n={A.n_rows} m={m} plan={spmv.spmv_get_plan(h)}", flush=True)
        spmv.spmv_lanczos_noalloc(h, qd, m, V1, V2, a, b)
        torch.cuda.synchronize()
        got = (a.cpu().numpy(), b.cpu().numpy(), V1.cpu().numpy(), V2.cpu().numpy())
        W1, W2 = torch.empty_like(qd), torch.empty_like(qd)
        ra, rb = spmv.spmv_lanczos(h, qd, m, W1, W2)
        torch.cuda.synchronize()
        ref = (ra.cpu().numpy(), rb.cpu().numpy(), W1.cpu().numpy(), W2.cpu().numpy())
        return got, ref
    finally:
        spmv.spmv_destroy(h)


def test_noalloc_matches_lanczos_twice_smaller_second():
    A1, _ = gen.workload_c3(N=300_000)
    q1 = gen.uniform_vector(A1.n_rows, gen.rng_for(44, 1))
    # the diagonal-panel plan: the product runs over several prepared parts
    got, ref = run_both(A1, q1, 30, plan=dict(panels=4, tile_items=8))
    for g, r in zip(got, ref):
        assert np.array_equal(g.view(np.uint64), r.view(np.uint64))
    oa, ob = oracle.lanczos(A1.row_ptr, A1.col_idx, A1.val, q1, 30)
    tol = bound(A1.row_ptr, A1.val, A1.n_rows, 30)
    assert np.all(np.abs(got[0] - oa) <= tol) and np.all(np.abs(got[1] - ob) <= tol)

    A2, _ = gen.workload_c1()  # 4,096 rows: fewer reduction workgroups than the first call
    q2 = gen.uniform_vector(A2.n_rows, gen.rng_for(44, 2))
    got2, ref2 = run_both(A2, q2, 12)
    for g, r in zip(got2, ref2):
        assert np.array_equal(g.view(np.uint64), r.view(np.uint64))
    oa, ob = oracle.lanczos(A2.row_ptr, A2.col_idx, A2.val, q2, 12)
    tol = bound(A2.row_ptr, A2.val, A2.n_rows, 12)
    assert np.all(np.abs(got2[0] - oa) <= tol) and np.all(np.abs(got2[1] - ob) <= tol)


def test_noalloc_validation():
    import torch

    A, _ = gen.workload_c1()
    lib = spmv.load()
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        q = torch.ones(A.n_rows, dtype=torch.float64, device="cuda")
        V = torch.empty_like(q)
        ab = torch.empty(4, dtype=torch.float64, device="cuda")
        p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        hp = ctypes.c_void_p(h.ptr)
        f = lib.spmv_lanczos_noalloc
        assert f(hp, 0, p(q), p(V), p(ab), p(ab), p(ab), None) == spmv.SPMV_ERR_INVALID_ARG
        assert f(hp, 4, p(q), p(q), p(V), p(ab), p(ab), None) == spmv.SPMV_ERR_INVALID_ARG
        assert f(hp, 4, p(q), p(V), None, p(ab), p(ab), None) == spmv.SPMV_ERR_INVALID_ARG
        assert f(hp, 4, p(q), p(V), p(ab), None, p(ab), None) == spmv.SPMV_ERR_INVALID_ARG
        torch.cuda.synchronize()
    finally:
        spmv.spmv_destroy(h)
    h32 = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, prec="f32", flags=NOTUNE)
    try:
        q = torch.ones(A.n_rows, dtype=torch.float64, device="cuda")
        V1, V2 = torch.empty_like(q), torch.empty_like(q)
        ab = torch.empty(2, dtype=torch.float64, device="cuda")
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_lanczos_noalloc(h32, q, 2, V1, V2, ab, ab.clone())
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
    finally:
        spmv.spmv_destroy(h32)


def test_noalloc_sorted_block_plan():
    """The same with the product in sorted blocks: its layout is built when
    the plan is set, so the noalloc call finds it ready, and its fixed
    summation order makes the two loops agree bit for bit."""
    A, _ = gen.workload_c3(N=300_000)
    q = gen.uniform_vector(A.n_rows, gen.rng_for(44, 3))
    got, ref = run_both(A, q, 20, plan=dict(kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS, tile_items=2))
    for g, r in zip(got, ref):
        assert np.array_equal(g.view(np.uint64), r.view(np.uint64))
    oa, ob = oracle.lanczos(A.row_ptr, A.col_idx, A.val, q, 20)
    tol = bound(A.row_ptr, A.val, A.n_rows, 20)
    assert np.all(np.abs(got[0] - oa) <= tol) and np.all(np.abs(got[1] - ob) <= tol)
