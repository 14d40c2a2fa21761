"""Parity at the benchmark sizes, in the launch configuration the benchmark
times (plans picked by the autotuner): every output entry is compared with
the oracle, except for the block products, where 2000 sampled rows are
recomputed one by one."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import FP64_TOL, assert_close, prec_bounds, rounded_inputs, to_dev
from paper_1106_5908_amd import spmv
from workloads import gen

pytestmark = pytest.mark.gpu

NOTUNE = spmv.SPMV_FLAG_NO_TUNE_CACHE


@pytest.fixture(scope="module")
def c2():
    A, x = gen.workload_c2()
    ref = oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
    den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, x)
    return A, x, ref, den


@pytest.fixture(scope="module")
def c3():
    A, x = gen.workload_c3()
    ref = oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
    den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, x)
    return A, x, ref, den


def _tuned_run(A, x, prec="f64", runs=1):
    import torch

    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, prec=prec, flags=NOTUNE)
    try:
        spmv.spmv_tune(h, 1)
        plan = spmv.spmv_get_plan(h)
        B = to_dev(x, prec)
        C = torch.zeros(A.n_rows, dtype=B.dtype, device="cuda")
        for _ in range(runs):
            spmv.spmv_run(h, B, C)
        torch.cuda.synchronize()
        return C.cpu().numpy().astype(np.float64), plan
    finally:
        spmv.spmv_destroy(h)


def test_27pt160_fp64(c2):
    A, x, ref, den = c2
    got, plan = _tuned_run(A, x)
    assert_close(got, ref, den, FP64_TOL, f"27-point 160^3 FP64, plan {plan}")


@pytest.mark.parametrize("plan", [dict(kernel=spmv.SPMV_KERNEL_STAGED, tile_items=16),
                                  dict(kernel=spmv.SPMV_KERNEL_STREAM, tile_items=16)],
                         ids=["staged16", "stream16"])
def test_27pt160_fp64_fixed_plans(c2, plan):
    """The two kernels the tuner chooses between on this matrix, each at the
    full size whatever the tuner picks; the staged one must stage nearly
    every tile."""
    import torch

    A, x, ref, den = c2
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        spmv.spmv_set_plan(h, **plan)
        info = spmv.spmv_get_info(h)
        if plan["kernel"] == spmv.SPMV_KERNEL_STAGED:
            assert info["n_staged_tiles"] > 0.99 * info["n_tiles"], info
        B = to_dev(x, "f64")
        C = torch.zeros(A.n_rows, dtype=B.dtype, device="cuda")
        spmv.spmv_run(h, B, C)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
    finally:
        spmv.spmv_destroy(h)
    assert_close(got, ref, den, FP64_TOL, f"27-point 160^3 FP64, plan {plan}")


def test_27pt160_integer_bit_exact():
    A = gen.stencil_27pt_3d(160)
    x = gen.integer_vector(A.n_cols, gen.rng_for(2, 9), vmax=8)
    got, _ = _tuned_run(A, x, runs=2)
    assert np.array_equal(got, 2 * oracle.spmv(A.row_ptr, A.col_idx, A.val, x))


def test_irregular8M_fp64(c3):
    A, x, ref, den = c3
    got, plan = _tuned_run(A, x)
    assert_close(got, ref, den, FP64_TOL, f"irregular 8M FP64, plan {plan}")


@pytest.mark.parametrize("items", [1, 2, 4])
def test_irregular8M_sorted_blocks(c3, items):
    """The sorted-block kernel at the full size whatever the tuner picks:
    every row against the oracle, the same bits on two calls, and a layout
    of about one slot per entry."""
    import torch

    A, x, ref, den = c3
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        spmv.spmv_set_plan(h, kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS, tile_items=items)
        chunks = spmv.spmv_get_info(h)["n_tiles"]
        assert A.nnz <= chunks * 1024 * items <= 1.05 * A.nnz + 512 * 1024 * items, chunks
        B = to_dev(x, "f64")
        C1 = torch.zeros(A.n_rows, dtype=B.dtype, device="cuda")
        C2 = torch.zeros_like(C1)
        spmv.spmv_run(h, B, C1)
        spmv.spmv_run(h, B, C2)
        torch.cuda.synchronize()
        assert torch.equal(C1, C2)
        got = C1.cpu().numpy()
    finally:
        spmv.spmv_destroy(h)
    assert_close(got, ref, den, FP64_TOL, f"irregular 8M FP64, sorted blocks, {items} per lane")


@pytest.mark.parametrize("prec", ["f32", "bf16", "f32f64"])
@pytest.mark.parametrize("which", ["27pt160", "irregular8M"])
def test_precision_modes_fullsize(prec, which, c2, c3):
    A, x, ref, den = c2 if which == "27pt160" else c3
    got, plan = _tuned_run(A, x, prec)
    b_orig, b_same = prec_bounds(prec, int(np.diff(A.row_ptr).max()))
    assert_close(got, ref, den, b_orig, f"{which} {prec} vs FP64 oracle, plan {plan}")
    rows = np.random.default_rng(3).integers(0, A.n_rows, size=20000)
    v, xr = rounded_inputs(A, x, prec)
    ref2 = oracle.spmv_rows(rows, A.row_ptr, A.col_idx, v, xr)
    den2 = oracle.spmv_rows(rows, A.row_ptr, A.col_idx, np.abs(v), np.abs(xr))
    assert_close(got[rows], ref2, den2, b_same, f"{which} {prec} vs oracle on rounded inputs")


def test_irregular8M_split_overlap(c3):
    import torch

    A, x, ref, den = c3
    hb = gen.halo_begin(A.n_cols)
    a = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    s = spmv.spmv_split_local_nonlocal(a, hb)
    try:
        spmv.spmv_tune(s, 1)
        halo = torch.from_numpy(np.ascontiguousarray(x[hb:])).pin_memory()
        Bh = x.copy()
        Bh[hb:] = np.nan
        B = to_dev(Bh, "f64")
        C = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
        spmv.spmv_run(s, B, C, halo)
        torch.cuda.synchronize()
        assert_close(C.cpu().numpy(), ref, den, FP64_TOL,
                     f"split with overlapped halo copy, local plan {spmv.spmv_get_plan(s)}")
        # the local part in sorted blocks, whatever the tuner picked
        spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS,
                           tile_items=2)
        B = to_dev(Bh, "f64")
        C.zero_()
        spmv.spmv_run(s, B, C, halo)
        torch.cuda.synchronize()
        assert_close(C.cpu().numpy(), ref, den, FP64_TOL, "split, local part in sorted blocks")
        # every schedule with the sorted local plan; the merged one here
        # runs its last blocks as one launch after whole rounds (256 blocks
        # of the local layout precede the first nonlocal row)
        spmv.spmv_set_phase_timing(s, True)
        for sch in (spmv.SPMV_SCHEDULE_OVERLAP_MERGED, spmv.SPMV_SCHEDULE_OVERLAP_NONLOCAL,
                    spmv.SPMV_SCHEDULE_SERIAL, spmv.SPMV_SCHEDULE_OVERLAP):
            spmv.spmv_set_schedule(s, sch)
            for with_copy in (True, False):
                B = to_dev(Bh if with_copy else x, "f64")
                C.zero_()
                spmv.spmv_run(s, B, C, halo if with_copy else None)
                torch.cuda.synchronize()
                assert_close(C.cpu().numpy(), ref, den, FP64_TOL,
                             f"split, sorted local plan, schedule {sch}, copy {with_copy}")
                t = spmv.spmv_phase_times(s)
                if with_copy and sch == spmv.SPMV_SCHEDULE_OVERLAP_MERGED:
                    assert t["copy"][1] <= t["nonlocal"][0] + 0.01
                    assert t["local"][0] <= t["nonlocal"][0] and t["nonlocal"][1] <= t["local"][1] + 0.01
        spmv.spmv_set_phase_timing(s, False)
        info = spmv.spmv_get_info(s)
        parts = oracle.split(A.row_ptr, A.col_idx, A.val, hb)
        assert info["nnz_nonlocal"] == parts["nl_col"].size
        assert info["n_nonlocal_rows"] == parts["nl_rows"].size
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


def test_irregular8M_exchange(c3):
    """The full exchange cycle at the benchmark size: symmetric send list and
    send buffer bit for bit, C to the FP64 bound."""
    import torch

    A, x, ref, den = c3
    hb = gen.halo_begin(A.n_cols)
    a = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    s = spmv.spmv_split_local_nonlocal(a, hb)
    try:
        spmv.spmv_tune(s, 1)
        n = spmv.spmv_send_list_symmetric(s)
        want = oracle.send_list_symmetric(A.row_ptr, A.col_idx, hb)
        assert np.array_equal(spmv.spmv_export(s, spmv.SPMV_ARR_SEND_IDX), want)
        halo = torch.from_numpy(np.ascontiguousarray(x[hb:])).pin_memory()
        send = torch.full((n,), float("nan"), dtype=torch.float64).pin_memory()
        Bh = x.copy()
        Bh[hb:] = np.nan
        B = to_dev(Bh, "f64")
        C = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
        spmv.spmv_run_exchange(s, B, C, halo, send)
        torch.cuda.synchronize()
        assert np.array_equal(send.numpy().view(np.uint64), oracle.pack(want, x).view(np.uint64))
        assert_close(C.cpu().numpy(), ref, den, FP64_TOL, "exchange cycle, 8M rows")
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


def test_irregular8M_kpm_moments(c3):
    """Chebyshev moments at the benchmark size (two start vectors, four
    moments; the oracle runs the plain recursion) to the bound derived in
    test_gpu_kpm.py."""
    import torch

    A = c3[0]
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    g = np.bincount(rows, weights=np.abs(A.val), minlength=A.n_rows).max()
    val = A.val / (1.01 * g)
    R, M = 2, 4
    V0 = gen.uniform_vector(A.n_rows * R, gen.rng_for(31, 0)).reshape(A.n_rows, R)
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, val, A.n_cols, flags=NOTUNE)
    try:
        spmv.spmv_tune(h, R)
        mu = spmv.spmv_kpm_moments(h, torch.from_numpy(V0).to("cuda"), M).cpu().numpy()
    finally:
        spmv.spmv_destroy(h)
    ref = oracle.kpm_moments(A.row_ptr, A.col_idx, val, V0, M)
    nmax = int(np.diff(A.row_ptr).max())
    tol = (4 * M * M * (nmax + 3) + 2 * A.n_rows) * 2.0 ** -53 * np.sum(V0 * V0, axis=0)
    assert np.all(np.abs(mu - ref) <= tol[None, :]), np.abs(mu - ref).max()


BLOCK_FIXED = {4: dict(kernel=5, panels=8, xcd_remap=0, block_kt=4),
               8: dict(kernel=5, panels=4, xcd_remap=0, block_kt=8),
               16: dict(kernel=5, panels=1, xcd_remap=0, block_kt=16)}


@pytest.mark.parametrize("plan", ["tuned", "fixed"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("k", [4, 8, 16])
def test_block_irregular8M_sampled(k, prec, plan, c3):
    """Block products at full size, with the tuner's plan and with the
    fused-panel plans the tuner picked on the MI355X (fused panels, XCD remap
    off), 2000 sampled rows against the oracle."""
    import torch

    A, _, _, _ = c3
    X = gen.block_rhs(A.n_cols, k)
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, prec=prec, flags=NOTUNE)
    try:
        if plan == "tuned":
            spmv.spmv_tune(h, k)
        else:
            spmv.spmv_set_plan(h, **BLOCK_FIXED[k])
        dt = torch.float64 if prec == "f64" else torch.float32
        B = torch.from_numpy(X).to("cuda", dtype=dt)
        C = torch.zeros((A.n_rows, k), dtype=dt, device="cuda")
        spmv.spmv_run_block(h, B, C)
        torch.cuda.synchronize()
        rows = np.random.default_rng(11).integers(0, A.n_rows, size=2000)
        got = C[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    finally:
        spmv.spmv_destroy(h)
    b_orig, _ = prec_bounds(prec, int(np.diff(A.row_ptr).max()))
    for t in range(k):
        xt = np.ascontiguousarray(X[:, t])
        ref = oracle.spmv_rows(rows, A.row_ptr, A.col_idx, A.val, xt)
        den = oracle.spmv_rows(rows, A.row_ptr, A.col_idx, np.abs(A.val), np.abs(xt))
        assert_close(got[:, t], ref, den, b_orig, f"block k={k} {prec} column {t}")


def test_batch_512_stencils():
    import torch

    mem = gen.workload_c5_batch()
    h = spmv.spmv_create_batch([(A.row_ptr, A.col_idx, A.val, A.n_cols) for A, _ in mem], flags=NOTUNE)
    try:
        spmv.spmv_tune(h, 1)
        B = to_dev(np.concatenate([x for _, x in mem]), "f64")
        C = torch.zeros(sum(A.n_rows for A, _ in mem), dtype=torch.float64, device="cuda")
        spmv.spmv_run(h, B, C)  # HIP-graph replay path
        torch.cuda.synchronize()
        got = C.cpu().numpy()
    finally:
        spmv.spmv_destroy(h)
    off = 0
    for m, (A, x) in enumerate(mem):
        sl = slice(off, off + A.n_rows)
        ref = oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
        den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, x)
        assert_close(got[sl], ref, den, FP64_TOL, f"batch member {m}")
        off += A.n_rows
