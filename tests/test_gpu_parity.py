"""GPU path against the oracle, element by element, through the C interface.

Sizes here keep the oracle to seconds while spanning many tiles and a ragged
tail; the benchmark sizes are covered in test_gpu_fullsize.py."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import (FP64_TOL, assert_close, gpu_spmv, oracle_ref, prec_bounds, rounded_inputs,
                      to_dev, torch_dtype)
from paper_1106_5908_amd import spmv
from workloads import gen

pytestmark = pytest.mark.gpu

NOTUNE = spmv.SPMV_FLAG_NO_TUNE_CACHE


def _matrices():
    A27, x27 = gen.workload_c2(n=30)          # 27000 rows, 27-point, perturbed
    A3, x3 = gen.workload_c3(N=100_000)       # irregular symmetric
    return {"27pt": (A27, x27), "irregular": (A3, x3)}


MATS = None


def mats():
    global MATS
    if MATS is None:
        MATS = _matrices()
    return MATS


PLANS = ([dict(kernel=1, tile_items=e, nontemporal=nt, xcd_remap=rm)
          for e in (4, 8, 16) for nt in (0, 1) for rm in (0, 1)] +
         [dict(kernel=1, tile_items=e, tiles_per_group=tpw)
          for e in (4, 8, 16) for tpw in (2, 7, 32)] +
         [dict(kernel=1, tile_items=e, panels=k, xcd_remap=rm)
          for e in (4, 8) for k in (2, 4, 8) for rm in (0, 1)] +
         [dict(kernel=1, tile_items=8, panels=4, tiles_per_group=4)] +
         [dict(kernel=2, lanes=l) for l in (2, 4, 8, 16, 32, 64)] +
         [dict(kernel=4, tile_items=e, nontemporal=nt) for e in (8, 16) for nt in (0, 1)] +
         [dict(kernel=5, tile_items=e, panels=k, xcd_remap=rm)
          for e in (4, 8, 16) for k in (1, 2, 4, 8) for rm in (0, 1)] +
         [dict(kernel=5, tile_items=8, panels=4, nontemporal=0)] +
         [dict(kernel=6, tile_items=e, xcd_remap=rm) for e in (1, 2, 4) for rm in (0, 1)] +
         [dict(kernel=6, tile_items=2, nontemporal=0)])


def _sorted_refused(A, items, prec="f64"):
    """Whether the sorted-block layout refuses A: its slots, at least
    max(ceil(m / Q), longest row) chunks of Q per block of R rows, would
    exceed four per entry plus one chunk per block plus 2^20."""
    R = 16384 if prec in ("f64", "f32f64") else 32768
    Q = 1024 * items
    lens = np.diff(A.row_ptr).astype(np.int64)
    bound, nb = 0, 0
    for r0 in range(0, A.n_rows, R):
        seg = lens[r0:r0 + R]
        bound += max(-(-int(seg.sum()) // Q), int(seg.max()) if seg.size else 0) * Q
        nb += 1
    return bound > 4 * int(lens.sum()) + nb * Q + (1 << 20)


def _pid(p):
    return "-".join(f"{k}{v}" for k, v in p.items())


# ---------------------------------------------------------------------------- a3

def test_small_laplacian():
    A, x = gen.workload_c1()
    ref, den = oracle_ref(A, x)
    got = gpu_spmv(A, x)
    assert_close(got, ref, den, FP64_TOL, "2D 5-point 64x64")
    xi = gen.integer_vector(A.n_cols, gen.rng_for(1, 9))
    assert np.array_equal(gpu_spmv(A, xi), oracle.spmv(A.row_ptr, A.col_idx, A.val, xi))


@pytest.mark.parametrize("plan", PLANS, ids=_pid)
@pytest.mark.parametrize("name", ["27pt", "irregular"])
def test_plans(name, plan):
    A, x = mats()[name]
    c0 = gen.uniform_vector(A.n_rows, gen.rng_for(7, 2))
    ref, den = oracle_ref(A, x, c0)
    got = gpu_spmv(A, x, c0, plan=plan)
    assert_close(got, ref, den, FP64_TOL, f"{name} {plan}")


@pytest.mark.parametrize("plan", PLANS, ids=_pid)
def test_integer_inputs_bit_exact(plan):
    rng = gen.rng_for(8, 0)
    A = gen.random_crs(5000, 4000, rng, max_len=40, integer_values=True)
    x = gen.integer_vector(A.n_cols, rng)
    c0 = gen.integer_vector(A.n_rows, rng)
    got = gpu_spmv(A, x, c0, plan=plan)
    assert np.array_equal(got, oracle.spmv(A.row_ptr, A.col_idx, A.val, x, c0))


def _long_row_matrix(long_len, n_short=300, n_cols=20000, seed=3):
    rng = gen.rng_for(10, seed)
    counts = np.concatenate([rng.integers(0, 30, size=n_short // 2), [long_len],
                             rng.integers(0, 30, size=n_short - n_short // 2)])
    cols = rng.integers(0, n_cols, size=int(counts.sum()))
    vals = rng.standard_normal(cols.size)
    return gen._finish(counts.size, n_cols, counts, cols, vals)


@pytest.mark.parametrize("long_len", [1021, 1022, 1023, 1024, 1025, 2046, 2047, 2048, 2049, 4094, 4095, 4096, 4097, 50_000])
@pytest.mark.parametrize("plan", [dict(kernel=1, tile_items=e) for e in (4, 8, 16)] +
                         [dict(kernel=1, tile_items=e, tiles_per_group=t) for e in (4, 8)
                          for t in (3, 16)] +
                         [dict(kernel=1, tile_items=8, panels=k) for k in (2, 8)] +
                         [dict(kernel=2, lanes=64)] +
                         [dict(kernel=4, tile_items=e) for e in (8, 16)] +
                         [dict(kernel=5, tile_items=e, panels=k) for e in (4, 16) for k in (1, 4)] +
                         [dict(kernel=6, tile_items=e) for e in (1, 4)],
                         ids=_pid)
def test_long_rows(long_len, plan):
    A = _long_row_matrix(long_len)
    x = gen.uniform_vector(A.n_cols, gen.rng_for(10, 5))
    ref, den = oracle_ref(A, x)
    if plan["kernel"] == 6 and _sorted_refused(A, plan["tile_items"]):
        with pytest.raises(spmv.SpmvError) as ei:
            gpu_spmv(A, x, plan=plan)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        return
    assert_close(gpu_spmv(A, x, plan=plan), ref, den, FP64_TOL, f"long row {long_len}")


def test_edge_shapes():
    rng = gen.rng_for(11, 0)
    import torch
    # no rows
    A = gen.CRS(0, 5, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert gpu_spmv(A, np.ones(5)).size == 0
    # no columns: every row empty, C untouched (signs of zero included)
    c0 = np.array([1.5, -0.0, 0.0, -2.0])
    A = gen.CRS(4, 0, np.zeros(5, np.int32), np.zeros(0, np.int32), np.zeros(0))
    got = gpu_spmv(A, np.zeros(0), c0)
    assert np.array_equal(got, c0) and np.array_equal(np.signbit(got), np.signbit(c0))
    # rectangular, both ways, with empty rows, duplicates and unsorted columns
    for (m, n) in ((1000, 3000), (3000, 10), (1, 70000), (70000, 1)):
        A = gen.random_crs(m, n, rng, max_len=12)
        x = gen.uniform_vector(n, rng)
        c0 = gen.uniform_vector(m, rng)
        ref, den = oracle_ref(A, x, c0)
        assert_close(gpu_spmv(A, x, c0), ref, den, FP64_TOL, f"{m}x{n}")
    # diagonal panels on rectangular shapes and an empty matrix
    for (m, n) in ((1000, 3000), (3000, 10), (0, 5)):
        A = gen.random_crs(m, n, rng, max_len=12)
        x = gen.uniform_vector(n, rng)
        c0 = gen.uniform_vector(m, rng)
        ref, den = oracle_ref(A, x, c0)
        for k in (2, 8):
            assert_close(gpu_spmv(A, x, c0, plan=dict(panels=k)), ref, den, FP64_TOL, f"{m}x{n} panels")
            assert_close(gpu_spmv(A, x, c0, plan=dict(kernel=5, panels=k)), ref, den, FP64_TOL,
                         f"{m}x{n} fused panels")
    # sorted blocks: ragged last block, one row, one column, few columns, empty
    for (m, n) in ((1000, 3000), (3000, 10), (1, 70000), (70000, 1), (40000, 5), (0, 5)):
        A = gen.random_crs(m, n, rng, max_len=12)
        x = gen.uniform_vector(n, rng)
        c0 = gen.uniform_vector(m, rng)
        ref, den = oracle_ref(A, x, c0)
        for e in (1, 4):
            assert_close(gpu_spmv(A, x, c0, plan=dict(kernel=6, tile_items=e)), ref, den, FP64_TOL,
                         f"{m}x{n} sorted blocks")
    # 1-based input gives the same product
    A = gen.random_crs(2000, 2000, rng, max_len=20)
    x = gen.uniform_vector(2000, rng)
    assert np.array_equal(gpu_spmv(A, x, base=1), gpu_spmv(A, x, base=0))
    del torch


def test_signed_zero_and_special_values():
    # products that are all -0.0 keep C0 = -0.0 negative, as the sequential loop does
    A = gen.CRS(3, 2, np.array([0, 2, 3, 3], np.int32), np.array([0, 1, 0], np.int32),
                np.array([-1.0, -1.0, 2.0]))
    x = np.array([0.0, 0.0])
    c0 = np.array([-0.0, -0.0, -0.0])
    got = gpu_spmv(A, x, c0)
    ref = oracle.spmv(A.row_ptr, A.col_idx, A.val, x, c0)
    assert np.array_equal(np.signbit(got), np.signbit(ref))
    # Inf and NaN propagate like the oracle
    rng = gen.rng_for(12, 0)
    A = gen.random_crs(3000, 3000, rng, max_len=10)
    A.val[::97] = np.inf
    A.val[::89] = -np.inf
    x = gen.uniform_vector(3000, rng)
    x[::500] = np.nan
    ref, den = oracle_ref(A, x)
    got = gpu_spmv(A, x)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    fin = np.isfinite(ref)
    assert np.array_equal(got[~fin & ~np.isnan(ref)], ref[~fin & ~np.isnan(ref)])
    assert_close(got[fin], ref[fin], den[fin], FP64_TOL, "finite rows")


def test_determinism():
    A, x = mats()["irregular"]
    a = gpu_spmv(A, x, runs=3)
    b = gpu_spmv(A, x, runs=3)
    assert np.array_equal(a, b)
    A27, x27 = mats()["27pt"]
    st = dict(kernel=spmv.SPMV_KERNEL_STAGED, tile_items=16)
    assert np.array_equal(gpu_spmv(A27, x27, plan=st, runs=2), gpu_spmv(A27, x27, plan=st, runs=2))
    # sorted blocks: row sums in a fixed chunk order, the same on every call
    for e in (1, 2, 4):
        sb = dict(kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS, tile_items=e)
        assert np.array_equal(gpu_spmv(A, x, plan=sb, runs=3), gpu_spmv(A, x, plan=sb, runs=3))


@pytest.mark.parametrize("kernel", [spmv.SPMV_KERNEL_STREAM, spmv.SPMV_KERNEL_TILE_GRID,
                                    spmv.SPMV_KERNEL_STAGED])
def test_batch_bit_deterministic(kernel):
    """Random data: two handles, each run twice, give the same bits, whichever
    workgroup the persistent queue hands a tile to."""
    import torch

    mem = _batch(count=40, seed_extra=6)
    xs = np.concatenate([x for _, x in mem])
    outs = []
    for _ in range(2):
        h = spmv.spmv_create_batch([(A.row_ptr, A.col_idx, A.val, A.n_cols) for A, _ in mem],
                                   flags=NOTUNE)
        try:
            spmv.spmv_set_plan(h, kernel=kernel, tile_items=8)
            B = to_dev(xs, "f64")
            C = torch.zeros(sum(A.n_rows for A, _ in mem), dtype=torch.float64, device="cuda")
            spmv.spmv_run(h, B, C)
            spmv.spmv_run(h, B, C)
            torch.cuda.synchronize()
            outs.append(C.cpu().numpy())
        finally:
            spmv.spmv_destroy(h)
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))


def test_handles_on_threads_and_streams():
    """Two handles driven from two host threads, each on a stream of its own
    (default priority), 20 products each: both results equal the same
    products run from one thread."""
    import threading

    import torch

    work = {"27pt": mats()["27pt"], "irregular": mats()["irregular"]}
    ref = {k: gpu_spmv(A, x, runs=20) for k, (A, x) in work.items()}
    out, errs = {}, []

    def run(key):
        try:
            A, x = work[key]
            st = torch.cuda.Stream()
            h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
            try:
                with torch.cuda.stream(st):
                    B = to_dev(x, "f64")
                    C = to_dev(np.zeros(A.n_rows), "f64")
                    for _ in range(20):
                        spmv.spmv_run(h, B, C, stream=st)
                st.synchronize()
                out[key] = C.cpu().numpy()
            finally:
                spmv.spmv_destroy(h)
        except Exception as e:  # reported below
            errs.append(repr(e))

    threads = [threading.Thread(target=run, args=(k,)) for k in work]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errs, errs
    for k in work:
        assert np.array_equal(out[k], ref[k]), k


@pytest.mark.parametrize("kind", ["plain", "split"])
def test_caller_graph_capture(kind):
    """A caller captures spmv_run in its own HIP graph (after one eager call,
    which builds the handle's tile tables) and replays it: every replay,
    with eager work and synchronisation in between, equals the same number of
    eager calls bit for bit."""
    import torch

    A, x = mats()["irregular"]
    hb = gen.halo_begin(A.n_cols)
    a = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    h = spmv.spmv_split_local_nonlocal(a, hb) if kind == "split" else a
    try:
        B = to_dev(x, "f64")
        halo = torch.from_numpy(np.ascontiguousarray(x[hb:])).pin_memory() if kind == "split" else None
        E = to_dev(np.zeros(A.n_rows), "f64")
        spmv.spmv_run(h, B, E, halo)  # eager warm-up
        torch.cuda.synchronize()
        C = torch.zeros_like(E)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            spmv.spmv_run(h, B, C, halo)
        for r in range(1, 6):
            g.replay()
            torch.cuda.synchronize()
            junk = torch.ones(1 << 20, device="cuda").cumsum(0)  # unrelated eager work
            torch.cuda.synchronize()
            del junk
            if r > 1:
                spmv.spmv_run(h, B, E, halo)
                torch.cuda.synchronize()
            assert torch.equal(C, E), f"replay {r}"
    finally:
        if h is not a:
            spmv.spmv_destroy(h)
        spmv.spmv_destroy(a)


def test_accumulates_into_c():
    A, x = mats()["27pt"]
    xi = np.round(x * 8)
    Ai = gen.stencil_27pt_3d(30)
    got = gpu_spmv(Ai, xi, runs=3)
    assert np.array_equal(got, 3 * oracle.spmv(Ai.row_ptr, Ai.col_idx, Ai.val, xi))


# ---------------------------------------------------------------------------- a1

SPECIAL = np.array([0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -24, 1 + 2 ** -23 + 2 ** -24,
                    3.0e38, 3.4e38, 3.5e38, 1e39, 1e-40, 9.1e-41, 5e-324, 1e-300, np.inf, -np.inf,
                    np.nan, 1.00000001, -7.5, 2.0 ** -126, 2.0 ** -127, 2.0 ** -133, 2.0 ** -134,
                    1.5 * 2.0 ** -134, 65504.0, 1 / 3])


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32f64"])
def test_ingest_export_matches_oracle_encoding(prec):
    rng = gen.rng_for(13, 0)
    A = gen.random_crs(4000, 500, rng, max_len=16)
    A.val[: SPECIAL.size] = SPECIAL
    A.val[SPECIAL.size:] *= 10.0 ** rng.integers(-40, 38, size=A.val.size - SPECIAL.size)
    for base in (0, 1):
        h = spmv.spmv_create_crs(A.row_ptr + base, A.col_idx + base, A.val, A.n_cols,
                                 index_base=base, prec=prec, flags=NOTUNE)
        try:
            assert np.array_equal(spmv.spmv_export(h, spmv.SPMV_ARR_ROW_PTR), A.row_ptr)
            assert np.array_equal(spmv.spmv_export(h, spmv.SPMV_ARR_COL), A.col_idx)
            v = spmv.spmv_export(h, spmv.SPMV_ARR_VAL)
            info = spmv.spmv_get_info(h)
        finally:
            spmv.spmv_destroy(h)
        if prec == "f64":
            assert np.array_equal(v.view(np.uint64), A.val.view(np.uint64))
        elif prec == "bf16":
            exp = oracle.round_bf16(A.val)
            nan = np.isnan(A.val)
            assert np.array_equal(v[~nan], exp[~nan])
            assert np.all((v[nan] & 0x7FFF) == 0x7FC0)
        else:
            exp = oracle.round_f32(A.val)
            nan = np.isnan(A.val)
            assert np.array_equal(v[~nan].view(np.uint32), exp[~nan].view(np.uint32))
            assert np.all(np.isnan(v[nan]))
        rl = np.diff(A.row_ptr)
        assert info["nnz"] == A.nnz and info["row_len_max"] == rl.max()
        assert abs(info["row_len_mean"] - rl.mean()) < 1e-9


# ---------------------------------------------------------------------------- a2, a4-a6

def _split_handles(A, h_begin, prec="f64", flags=NOTUNE):
    a = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, prec=prec, flags=flags)
    s = spmv.spmv_split_local_nonlocal(a, h_begin)
    return a, s


@pytest.mark.parametrize("prec", ["f64", "bf16"])
@pytest.mark.parametrize("where", ["band", "zero", "all", "mid"])
def test_split_bookkeeping_bit_exact(prec, where):
    A, x = mats()["irregular"]
    h_begin = {"band": gen.halo_begin(A.n_cols), "zero": 0, "all": A.n_cols,
               "mid": A.n_cols // 2 + 1}[where]
    a, s = _split_handles(A, h_begin, prec)
    try:
        got = {k: spmv.spmv_export(s, w) for k, w in (
            ("loc_row_ptr", spmv.SPMV_ARR_ROW_PTR), ("loc_col", spmv.SPMV_ARR_COL),
            ("loc_val", spmv.SPMV_ARR_VAL), ("nl_rows", spmv.SPMV_ARR_NL_ROWS),
            ("nl_ptr", spmv.SPMV_ARR_NL_PTR), ("nl_col", spmv.SPMV_ARR_NL_COL),
            ("nl_val", spmv.SPMV_ARR_NL_VAL))}
        info = spmv.spmv_get_info(s)
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)
    ref = oracle.split(A.row_ptr, A.col_idx, A.val, h_begin)
    for k in ("loc_row_ptr", "loc_col", "nl_rows", "nl_ptr", "nl_col"):
        assert np.array_equal(got[k], ref[k]), k
    enc = (lambda v: v) if prec == "f64" else oracle.round_bf16
    for k in ("loc_val", "nl_val"):
        assert np.array_equal(got[k], enc(ref[k])), k
    assert info["nnz_local"] == ref["loc_col"].size
    assert info["n_nonlocal_rows"] == ref["nl_rows"].size
    assert info["halo_begin"] == h_begin


def _run_split(A, x, h_begin, schedule, prec="f64", halo="pinned", c0=None, flags=NOTUNE):
    import torch

    a, s = _split_handles(A, h_begin, prec, flags)
    try:
        spmv.spmv_set_schedule(s, schedule)
        xd = np.asarray(x, dtype=np.float64)
        B_host = xd.copy()
        B_host[h_begin:] = np.nan  # receive area: must be overwritten by the halo copy
        B = to_dev(B_host, prec)
        C = to_dev(np.zeros(A.n_rows) if c0 is None else c0, prec)
        halo_t = torch.from_numpy(np.ascontiguousarray(xd[h_begin:])).to(B.dtype)
        if halo == "pinned":
            halo_t = halo_t.pin_memory()
        spmv.spmv_run(s, B, C, halo_t)
        torch.cuda.synchronize()
        recv = B[h_begin:].cpu().numpy()
        return C.cpu().numpy().astype(np.float64), recv
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


def test_split_tune_schedule_unless_set():
    """spmv_tune on a split handle may switch it to the nonlocal-beside
    schedule (the product stays the oracle's); once the caller has set a
    schedule, tuning keeps it (serial: the copy ends before the local part)."""
    import torch

    A, x = mats()["irregular"]
    hb = gen.halo_begin(A.n_cols)
    ref, den = oracle_ref(A, x)
    halo = torch.from_numpy(np.ascontiguousarray(x[hb:])).pin_memory()
    for preset in (None, spmv.SPMV_SCHEDULE_SERIAL):
        a, s = _split_handles(A, hb)
        try:
            spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS,
                               tile_items=2)
            if preset is not None:
                spmv.spmv_set_schedule(s, preset)
            spmv.spmv_tune(s, 1)
            spmv.spmv_set_phase_timing(s, True)
            Bh = x.copy()
            Bh[hb:] = np.nan
            B = to_dev(Bh, "f64")
            C = to_dev(np.zeros(A.n_rows), "f64")
            spmv.spmv_run(s, B, C, halo)
            torch.cuda.synchronize()
            assert_close(C.cpu().numpy(), ref, den, FP64_TOL, f"tuned split, preset {preset}")
            t = spmv.spmv_phase_times(s)
            if preset == spmv.SPMV_SCHEDULE_SERIAL:
                assert t["copy"][1] <= t["local"][0] + 0.01
        finally:
            spmv.spmv_destroy(s)
            spmv.spmv_destroy(a)


@pytest.mark.parametrize("schedule", [spmv.SPMV_SCHEDULE_OVERLAP, spmv.SPMV_SCHEDULE_OVERLAP_NONLOCAL,
                                      spmv.SPMV_SCHEDULE_OVERLAP_MERGED, spmv.SPMV_SCHEDULE_SERIAL])
def test_split_run_matches_oracle(schedule):
    A, x = mats()["irregular"]
    h_begin = gen.halo_begin(A.n_cols)
    c0 = gen.uniform_vector(A.n_rows, gen.rng_for(14, 0))
    got, recv = _run_split(A, x, h_begin, schedule, c0=c0)
    assert np.array_equal(recv, x[h_begin:])
    ref, den = oracle_ref(A, x, c0)
    assert_close(got, ref, den, FP64_TOL, "split vs unsplit oracle")
    parts = oracle.split(A.row_ptr, A.col_idx, A.val, h_begin)
    assert_close(got, oracle.spmv_split(parts, x, c0), den, FP64_TOL, "split vs split oracle")


@pytest.mark.parametrize("plan", [None, dict(kernel=1, tile_items=8, panels=4),
                                  dict(kernel=2, lanes=8), dict(kernel=1, tile_items=16, tiles_per_group=4),
                                  dict(kernel=4, tile_items=8), dict(kernel=5, tile_items=8, panels=2),
                                  dict(kernel=5, tile_items=16, panels=1),
                                  dict(kernel=6, tile_items=2)],
                         ids=["default", "panels4", "vector8", "pipelined", "staged8", "fused2",
                              "fused1", "sorted2"])
def test_local_part_never_reads_halo(plan):
    """The receive area B[h:] holds NaN and no halo is copied: rows without a
    halo entry are computed by the local part alone and must be finite and
    equal to the oracle's local product; a single read of the receive area by
    the local kernel would make some of them NaN."""
    import torch

    A, x = mats()["irregular"]
    h_begin = gen.halo_begin(A.n_cols)
    a, s = _split_handles(A, h_begin)
    try:
        if plan:
            spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, **plan)
        Bh = x.copy()
        Bh[h_begin:] = np.nan
        B = to_dev(Bh, "f64")
        C = to_dev(np.zeros(A.n_rows), "f64")
        spmv.spmv_run(s, B, C)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)
    parts = oracle.split(A.row_ptr, A.col_idx, A.val, h_begin)
    only_local = np.ones(A.n_rows, bool)
    only_local[parts["nl_rows"]] = False
    assert np.isnan(got[parts["nl_rows"]]).all()
    assert np.isfinite(got[only_local]).all()
    ref = oracle.spmv(parts["loc_row_ptr"], parts["loc_col"], parts["loc_val"], x)
    den = oracle.abs_spmv(parts["loc_row_ptr"], parts["loc_col"], parts["loc_val"], x)
    assert_close(got[only_local], ref[only_local], den[only_local], FP64_TOL, "local rows")


def test_split_local_part_panels():
    import torch

    A, x = mats()["irregular"]
    h_begin = gen.halo_begin(A.n_cols)
    a, s = _split_handles(A, h_begin)
    try:
        spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, panels=4)
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_set_plan(s, spmv.SPMV_PART_NONLOCAL, panels=2)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_set_plan(s, spmv.SPMV_PART_NONLOCAL, kernel=5, panels=1)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        B = to_dev(x, "f64")
        C = to_dev(np.zeros(A.n_rows), "f64")
        spmv.spmv_run(s, B, C)
        torch.cuda.synchronize()
        ref, den = oracle_ref(A, x)
        assert_close(C.cpu().numpy(), ref, den, FP64_TOL, "split with local panels")
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


@pytest.mark.parametrize("tpw", [1, 4, 32])
def test_split_pipelined_plans(tpw):
    import torch

    A, x = mats()["irregular"]
    h_begin = gen.halo_begin(A.n_cols)
    a, s = _split_handles(A, h_begin)
    try:
        spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, tiles_per_group=tpw, tile_items=8)
        spmv.spmv_set_plan(s, spmv.SPMV_PART_NONLOCAL, tiles_per_group=tpw, tile_items=4)
        B = to_dev(x, "f64")
        C = to_dev(np.zeros(A.n_rows), "f64")
        spmv.spmv_run(s, B, C)
        torch.cuda.synchronize()
        ref, den = oracle_ref(A, x)
        assert_close(C.cpu().numpy(), ref, den, FP64_TOL, f"split tpw={tpw}")
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


def test_split_integer_bit_exact_and_edges():
    rng = gen.rng_for(15, 0)
    A = gen.random_crs(20000, 20000, rng, max_len=20, integer_values=True)
    x = gen.integer_vector(A.n_cols, rng)
    exact = oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
    for h_begin in (0, 1, 18800, 19999, 20000):
        for sch in (spmv.SPMV_SCHEDULE_OVERLAP, spmv.SPMV_SCHEDULE_OVERLAP_NONLOCAL,
                    spmv.SPMV_SCHEDULE_OVERLAP_MERGED, spmv.SPMV_SCHEDULE_SERIAL):
            got, _ = _run_split(A, x, h_begin, sch)
            assert np.array_equal(got, exact), (h_begin, sch)


@pytest.mark.parametrize("plan", [dict(kernel=1, tile_items=8), dict(kernel=1, tile_items=8, panels=4),
                                  dict(kernel=1, tile_items=4, tiles_per_group=4),
                                  dict(kernel=4, tile_items=8), dict(kernel=2, lanes=8),
                                  dict(kernel=5, tile_items=8, panels=2),
                                  dict(kernel=6, tile_items=2), dict(kernel=6, tile_items=1)],
                         ids=["stream", "panels4", "pipelined", "staged", "vector", "fused",
                              "sorted2", "sorted1"])
def test_split_local_halves_beside_nonlocal(plan):
    """The banded irregular matrix's nonlocal rows are a tail of the rows, so
    the local part is tiled in two halves cut at the first nonlocal row: the
    upper half runs while the nonlocal part runs on its own stream.  Its tile
    table has a tile starting exactly at that row, and on integer data every
    schedule gives the oracle's product bit for bit (with C0); plans that
    cannot run halves (vector, fused) take the ordered path, and so do plans
    other than sorted blocks under the merged schedule."""
    import torch

    A, _ = mats()["irregular"]
    rng = gen.rng_for(15, 1)
    A = gen.CRS(A.n_rows, A.n_cols, A.row_ptr, A.col_idx,
                rng.integers(-9, 10, size=A.nnz).astype(np.float64))
    x = gen.integer_vector(A.n_cols, rng)
    c0 = gen.integer_vector(A.n_rows, rng)
    h_begin = gen.halo_begin(A.n_cols)
    exact = oracle.spmv(A.row_ptr, A.col_idx, A.val, x, c0)
    parts = oracle.split(A.row_ptr, A.col_idx, A.val, h_begin)
    first_nl = int(parts["nl_rows"][0])
    assert 0 < first_nl < A.n_rows
    a, s = _split_handles(A, h_begin)
    try:
        spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, **plan)
        if plan["kernel"] in (1, 4) and plan.get("panels", 1) == 1:
            tiles = spmv.spmv_export(s, spmv.SPMV_ARR_TILES).view(np.int32).reshape(-1, 2)
            assert first_nl in set(tiles[:, 0].tolist())
        halo = torch.from_numpy(np.ascontiguousarray(x[h_begin:])).pin_memory()
        for sch in (spmv.SPMV_SCHEDULE_OVERLAP, spmv.SPMV_SCHEDULE_OVERLAP_NONLOCAL,
                    spmv.SPMV_SCHEDULE_OVERLAP_MERGED, spmv.SPMV_SCHEDULE_SERIAL):
            spmv.spmv_set_schedule(s, sch)
            for with_copy in (True, False):
                Bh = x.copy()
                if with_copy:
                    Bh[h_begin:] = np.nan
                B = to_dev(Bh, "f64")
                C = to_dev(c0, "f64")
                spmv.spmv_run(s, B, C, halo if with_copy else None)
                torch.cuda.synchronize()
                assert np.array_equal(C.cpu().numpy(), exact), (sch, with_copy)
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32f64"])
@pytest.mark.parametrize("items", [1, 2, 4])
def test_split_merged_tail(prec, items):
    """SPMV_SCHEDULE_OVERLAP_MERGED with a sorted-block local plan: the
    blocks from the one that holds the first nonlocal row run over their
    rows' local and nonlocal entries together, after the halo copy and
    inside the local part's span, with no nonlocal kernel.  Checked against
    the oracle (to the precision's bound) with the band's halo, with halos
    whose first nonlocal row falls in the second block and in the first
    (every block merged), and with no halo and an all-halo B (the ordered
    path); the same bits on a second call."""
    import torch

    A, x = mats()["irregular"]
    n = int(np.diff(A.row_ptr).max())
    b_orig, _ = prec_bounds(prec, n)
    c0 = gen.uniform_vector(A.n_rows, gen.rng_for(14, 3))
    ref, den = oracle_ref(A, x, c0)
    for hb in (gen.halo_begin(A.n_cols), A.n_cols // 4, 10000, A.n_cols, 0):
        a, s = _split_handles(A, hb, prec)
        try:
            spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS,
                               tile_items=items)
            spmv.spmv_set_schedule(s, spmv.SPMV_SCHEDULE_OVERLAP_MERGED)
            spmv.spmv_set_phase_timing(s, True)
            info = spmv.spmv_get_info(s)
            merged = 0 < hb < A.n_cols and info["nnz_local"] > 0
            Bh = x.copy()
            Bh[hb:] = np.nan
            halo = torch.from_numpy(np.ascontiguousarray(x[hb:])).to(torch_dtype(prec))
            halo = halo.pin_memory() if hb < A.n_cols else None
            outs = []
            for _ in range(2):
                B = to_dev(Bh, prec)
                C = to_dev(c0, prec)
                spmv.spmv_run(s, B, C, halo)
                torch.cuda.synchronize()
                outs.append(C.cpu().numpy().astype(np.float64))
                t = spmv.spmv_phase_times(s)
                if merged:
                    eps = 0.01
                    assert t["copy"][1] <= t["nonlocal"][0] + eps
                    assert t["local"][0] <= t["nonlocal"][0] + eps
                    assert t["nonlocal"][1] <= t["local"][1] + eps
            assert_close(outs[0], ref, den, b_orig, f"merged tail {prec} E={items} halo {hb}")
            assert np.array_equal(outs[0], outs[1]), f"merged tail {prec} E={items} halo {hb}"
        finally:
            spmv.spmv_destroy(s)
            spmv.spmv_destroy(a)


def test_split_merged_tail_integer_exact():
    """The merged layout on integer data: the oracle's product bit for bit,
    with the copy and with the halo resident, for every chunk size."""
    import torch

    A, _ = mats()["irregular"]
    rng = gen.rng_for(15, 2)
    A = gen.CRS(A.n_rows, A.n_cols, A.row_ptr, A.col_idx,
                rng.integers(-9, 10, size=A.nnz).astype(np.float64))
    x = gen.integer_vector(A.n_cols, rng)
    c0 = gen.integer_vector(A.n_rows, rng)
    hb = gen.halo_begin(A.n_cols)
    exact = oracle.spmv(A.row_ptr, A.col_idx, A.val, x, c0)
    halo = torch.from_numpy(np.ascontiguousarray(x[hb:])).pin_memory()
    a, s = _split_handles(A, hb)
    try:
        spmv.spmv_set_schedule(s, spmv.SPMV_SCHEDULE_OVERLAP_MERGED)
        for e in (1, 2, 4):
            spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS,
                               tile_items=e)
            for with_copy in (True, False):
                Bh = x.copy()
                if with_copy:
                    Bh[hb:] = np.nan
                B = to_dev(Bh, "f64")
                C = to_dev(c0, "f64")
                spmv.spmv_run(s, B, C, halo if with_copy else None)
                torch.cuda.synchronize()
                assert np.array_equal(C.cpu().numpy(), exact), (e, with_copy)
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


def test_split_resident_halo_and_pageable_rejection():
    import torch

    A, x = mats()["irregular"]
    h_begin = gen.halo_begin(A.n_cols)
    a, s = _split_handles(A, h_begin)
    try:
        B = to_dev(x, "f64")
        C = to_dev(np.zeros(A.n_rows), "f64")
        spmv.spmv_run(s, B, C)  # halo already resident
        torch.cuda.synchronize()
        ref, den = oracle_ref(A, x)
        assert_close(C.cpu().numpy(), ref, den, FP64_TOL, "resident halo")
        pageable = torch.from_numpy(np.ascontiguousarray(x[h_begin:]))
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_run(s, B, C, pageable)
        assert ei.value.status == spmv.SPMV_ERR_INVALID_ARG and "pinned" in ei.value.message
        with pytest.raises((ValueError, spmv.SpmvError)):
            spmv.spmv_run(a, B, C, pageable.pin_memory())  # plain handle takes no halo
        hp = pageable.pin_memory()
        st = spmv.load().spmv_run(spmv.ctypes.c_void_p(a.ptr), spmv.ctypes.c_void_p(B.data_ptr()),
                                  spmv.ctypes.c_void_p(C.data_ptr()),
                                  spmv.ctypes.c_void_p(hp.data_ptr()), None)
        assert st == spmv.SPMV_ERR_INVALID_ARG
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)
    got, _ = _run_split(A, x, h_begin, spmv.SPMV_SCHEDULE_OVERLAP, halo="pageable",
                        flags=NOTUNE | spmv.SPMV_FLAG_ALLOW_PAGEABLE_HALO)
    assert_close(got, ref, den, FP64_TOL, "pageable halo with flag")


def test_split_of_split_unsupported():
    A, _ = mats()["irregular"]
    a, s = _split_handles(A, 10)
    try:
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_split_local_nonlocal(s, 5)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_split_local_nonlocal(a, A.n_cols + 1)
        assert ei.value.status == spmv.SPMV_ERR_INVALID_ARG
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


# ---------------------------------------------------------------------------- a7

@pytest.mark.parametrize("prec", ["f32", "bf16", "f32f64"])
@pytest.mark.parametrize("name", ["27pt", "irregular"])
def test_precision_modes(prec, name):
    A, x = mats()[name]
    n = int(np.diff(A.row_ptr).max())
    b_orig, b_same = prec_bounds(prec, n)
    got = gpu_spmv(A, x, prec=prec)
    ref, den = oracle_ref(A, x)
    assert_close(got, ref, den, b_orig, f"{prec} vs FP64 oracle")
    v, xr = rounded_inputs(A, x, prec)
    ref2 = oracle.spmv(A.row_ptr, A.col_idx, v, xr)
    den2 = oracle.abs_spmv(A.row_ptr, A.col_idx, v, xr)
    assert_close(got, ref2, den2, b_same, f"{prec} vs oracle on rounded inputs")


@pytest.mark.parametrize("prec", ["f32", "bf16", "f32f64"])
@pytest.mark.parametrize("items", [1, 4])
def test_precision_modes_sorted_blocks(prec, items):
    plan = dict(kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS, tile_items=items)
    for name in ("27pt", "irregular"):
        A, x = mats()[name]
        n = int(np.diff(A.row_ptr).max())
        b_orig, b_same = prec_bounds(prec, n)
        got = gpu_spmv(A, x, prec=prec, plan=plan)
        ref, den = oracle_ref(A, x)
        assert_close(got, ref, den, b_orig, f"{name} {prec} sorted vs FP64 oracle")
        v, xr = rounded_inputs(A, x, prec)
        ref2 = oracle.spmv(A.row_ptr, A.col_idx, v, xr)
        den2 = oracle.abs_spmv(A.row_ptr, A.col_idx, v, xr)
        assert_close(got, ref2, den2, b_same, f"{name} {prec} sorted vs oracle on rounded inputs")
    rng = gen.rng_for(16, 1)
    A = gen.random_crs(70000, 6000, rng, max_len=30, integer_values=True, vmax=8)
    x = gen.integer_vector(A.n_cols, rng, vmax=8)
    assert np.array_equal(gpu_spmv(A, x, prec=prec, plan=plan),
                          oracle.spmv(A.row_ptr, A.col_idx, A.val, x))


@pytest.mark.parametrize("prec", ["f32", "bf16", "f32f64"])
def test_precision_modes_integer_exact(prec):
    rng = gen.rng_for(16, 0)
    A = gen.random_crs(6000, 6000, rng, max_len=30, integer_values=True, vmax=8)
    x = gen.integer_vector(A.n_cols, rng, vmax=8)
    assert np.array_equal(gpu_spmv(A, x, prec=prec), oracle.spmv(A.row_ptr, A.col_idx, A.val, x))


# ---------------------------------------------------------------------------- a8

def _gpu_block(A, X, prec="f64", kt=0, ldb_pad=0, ldc_pad=0, c0=None):
    import torch

    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, prec=prec, flags=NOTUNE)
    try:
        if kt:
            spmv.spmv_set_plan(h, block_kt=kt)
        k = X.shape[1]
        dt = torch.float64 if spmv.VEC_DTYPE[prec] == "float64" else torch.float32
        Bw = torch.zeros((A.n_cols, k + ldb_pad), dtype=dt, device="cuda")
        Bw[:, :k] = torch.from_numpy(X).to(dt)
        Cw = torch.zeros((A.n_rows, k + ldc_pad), dtype=dt, device="cuda")
        if c0 is not None:
            Cw[:, :k] = torch.from_numpy(c0).to(dt)
        spmv.spmv_run_block(h, Bw[:, :k], Cw[:, :k])
        torch.cuda.synchronize()
        return Cw[:, :k].cpu().numpy().astype(np.float64), Cw[:, k:].cpu().numpy()
    finally:
        spmv.spmv_destroy(h)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 16, 17, 33, 64])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_block(k, prec):
    A, _ = mats()["irregular"]
    X = gen.block_rhs(A.n_cols, k)
    c0 = gen.block_rhs(A.n_rows, k, extra=1)
    got, pad = _gpu_block(A, X, prec, c0=c0, ldb_pad=1 if k % 2 else 2, ldc_pad=3)
    assert np.all(pad == 0)
    n = int(np.diff(A.row_ptr).max())
    b_orig, _ = prec_bounds(prec, n)
    ref = oracle.spmv_block(A.row_ptr, A.col_idx, A.val, X, c0)
    for t in range(k):
        den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, X[:, t], c0[:, t])
        assert_close(got[:, t], ref[:, t], den, b_orig, f"block k={k} column {t}")


@pytest.mark.parametrize("kt", [4, 8, 16])
@pytest.mark.parametrize("k", [3, 8, 16])
def test_block_tiles_integer_exact(kt, k):
    rng = gen.rng_for(17, 0)
    A = _long_row_matrix(3000, n_short=2000, n_cols=5000)
    A.val = np.round(A.val * 4)
    X = rng.integers(-5, 6, size=(A.n_cols, k)).astype(np.float64)
    got, _ = _gpu_block(A, X, "f64", kt=kt)
    assert np.array_equal(got, oracle.spmv_block(A.row_ptr, A.col_idx, A.val, X))


@pytest.mark.parametrize("panels", [2, 8])
@pytest.mark.parametrize("k", [3, 16])
def test_block_with_panels(k, panels):
    import torch

    A, _ = mats()["irregular"]
    X = gen.block_rhs(A.n_cols, k, extra=7)
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        spmv.spmv_set_plan(h, panels=panels)
        B = torch.from_numpy(X).cuda()
        C = torch.zeros((A.n_rows, k), dtype=torch.float64, device="cuda")
        spmv.spmv_run_block(h, B, C)
        c1 = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
        spmv.spmv_run(h, B[:, 0].contiguous(), c1)  # single-vector path shares the panels
        torch.cuda.synchronize()
        got = C.cpu().numpy()
    finally:
        spmv.spmv_destroy(h)
    ref = oracle.spmv_block(A.row_ptr, A.col_idx, A.val, X)
    for t in range(k):
        den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, X[:, t])
        assert_close(got[:, t], ref[:, t], den, FP64_TOL, f"block k={k} panels={panels} col {t}")
    den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, X[:, 0])
    assert_close(c1.cpu().numpy(), ref[:, 0], den, FP64_TOL, "single vector with panels")


def _gpu_block_plan(A, X, plan, c0=None, prec="f64", ldb_pad=0, ldc_pad=0):
    import torch

    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, prec=prec, flags=NOTUNE)
    try:
        spmv.spmv_set_plan(h, **plan)
        bp = spmv.spmv_get_block_plan(h, X.shape[1])
        assert all(bp[f] == v for f, v in plan.items()), (bp, plan)
        k = X.shape[1]
        dt = torch.float64 if spmv.VEC_DTYPE[prec] == "float64" else torch.float32
        Bw = torch.zeros((A.n_cols, k + ldb_pad), dtype=dt, device="cuda")
        Bw[:, :k] = torch.from_numpy(X).to(dt)
        Cw = torch.zeros((A.n_rows, k + ldc_pad), dtype=dt, device="cuda")
        if c0 is not None:
            Cw[:, :k] = torch.from_numpy(c0).to(dt)
        spmv.spmv_run_block(h, Bw[:, :k], Cw[:, :k])
        torch.cuda.synchronize()
        return Cw[:, :k].cpu().numpy().astype(np.float64), Cw[:, k:].cpu().numpy()
    finally:
        spmv.spmv_destroy(h)


@pytest.mark.parametrize("panels", [1, 2, 4, 8])
@pytest.mark.parametrize("kt", [4, 8, 16])
@pytest.mark.parametrize("k", [1, 3, 4, 8, 16, 17])
def test_block_fused_panels(k, kt, panels):
    """The fused-panel block kernel (all panels of a row block in one
    workgroup, C written once) against the oracle, with C0, padded leading
    dimensions (odd k takes the one-column-per-lane layout)."""
    A, _ = mats()["irregular"]
    X = gen.block_rhs(A.n_cols, k, extra=11)
    c0 = gen.block_rhs(A.n_rows, k, extra=12)
    plan = dict(kernel=5, panels=panels, block_kt=kt, xcd_remap=panels % 2)
    got, pad = _gpu_block_plan(A, X, plan, c0, ldb_pad=1 if k % 2 else 2, ldc_pad=3)
    assert np.all(pad == 0)
    ref = oracle.spmv_block(A.row_ptr, A.col_idx, A.val, X, c0)
    for t in range(k):
        den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, X[:, t], c0[:, t])
        assert_close(got[:, t], ref[:, t], den, FP64_TOL, f"fused block k={k} kt={kt} panels={panels} col {t}")


@pytest.mark.parametrize("panels", [1, 4])
@pytest.mark.parametrize("k", [3, 16])
def test_block_fused_integer_exact_long_rows(k, panels):
    """Rows far longer than a staged tile (the row-by-row path) and ordinary
    ones, integer data: bit for bit against the oracle; F32 too."""
    rng = gen.rng_for(17, 1)
    A = _long_row_matrix(3000, n_short=2000, n_cols=5000)
    A.val = np.round(A.val * 4)
    X = rng.integers(-5, 6, size=(A.n_cols, k)).astype(np.float64)
    want = oracle.spmv_block(A.row_ptr, A.col_idx, A.val, X)
    for prec in ("f64", "f32"):
        got, _ = _gpu_block_plan(A, X, dict(kernel=5, panels=panels, block_kt=8), prec=prec)
        assert np.array_equal(got, want), prec


@pytest.mark.parametrize("items", [1, 2, 4])
@pytest.mark.parametrize("kt", [4, 8, 16])
@pytest.mark.parametrize("k", [1, 3, 4, 8, 16, 17])
def test_block_sorted(k, kt, items):
    """The sorted-block kernel for blocks (plan kernel 6 with block_kt: R * kt
    sums per block in LDS, kt lanes per slot, one pass per kt columns)
    against the oracle, with C0 and padded leading dimensions; a second call
    adds the same bits again (C0 + 2 A X)."""
    import torch

    A, _ = mats()["irregular"]
    X = gen.block_rhs(A.n_cols, k, extra=21)
    c0 = gen.block_rhs(A.n_rows, k, extra=22)
    plan = dict(kernel=6, tile_items=items, block_kt=kt)
    got, pad = _gpu_block_plan(A, X, plan, c0, ldb_pad=1 if k % 2 else 2, ldc_pad=3)
    assert np.all(pad == 0)
    ref = oracle.spmv_block(A.row_ptr, A.col_idx, A.val, X, c0)
    for t in range(k):
        den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, X[:, t], c0[:, t])
        assert_close(got[:, t], ref[:, t], den, FP64_TOL, f"sorted block k={k} kt={kt} E={items} col {t}")
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        spmv.spmv_set_plan(h, **plan)
        B = torch.from_numpy(X).cuda()
        C1 = torch.zeros((A.n_rows, k), dtype=torch.float64, device="cuda")
        C2 = torch.zeros((A.n_rows, k), dtype=torch.float64, device="cuda")
        spmv.spmv_run_block(h, B, C1)
        spmv.spmv_run_block(h, B, C2)
        spmv.spmv_run_block(h, B, C2)
        torch.cuda.synchronize()
        assert torch.equal(C2, C1 + C1), "two calls add the same bits twice"
    finally:
        spmv.spmv_destroy(h)


@pytest.mark.parametrize("prec", ["f32", "bf16", "f32f64"])
def test_block_sorted_precision(prec):
    A, _ = mats()["irregular"]
    k = 8
    X = gen.block_rhs(A.n_cols, k, extra=23)
    got, _ = _gpu_block_plan(A, X, dict(kernel=6, tile_items=2, block_kt=4), prec=prec)
    n = int(np.diff(A.row_ptr).max())
    b_orig, _ = prec_bounds(prec, n)
    ref = oracle.spmv_block(A.row_ptr, A.col_idx, A.val, X)
    for t in range(k):
        den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, X[:, t])
        assert_close(got[:, t], ref[:, t], den, b_orig, f"sorted block {prec} col {t}")


def test_block_sorted_integer_exact_and_edges():
    """Integer data: bit for bit for every width; a matrix with empty rows
    and a ragged last block; and a part of rows too long for the layout is
    refused when the plan is set."""
    rng = gen.rng_for(17, 3)
    A = gen.random_crs(70000, 6000, rng, max_len=30, integer_values=True, vmax=8)
    for k in (1, 5, 16):
        X = rng.integers(-5, 6, size=(A.n_cols, k)).astype(np.float64)
        want = oracle.spmv_block(A.row_ptr, A.col_idx, A.val, X)
        for kt in (4, 16):
            got, _ = _gpu_block_plan(A, X, dict(kernel=6, tile_items=2, block_kt=kt))
            assert np.array_equal(got, want), (k, kt)
    L = _long_row_matrix(3000, n_short=2000, n_cols=5000)
    if _sorted_refused(L, 2):
        h = spmv.spmv_create_crs(L.row_ptr, L.col_idx, L.val, L.n_cols, flags=NOTUNE)
        try:
            before = spmv.spmv_get_plan(h)
            with pytest.raises(spmv.SpmvError) as ei:
                spmv.spmv_set_plan(h, kernel=6, tile_items=2, block_kt=4)
            assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
            assert spmv.spmv_get_plan(h) == before, "a refused plan is not kept"
            X = rng.integers(-5, 6, size=(L.n_cols, 3)).astype(np.float64)
            import torch
            C = torch.zeros((L.n_rows, 3), dtype=torch.float64, device="cuda")
            spmv.spmv_run_block(h, torch.from_numpy(X).cuda(), C)
            torch.cuda.synchronize()
            Lr = gen.CRS(L.n_rows, L.n_cols, L.row_ptr, L.col_idx, L.val)
            ref = oracle.spmv_block(Lr.row_ptr, Lr.col_idx, Lr.val, X)
            for t in range(3):
                den = oracle.abs_spmv(Lr.row_ptr, Lr.col_idx, Lr.val, X[:, t])
                assert_close(C.cpu().numpy()[:, t], ref[:, t], den, FP64_TOL, "after a refused plan")
        finally:
            spmv.spmv_destroy(h)


def test_block_rejects_split_and_bad_k():
    import torch

    A, _ = mats()["irregular"]
    a, s = _split_handles(A, 100)
    try:
        B = torch.zeros((A.n_cols, 4), dtype=torch.float64, device="cuda")
        C = torch.zeros((A.n_rows, 4), dtype=torch.float64, device="cuda")
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_run_block(s, B, C)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        B = torch.zeros((A.n_cols, 65), dtype=torch.float64, device="cuda")
        C = torch.zeros((A.n_rows, 65), dtype=torch.float64, device="cuda")
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_run_block(a, B, C)
        assert ei.value.status == spmv.SPMV_ERR_INVALID_ARG
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


# ---------------------------------------------------------------------------- a9

def _batch(count=40, nmax=30000, seed_extra=1):
    return gen.workload_c5_batch(count=count, nmin=1000, nmax=nmax, seed_extra=seed_extra)


@pytest.mark.parametrize("kernel,tile_items",
                         [(k, e) for k in (spmv.SPMV_KERNEL_STREAM, spmv.SPMV_KERNEL_TILE_GRID)
                          for e in (4, 8, 16)] +
                         [(spmv.SPMV_KERNEL_STAGED, e) for e in (8, 16)])
@pytest.mark.parametrize("schedule", [spmv.SPMV_SCHEDULE_BATCH_GRAPH, spmv.SPMV_SCHEDULE_BATCH_DIRECT,
                                      spmv.SPMV_SCHEDULE_BATCH_FLAT])
def test_batch_matches_members(schedule, tile_items, kernel):
    import torch

    mem = _batch()
    h = spmv.spmv_create_batch([(A.row_ptr, A.col_idx, A.val, A.n_cols) for A, _ in mem], flags=NOTUNE)
    try:
        spmv.spmv_set_schedule(h, schedule)
        spmv.spmv_set_plan(h, tile_items=tile_items, kernel=kernel)
        xs = np.concatenate([x for _, x in mem])
        c0 = gen.uniform_vector(sum(A.n_rows for A, _ in mem), gen.rng_for(18, 0))
        B = to_dev(xs, "f64")
        C = to_dev(c0, "f64")
        spmv.spmv_run(h, B, C)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
    finally:
        spmv.spmv_destroy(h)
    off = 0
    for A, x in mem:
        sl = slice(off, off + A.n_rows)
        ref, den = oracle_ref(A, x, c0[sl])
        assert_close(got[sl], ref, den, FP64_TOL, f"member at {off}")
        off += A.n_rows


@pytest.mark.parametrize("count", [1, 3, 8, 9, 17])
@pytest.mark.parametrize("schedule", [spmv.SPMV_SCHEDULE_BATCH_GRAPH, spmv.SPMV_SCHEDULE_BATCH_DIRECT])
def test_batch_queue_fewer_tiles_than_queues(count, schedule):
    """The persistent queue with fewer tiles than XCD queues (some queues
    empty) or a few more: every tile is claimed exactly once, on each of
    three calls in a row (the counters are reset before every launch)."""
    import torch

    rng = gen.rng_for(19, count)
    mem = [gen.random_crs(int(rng.integers(1, 400)), int(rng.integers(1, 300)), rng, max_len=6,
                          integer_values=True) for _ in range(count)]
    xs = [gen.integer_vector(A.n_cols, rng) for A in mem]
    exact = np.concatenate([oracle.spmv(A.row_ptr, A.col_idx, A.val, x) for A, x in zip(mem, xs)])
    h = spmv.spmv_create_batch([(A.row_ptr, A.col_idx, A.val, A.n_cols) for A in mem], flags=NOTUNE)
    try:
        spmv.spmv_set_schedule(h, schedule)
        spmv.spmv_set_plan(h, kernel=spmv.SPMV_KERNEL_STREAM, tile_items=4)
        B = to_dev(np.concatenate(xs), "f64")
        C = torch.zeros(exact.size, dtype=torch.float64, device="cuda")
        for r in range(1, 4):
            spmv.spmv_run(h, B, C)
            torch.cuda.synchronize()
            assert np.array_equal(C.cpu().numpy(), r * exact), f"call {r}"
    finally:
        spmv.spmv_destroy(h)


@pytest.mark.parametrize("kernel", [spmv.SPMV_KERNEL_STREAM, spmv.SPMV_KERNEL_TILE_GRID,
                                    spmv.SPMV_KERNEL_STAGED])
def test_batch_graph_replays_and_recapture(kernel):
    import torch

    mem = _batch(count=24, seed_extra=2)
    xs = np.concatenate([np.round(8 * x) for _, x in mem])  # integer RHS: exact results
    exact = []
    off = 0
    for A, _ in mem:
        exact.append(oracle.spmv(A.row_ptr, A.col_idx, A.val, xs[off:off + A.n_cols]))
        off += A.n_cols
    exact = np.concatenate(exact)
    h = spmv.spmv_create_batch([(A.row_ptr, A.col_idx, A.val, A.n_cols) for A, _ in mem], flags=NOTUNE)
    try:
        spmv.spmv_set_plan(h, kernel=kernel)
        B = to_dev(xs, "f64")
        C = torch.zeros(exact.size, dtype=torch.float64, device="cuda")
        for r in range(1, 5):
            spmv.spmv_run(h, B, C)  # graph replay (captured on the first call)
            torch.cuda.synchronize()
            junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
            torch.cuda.synchronize()
            assert np.array_equal(C.cpu().numpy(), r * exact), f"replay {r}"
            del junk
        # new buffers: the graph is captured again for them
        B2 = B.clone()
        C2 = torch.zeros_like(C)
        spmv.spmv_run(h, B2, C2)
        spmv.spmv_run(h, B2, C2)
        torch.cuda.synchronize()
        assert np.array_equal(C2.cpu().numpy(), 2 * exact)
        assert np.array_equal(C.cpu().numpy(), 4 * exact)
    finally:
        spmv.spmv_destroy(h)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_batch_precision(prec):
    import torch

    mem = _batch(count=12, seed_extra=3)
    h = spmv.spmv_create_batch([(A.row_ptr, A.col_idx, A.val, A.n_cols) for A, _ in mem], prec=prec,
                               flags=NOTUNE)
    try:
        xs = np.concatenate([x for _, x in mem])
        B = to_dev(xs, prec)
        C = to_dev(np.zeros(sum(A.n_rows for A, _ in mem)), prec)
        spmv.spmv_run(h, B, C)
        torch.cuda.synchronize()
        got = C.cpu().numpy().astype(np.float64)
    finally:
        spmv.spmv_destroy(h)
    off = 0
    for A, x in mem:
        sl = slice(off, off + A.n_rows)
        ref, den = oracle_ref(A, x)
        assert_close(got[sl], ref, den, prec_bounds(prec, 7)[0], f"{prec} member at {off}")
        off += A.n_rows


# ---------------------------------------------------------------------------- a10

def test_tuner_and_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("SPMV_TUNE_CACHE", str(tmp_path / "tune.json"))
    A, x = mats()["irregular"]
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols)
    try:
        spmv.spmv_tune(h, 1)
        plan = spmv.spmv_get_plan(h)
        spmv.spmv_tune(h, 8)
    finally:
        spmv.spmv_destroy(h)
    text = (tmp_path / "tune.json").read_text()
    assert "|k1|main|" in text and "|k8|block|" in text
    # a new handle with the same statistics starts from the cached plan
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols)
    try:
        assert spmv.spmv_get_plan(h) == plan
    finally:
        spmv.spmv_destroy(h)
    ref, den = oracle_ref(A, x)
    assert_close(gpu_spmv(A, x, flags=0), ref, den, FP64_TOL, "tuned plan")
    # split and batch handles tune too
    a, s = _split_handles(A, gen.halo_begin(A.n_cols), flags=0)
    try:
        spmv.spmv_tune(s, 1)
        assert spmv.spmv_get_plan(s, spmv.SPMV_PART_NONLOCAL)["kernel"] in (1, 2, 4)
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)
    mem = _batch(count=8, seed_extra=4)
    hb = spmv.spmv_create_batch([(M.row_ptr, M.col_idx, M.val, M.n_cols) for M, _ in mem])
    try:
        spmv.spmv_tune(hb, 1)
    finally:
        spmv.spmv_destroy(hb)


def test_set_plan_validation():
    A, _ = mats()["irregular"]
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        for bad in (dict(kernel=7), dict(kernel=0), dict(kernel=3), dict(kernel=4, tile_items=4),
                    dict(tile_items=5), dict(lanes=3), dict(block_kt=2),
                    dict(tiles_per_group=0), dict(tiles_per_group=65), dict(panels=3),
                    dict(kernel=6, tile_items=8), dict(kernel=6, tile_items=1, panels=2)):
            with pytest.raises(spmv.SpmvError):
                spmv.spmv_set_plan(h, **bad)
        with pytest.raises(spmv.SpmvError):
            spmv.spmv_get_plan(h, spmv.SPMV_PART_NONLOCAL)
    finally:
        spmv.spmv_destroy(h)
    # a destroyed handle is refused without being dereferenced
    assert spmv.load().spmv_run(spmv.ctypes.c_void_p(1), None, None, None, None) == spmv.SPMV_ERR_STATE


def test_sorted_blocks_need_a_part_covering_all_rows():
    A, x = mats()["irregular"]
    sb = dict(kernel=spmv.SPMV_KERNEL_SORTED_BLOCKS, tile_items=2)
    a, s = _split_handles(A, gen.halo_begin(A.n_cols))
    try:
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_set_plan(s, spmv.SPMV_PART_NONLOCAL, **sb)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
        spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, **sb)  # the local part covers all rows
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)
    mem = _batch(count=3, seed_extra=4)
    hb = spmv.spmv_create_batch([(M.row_ptr, M.col_idx, M.val, M.n_cols) for M, _ in mem], flags=NOTUNE)
    try:
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_set_plan(hb, **sb)
        assert ei.value.status == spmv.SPMV_ERR_UNSUPPORTED
    finally:
        spmv.spmv_destroy(hb)


# ---------------------------------------------------------------------------- probes

def test_probes():
    import time

    import torch

    n = (1 << 20) + 1
    src = torch.randn(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    spmv.spmv_probe_copy(dst, src)
    a = torch.empty_like(src)
    c = torch.randn(n, dtype=torch.float64, device="cuda")
    spmv.spmv_probe_triad(a, src, c, 3.0)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    assert torch.allclose(a, src + 3.0 * c, rtol=0, atol=1e-12)
    sums = torch.full((spmv.read_sums_needed(n),), float("nan"), dtype=torch.float64, device="cuda")
    spmv.spmv_probe_read(src, sums)
    torch.cuda.synchronize()
    nb = ((n // 2) + 1023) // 1024
    assert torch.allclose(sums[:nb].sum(), src[: 2 * (n // 2)].sum(), rtol=1e-9)
    t0 = time.perf_counter()
    spmv.spmv_probe_spin(20_000_000)  # 20 ms
    torch.cuda.synchronize()
    assert time.perf_counter() - t0 >= 0.015
    # atomic adds: every one lands (integer sums of 1.0 are exact)
    for scattered in (False, True):
        C = torch.zeros(1 << 16, dtype=torch.float64, device="cuda")
        made = spmv.spmv_probe_atomic(C, scattered, 3)
        torch.cuda.synchronize()
        assert made == spmv.ATOMIC_THREADS * 3 and C.sum().item() == float(made)
        if not scattered:
            # each wavefront covers 64 consecutive slots per step: all slots are hit equally
            assert torch.all(C == C[0]).item()
    with pytest.raises(spmv.SpmvError):
        spmv.spmv_probe_atomic(torch.zeros(100, dtype=torch.float64, device="cuda"), False, 1)
    with pytest.raises(spmv.SpmvError):
        spmv.spmv_probe_atomic(torch.zeros(64, dtype=torch.float64, device="cuda"), False, 0)


@pytest.mark.parametrize("width", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("remap", [0, 1])
def test_gather_probe_sums(width, remap):
    """The gather probe's per-workgroup sums add up to the sum of the gathered
    rows (integer values: exact in any order), including a ragged last
    workgroup, and out-of-range indices are clamped to the first or last row."""
    import torch

    rng = np.random.default_rng(77 + width)
    n_rows = 5000
    src = rng.integers(-50, 51, size=n_rows * width).astype(np.float64)
    idx = rng.integers(0, n_rows, size=30_011).astype(np.int32)
    idx[:3] = [-7, n_rows, 2 ** 31 - 1]  # clamped to rows 0, n_rows - 1, n_rows - 1
    S = torch.from_numpy(src).cuda()
    I = torch.from_numpy(idx).cuda()
    sums = spmv.spmv_probe_gather(S, I, width, bool(remap))
    torch.cuda.synchronize()
    rows = src.reshape(n_rows, width)
    want = rows[np.clip(idx.astype(np.int64), 0, n_rows - 1)].sum()
    assert sums.numel() == spmv.gather_sums_needed(idx.size, width)
    assert float(sums.sum().item()) == float(want)

