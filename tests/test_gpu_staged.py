"""Staged stream kernel (SPMV_KERNEL_STAGED): each tile's B columns merged
into at most four runs and read from LDS.

The run table is checked on the host against the tiles' own columns (every
column covered, runs tight, ascending and far enough apart, LDS slots
contiguous, within the budget; a tile left to gather must really not fit),
then the products are compared with the oracle on stencils, where most tiles
are staged, and on matrices where tiles fall back, in every precision, for
split handles (local part next to a NaN receive area, nonlocal part) and with
diagonal panels, and over the tiles of a batch.  Integer data must match
bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import (FP64_TOL, assert_close, gpu_spmv, oracle_ref, prec_bounds, rounded_inputs,
                      to_dev)
from paper_1106_5908_amd import spmv
from workloads import gen

pytestmark = pytest.mark.gpu

NOTUNE = spmv.SPMV_FLAG_NO_TUNE_CACHE
GAP = 16          # columns a run may skip
MAX_RUNS = 4
STAGE_BYTES = 12288


def staged(e=16, **kw):
    return dict(kernel=spmv.SPMV_KERNEL_STAGED, tile_items=e, **kw)


def _mats():
    rng = gen.rng_for(40, 0)
    out = {
        "27pt-30": gen.workload_c2(n=30)[0],
        "7pt-40": gen.laplace_7pt_3d(40),
        "5pt-300": gen.laplace_5pt_2d(300),
        "irregular": gen.workload_c3(N=60_000)[0],
        "random": gen.random_crs(7000, 9000, rng, max_len=30),
    }
    # stencil rows with a long row and empty rows in between
    A = gen.laplace_5pt_2d(200)
    counts = np.diff(A.row_ptr).astype(np.int64)
    counts[5000] = 0
    counts[5001:5003] = 0
    cols = [A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]] for i in range(A.n_rows)]
    cols[5000] = np.zeros(0, np.int32)
    cols[5001] = np.zeros(0, np.int32)
    cols[5002] = np.zeros(0, np.int32)
    cols[20000] = np.arange(0, 40000, 7, dtype=np.int32)[:5000]
    counts[20000] = cols[20000].size
    allc = np.concatenate(cols)
    vals = rng.standard_normal(allc.size)
    out["5pt-gaps-long"] = gen._finish(A.n_rows, A.n_cols, counts, allc, vals)
    return out


MATS = None


def mats():
    global MATS
    if MATS is None:
        MATS = _mats()
    return MATS


def minimal_runs(cols):
    """Ascending runs of the distinct columns, merged across gaps <= GAP."""
    runs = []
    for c in np.unique(cols):
        if runs and c - runs[-1][1] <= GAP:
            runs[-1][1] = c + 1
        elif runs and c < runs[-1][1]:
            continue
        else:
            runs.append([int(c), int(c) + 1])
    return runs


def check_table(A, h, e, x_bytes):
    tiles = spmv.spmv_export(h, spmv.SPMV_ARR_TILES)
    table = spmv.spmv_export(h, spmv.SPMV_ARR_RUNS)
    n_tiles = tiles.shape[0] - 1
    assert table.shape == (n_tiles, 12)
    budget = STAGE_BYTES // x_bytes
    cap = 256 * e - 4
    staged_count = 0
    for t in range(n_tiles):
        p0, p1 = int(tiles[t, 1]), int(tiles[t + 1, 1])
        assert tiles[t, 1] == A.row_ptr[tiles[t, 0]]
        cols = A.col_idx[p0:p1]
        row = table[t]
        nr, L = int(row[0]), int(row[1])
        want = minimal_runs(cols) if p1 > p0 else []
        fits = (0 < p1 - p0 <= cap and len(want) <= MAX_RUNS and
                sum(b - a for a, b in want) <= budget)
        if nr == 0:
            assert not fits, f"tile {t} fits but gathers"
            continue
        assert fits, f"tile {t} staged but does not fit"
        staged_count += 1
        assert 1 <= nr <= MAX_RUNS and 1 <= L <= budget
        starts = [int(v) for v in row[2:2 + nr]]
        deltas = [int(v) for v in row[6:6 + nr]]
        assert [r[0] for r in want] == starts
        lens = [b - a for a, b in want]
        assert sum(lens) == L
        slot = 0
        for r in range(nr):
            assert starts[r] + deltas[r] == slot  # slots contiguous from 0
            slot += lens[r]
        # every column lies in a run and maps into [0, L)
        idx = np.searchsorted(np.array(starts), cols, side="right") - 1
        assert (idx >= 0).all()
        ends = np.array(starts) + np.array(lens)
        assert (cols < ends[idx]).all()
        assert ((cols + np.array(deltas)[idx] >= 0) & (cols + np.array(deltas)[idx] < L)).all()
        assert (row[2 + nr:6] == 0).all() and (row[6 + nr:] == 0).all()
    return staged_count


@pytest.mark.parametrize("e", [8, 16])
@pytest.mark.parametrize("name", ["27pt-30", "7pt-40", "5pt-300", "irregular", "random",
                                  "5pt-gaps-long"])
def test_run_table(name, e):
    A = mats()[name]
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        spmv.spmv_set_plan(h, **staged(e))
        n = check_table(A, h, e, 8)
        assert spmv.spmv_get_info(h)["n_staged_tiles"] == n
        # tiles of these stencils read at most four short column ranges (the
        # 7-point one at 16 entries per lane spans 512 rows: three ranges of
        # over 512 columns, more than 12 KB, so its tiles gather)
        if (name, e) in (("27pt-30", 8), ("27pt-30", 16), ("5pt-300", 8), ("5pt-300", 16),
                         ("7pt-40", 8)):
            assert n > 0.8 * (spmv.spmv_export(h, spmv.SPMV_ARR_TILES).shape[0] - 1)
    finally:
        spmv.spmv_destroy(h)


def test_run_table_f32_budget():
    """FP32 B values: twice the columns fit in the same LDS bytes."""
    A = mats()["5pt-300"]
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, prec="f32", flags=NOTUNE)
    try:
        spmv.spmv_set_plan(h, **staged(16))
        assert check_table(A, h, 16, 4) > 0
    finally:
        spmv.spmv_destroy(h)


PLANS = [staged(e, nontemporal=nt, xcd_remap=rm) for e in (8, 16) for nt in (0, 1) for rm in (0, 1)]


def _pid(p):
    return "-".join(f"{k}{v}" for k, v in p.items())


@pytest.mark.parametrize("plan", PLANS, ids=_pid)
@pytest.mark.parametrize("name", ["27pt-30", "7pt-40", "5pt-300", "irregular", "random",
                                  "5pt-gaps-long"])
def test_parity(name, plan):
    A = mats()[name]
    x = gen.uniform_vector(A.n_cols, gen.rng_for(41, 1))
    c0 = gen.uniform_vector(A.n_rows, gen.rng_for(41, 2))
    ref, den = oracle_ref(A, x, c0)
    assert_close(gpu_spmv(A, x, c0, plan=plan), ref, den, FP64_TOL, f"{name} {plan}")


@pytest.mark.parametrize("e", [8, 16])
@pytest.mark.parametrize("name", ["27pt-30", "5pt-gaps-long", "random"])
def test_integer_bit_exact_and_base(name, e):
    A0 = mats()[name]
    rng = gen.rng_for(42, e)
    A = gen.CRS(A0.n_rows, A0.n_cols, A0.row_ptr, A0.col_idx,
                rng.integers(-8, 9, size=A0.nnz).astype(np.float64))
    x = gen.integer_vector(A.n_cols, rng)
    c0 = gen.integer_vector(A.n_rows, rng)
    ref = oracle.spmv(A.row_ptr, A.col_idx, A.val, x, c0)
    for base in (0, 1):
        got = gpu_spmv(A, x, c0, plan=staged(e), base=base)
        assert np.array_equal(got, ref), base
    # two calls accumulate: C0 + 2 A x
    got2 = gpu_spmv(A, x, c0, plan=staged(e), runs=2)
    assert np.array_equal(got2, oracle.spmv(A.row_ptr, A.col_idx, A.val, x, ref))


@pytest.mark.parametrize("prec", ["f32", "bf16", "f32f64"])
@pytest.mark.parametrize("e", [8, 16])
def test_precisions(prec, e):
    A = mats()["27pt-30"]
    x = gen.uniform_vector(A.n_cols, gen.rng_for(43, 1))
    c0 = gen.uniform_vector(A.n_rows, gen.rng_for(43, 2))
    got = gpu_spmv(A, x, c0, prec=prec, plan=staged(e))
    v, xr = rounded_inputs(A, x, prec)
    if prec != "f32f64":
        c0 = c0.astype(np.float32).astype(np.float64)
    ref = oracle.spmv(A.row_ptr, A.col_idx, v, xr, c0)
    den = oracle.abs_spmv(A.row_ptr, A.col_idx, v, xr, c0)
    _, b_same = prec_bounds(prec, int(np.diff(A.row_ptr).max()))
    assert_close(got, ref, den, b_same, f"{prec} staged E{e}")


@pytest.mark.parametrize("panels", [2, 4])
def test_with_panels(panels):
    A = mats()["27pt-30"]
    x = gen.uniform_vector(A.n_cols, gen.rng_for(44, 1))
    ref, den = oracle_ref(A, x)
    assert_close(gpu_spmv(A, x, plan=staged(16, panels=panels)), ref, den, FP64_TOL,
                 f"staged panels {panels}")


def test_split_local_never_reads_halo_and_nonlocal():
    """Stencil split with the last planes as halo: the staged local part
    must not read the receive area (NaN there, no copy) and the staged
    nonlocal part (a row list) must give the oracle's rows."""
    import torch

    A = mats()["27pt-30"]
    x = gen.uniform_vector(A.n_cols, gen.rng_for(45, 1))
    h_begin = A.n_cols - 2 * 900
    a = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    s = spmv.spmv_split_local_nonlocal(a, h_begin)
    try:
        spmv.spmv_set_plan(s, spmv.SPMV_PART_MAIN, **staged(16))
        spmv.spmv_set_plan(s, spmv.SPMV_PART_NONLOCAL, **staged(8))
        Bh = x.copy()
        Bh[h_begin:] = np.nan
        B = to_dev(Bh, "f64")
        C = to_dev(np.zeros(A.n_rows), "f64")
        spmv.spmv_run(s, B, C)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        parts = oracle.split(A.row_ptr, A.col_idx, A.val, h_begin)
        only_local = np.ones(A.n_rows, bool)
        only_local[parts["nl_rows"]] = False
        assert np.isnan(got[parts["nl_rows"]]).all()
        ref = oracle.spmv(parts["loc_row_ptr"], parts["loc_col"], parts["loc_val"], x)
        den = oracle.abs_spmv(parts["loc_row_ptr"], parts["loc_col"], parts["loc_val"], x)
        assert_close(got[only_local], ref[only_local], den[only_local], FP64_TOL, "local rows")
        # with the halo present the whole product matches
        B = to_dev(x, "f64")
        C = to_dev(np.zeros(A.n_rows), "f64")
        spmv.spmv_run(s, B, C)
        torch.cuda.synchronize()
        ref, den = oracle_ref(A, x)
        assert_close(C.cpu().numpy(), ref, den, FP64_TOL, "split staged")
    finally:
        spmv.spmv_destroy(s)
        spmv.spmv_destroy(a)


def test_graph_capture_replays():
    """The run table is built by set_plan, so spmv_run only enqueues work and
    can be captured; every replay adds A x again."""
    import torch

    A = mats()["27pt-30"]
    rng = gen.rng_for(46, 0)
    A = gen.CRS(A.n_rows, A.n_cols, A.row_ptr, A.col_idx,
                rng.integers(-4, 5, size=A.nnz).astype(np.float64))
    x = gen.integer_vector(A.n_cols, rng)
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        spmv.spmv_set_plan(h, **staged(16))
        B = to_dev(x, "f64")
        C = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            spmv.spmv_run(h, B, C)
        torch.cuda.synchronize()
        ax = oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
        for r in range(1, 4):
            g.replay()
            torch.cuda.synchronize()
            junk = torch.ones(1 << 20, device="cuda").cumsum(0)  # unrelated eager work
            torch.cuda.synchronize()
            del junk
            assert np.array_equal(C.cpu().numpy(), r * ax), r
    finally:
        spmv.spmv_destroy(h)


def test_validation():
    A = mats()["5pt-300"]
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols, flags=NOTUNE)
    try:
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_set_plan(h, **staged(4))
        assert ei.value.status == spmv.SPMV_ERR_INVALID_ARG
    finally:
        spmv.spmv_destroy(h)
    b = spmv.spmv_create_batch([(A.row_ptr, A.col_idx, A.val, A.n_cols)] * 2)
    try:
        with pytest.raises(spmv.SpmvError) as ei:
            spmv.spmv_set_plan(b, **staged(4))
        assert ei.value.status == spmv.SPMV_ERR_INVALID_ARG
        with pytest.raises(spmv.SpmvError):
            spmv.spmv_export(b, spmv.SPMV_ARR_RUNS)
    finally:
        spmv.spmv_destroy(b)


@pytest.mark.parametrize("e", [8, 16])
def test_batch_members(e):
    """A batch of stencils of many sizes plus a random member: most batch
    tiles are staged, and every member's rows match the oracle."""
    import torch

    rng = gen.rng_for(47, e)
    mem = [gen.laplace_5pt_2d(int(n)) for n in (17, 64, 150, 301)]
    mem += [gen.laplace_7pt_3d(int(n)) for n in (9, 20, 33)]
    mem += [gen.stencil_27pt_3d(12), gen.random_crs(900, 1300, rng, max_len=9)]
    xs = [gen.uniform_vector(A.n_cols, rng) for A in mem]
    c0 = gen.uniform_vector(sum(A.n_rows for A in mem), rng)
    h = spmv.spmv_create_batch([(A.row_ptr, A.col_idx, A.val, A.n_cols) for A in mem], flags=NOTUNE)
    try:
        spmv.spmv_set_plan(h, **staged(e))
        info = spmv.spmv_get_info(h)
        assert info["n_staged_tiles"] > 0.5 * info["n_tiles"], info
        B = to_dev(np.concatenate(xs), "f64")
        C = to_dev(c0, "f64")
        spmv.spmv_run(h, B, C)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
    finally:
        spmv.spmv_destroy(h)
    off = 0
    for A, x in zip(mem, xs):
        sl = slice(off, off + A.n_rows)
        ref, den = oracle_ref(A, x, c0[sl])
        assert_close(got[sl], ref, den, FP64_TOL, f"member at {off}")
        off += A.n_rows


def test_cached_staged_plan(tmp_path, monkeypatch):
    """A staged plan read from the tuning cache is prepared at creation (run
    table built), so the first spmv_run already stages and gives the
    oracle's result."""
    import json

    monkeypatch.setenv("SPMV_TUNE_CACHE", str(tmp_path / "tune.json"))
    A = mats()["27pt-30"]
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols)
    try:
        spmv.spmv_tune(h, 1)
    finally:
        spmv.spmv_destroy(h)
    cache = json.loads((tmp_path / "tune.json").read_text())
    keys = [k for k in cache if "|k1|main|" in k]
    assert len(keys) == 1
    cache[keys[0]] = dict(kernel=spmv.SPMV_KERNEL_STAGED, tile_items=16, lanes=32, nontemporal=1,
                          xcd_remap=1, block_kt=0, tiles_per_group=1, panels=1)
    (tmp_path / "tune.json").write_text(json.dumps(cache))
    h = spmv.spmv_create_crs(A.row_ptr, A.col_idx, A.val, A.n_cols)
    try:
        assert spmv.spmv_get_plan(h)["kernel"] == spmv.SPMV_KERNEL_STAGED
        assert spmv.spmv_get_info(h)["n_staged_tiles"] > 0
    finally:
        spmv.spmv_destroy(h)
    x = gen.uniform_vector(A.n_cols, gen.rng_for(48, 0))
    ref, den = oracle_ref(A, x)
    assert_close(gpu_spmv(A, x, flags=0), ref, den, FP64_TOL, "cached staged plan")


@pytest.mark.parametrize("plan", [staged(16), staged(8), dict(kernel=spmv.SPMV_KERNEL_STREAM,
                                                              tile_items=16)], ids=_pid)
def test_tiles_without_entries(plan):
    """More than 512 empty rows in a row make tiles that hold no entry at all
    (a tile never spans more than 512 rows): they leave C untouched, signed
    zeros included, and the stencil rows around them match the oracle."""
    S = gen.laplace_5pt_2d(60)
    n_gap = 3000
    counts = np.concatenate([np.diff(S.row_ptr), np.zeros(n_gap, np.int64), np.diff(S.row_ptr)])
    cols = np.concatenate([S.col_idx, S.col_idx])
    vals = np.concatenate([S.val, -S.val])
    A = gen._finish(counts.size, S.n_cols, counts, cols, vals)
    x = gen.uniform_vector(A.n_cols, gen.rng_for(49, 0))
    c0 = gen.uniform_vector(A.n_rows, gen.rng_for(49, 1))
    c0[S.n_rows:S.n_rows + n_gap:2] = -0.0
    c0[S.n_rows + 1:S.n_rows + n_gap:2] = 0.0
    got = gpu_spmv(A, x, c0, plan=plan)
    gap = slice(S.n_rows, S.n_rows + n_gap)
    assert np.array_equal(got[gap], c0[gap]) and np.array_equal(np.signbit(got[gap]),
                                                               np.signbit(c0[gap]))
    ref, den = oracle_ref(A, x, c0)
    assert_close(got, ref, den, FP64_TOL, f"empty tiles {plan}")
