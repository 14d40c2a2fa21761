"""Property-based parity: random CRS matrices whose row-length mix puts row
boundaries everywhere relative to the tiles (empty rows, single entries,
rows of exactly a tile, rows longer than a tile, duplicates, unsorted
columns, rectangular shapes), random plans of every kernel family, every
precision mode and both index bases, each compared with the oracle.  Integer
data must match bit for bit; random data to the FP64 bound or the
reduced-precision bounds."""
from __future__ import annotations

import os

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from gpu_util import FP64_TOL, assert_close, gpu_spmv, prec_bounds, rounded_inputs
from workloads import gen

pytestmark = pytest.mark.gpu

# examples per test; the default run draws the same examples every time
# (derandomized), SPMV_RANDOM_EXAMPLES asks for a longer, freshly seeded search
N_FP64 = int(os.environ.get("SPMV_RANDOM_EXAMPLES", "60"))
N_REDUCED = max(1, N_FP64 // 2)
FIXED = "SPMV_RANDOM_EXAMPLES" not in os.environ

PLANS = st.one_of(
    st.builds(lambda e, nt, rm, tpw: dict(kernel=1, tile_items=e, nontemporal=nt, xcd_remap=rm,
                                          tiles_per_group=tpw),
              st.sampled_from([4, 8, 16]), st.integers(0, 1), st.integers(0, 1),
              st.sampled_from([1, 1, 2, 5])),
    st.builds(lambda e, k: dict(kernel=1, tile_items=e, panels=k),
              st.sampled_from([4, 8]), st.sampled_from([2, 4, 8])),
    st.builds(lambda l: dict(kernel=2, lanes=l), st.sampled_from([2, 4, 8, 16, 32, 64])),
    st.builds(lambda e, nt: dict(kernel=4, tile_items=e, nontemporal=nt),
              st.sampled_from([8, 16]), st.integers(0, 1)),
)


@st.composite
def matrices(draw):
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    n_rows = draw(st.integers(0, 3000))
    n_cols = draw(st.integers(0, 5000))
    # row lengths from a mix that straddles tile sizes (256 * 4 .. 256 * 16 entries)
    kinds = rng.integers(0, 6, size=n_rows)
    lens = np.select([kinds == 0, kinds == 1, kinds == 2, kinds == 3, kinds == 4],
                     [np.zeros(n_rows, int), np.ones(n_rows, int), rng.integers(2, 40, n_rows),
                      rng.choice([1020, 1021, 1024, 2044, 2048, 4092, 4096], n_rows),
                      rng.integers(4097, 9000, n_rows)],
                     rng.integers(0, 12, n_rows))
    # keep the total modest: long rows are rare
    keep_long = rng.random(n_rows) < 0.01
    lens = np.where((lens > 40) & ~keep_long, rng.integers(0, 12, n_rows), lens)
    if n_cols == 0:
        lens[:] = 0
    nnz = int(lens.sum())
    cols = rng.integers(0, max(n_cols, 1), size=nnz).astype(np.int32)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    for i in np.flatnonzero(lens >= 2)[:50]:
        cols[rp[i + 1] - 1] = cols[rp[i]]  # a duplicate column in some rows
    integer = draw(st.booleans())
    vals = (rng.integers(-8, 9, size=nnz).astype(np.float64) if integer
            else rng.standard_normal(nnz))
    x = (rng.integers(-8, 9, size=n_cols).astype(np.float64) if integer
         else rng.uniform(-1, 1, size=n_cols))
    c0 = (rng.integers(-8, 9, size=n_rows).astype(np.float64) if integer
          else rng.uniform(-1, 1, size=n_rows))
    return gen.CRS(n_rows, n_cols, rp, cols, vals), x, c0, integer


@settings(max_examples=N_FP64, deadline=None, derandomize=FIXED,
          suppress_health_check=list(HealthCheck))
@given(m=matrices(), plan=PLANS, base=st.integers(0, 1))
def test_random_fp64(m, plan, base):
    A, x, c0, integer = m
    print(f"case fp64 {A.n_rows}x{A.n_cols} nnz={A.nnz} plan={plan} base={base}", flush=True)
    got = gpu_spmv(A, x, c0, plan=plan, base=base)
    ref, den = oracle.spmv(A.row_ptr, A.col_idx, A.val, x, c0), None
    if integer:
        assert np.array_equal(got, ref), plan
    else:
        den = oracle.abs_spmv(A.row_ptr, A.col_idx, A.val, x, c0)
        assert_close(got, ref, den, FP64_TOL, str(plan))


@settings(max_examples=N_REDUCED, deadline=None, derandomize=FIXED,
          suppress_health_check=list(HealthCheck))
@given(m=matrices(), plan=PLANS, prec=st.sampled_from(["f32", "bf16", "f32f64"]))
def test_random_reduced_precision(m, plan, prec):
    A, x, c0, integer = m
    print(f"case {prec} {A.n_rows}x{A.n_cols} nnz={A.nnz} plan={plan}", flush=True)
    got = gpu_spmv(A, x, c0, prec=prec, plan=plan)
    v, xr = rounded_inputs(A, x, prec)
    if prec != "f32f64":
        c0 = c0.astype(np.float32).astype(np.float64)  # C lives in float32 in these modes
    ref = oracle.spmv(A.row_ptr, A.col_idx, v, xr, c0)
    den = oracle.abs_spmv(A.row_ptr, A.col_idx, v, xr, c0)
    n = int(np.diff(A.row_ptr).max()) if A.n_rows else 1
    _, b_same = prec_bounds(prec, n)
    assert_close(got, ref, den, b_same, f"{prec} {plan}")
