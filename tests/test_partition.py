"""One process's share, generalised to P processes on the host (no GPU):
rows are cut into P nnz-balanced shares, each share owns the columns with
its own row numbers and receives every other column it uses (its halo).
Renumbering the share's columns so that the owned ones come first turns the
halo into a column tail, which is exactly the split of Sect. 3.4.  The sum
over shares of (local part + nonlocal part) must then reproduce the full
product bit for bit on integer data, and, for a symmetric matrix, what each
share sends (Sect. 3.3) must be what the other shares receive."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from workloads import gen


def shares(row_ptr, P):
    nnz = row_ptr[-1]
    cuts = np.searchsorted(row_ptr, [p * nnz // P for p in range(P + 1)], side="left")
    cuts[0], cuts[-1] = 0, row_ptr.size - 1
    return np.maximum.accumulate(cuts)


def share_matrix(A, r0, r1):
    """Rows [r0, r1) with columns renumbered: owned columns r0..r1-1 first,
    then the halo columns in ascending order.  Returns (row_ptr, col, val,
    h, halo_columns)."""
    rp = A.row_ptr[r0:r1 + 1] - A.row_ptr[r0]
    cols = A.col_idx[A.row_ptr[r0]:A.row_ptr[r1]]
    vals = A.val[A.row_ptr[r0]:A.row_ptr[r1]]
    owned = (cols >= r0) & (cols < r1)
    halo = np.unique(cols[~owned])
    new = np.empty_like(cols)
    new[owned] = cols[owned] - r0
    new[~owned] = (r1 - r0) + np.searchsorted(halo, cols[~owned])
    return rp.astype(np.int32), new.astype(np.int32), vals, r1 - r0, halo


def integer_symmetric(n, rng):
    A = gen.irregular_symmetric(n, max(n // 16, 1), rng)
    vals = rng.integers(-9, 10, size=A.nnz).astype(np.float64)
    # symmetric integer values: value of (i, j) and (j, i) from the smaller index pair
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
    key = np.minimum(rows, A.col_idx).astype(np.int64) * n + np.maximum(rows, A.col_idx)
    _, first = np.unique(key, return_index=True)
    lut = dict(zip(key[first], vals[first]))
    A.val = np.array([lut[k] for k in key], dtype=np.float64)
    return A


@pytest.mark.parametrize("P", [1, 2, 3, 5, 8])
def test_shares_sum_to_full_product(P):
    rng = gen.rng_for(950, P)
    A = integer_symmetric(3000, rng)
    x = gen.integer_vector(A.n_cols, rng)
    full = oracle.spmv(A.row_ptr, A.col_idx, A.val, x)
    cuts = shares(A.row_ptr, P)
    got = np.full(A.n_rows, np.nan)
    received, sent = {}, {}
    for p in range(P):
        r0, r1 = int(cuts[p]), int(cuts[p + 1])
        rp, col, val, h, halo = share_matrix(A, r0, r1)
        Bp = np.concatenate([x[r0:r1], x[halo]])
        parts = oracle.split(rp, col, val, h)
        assert np.all(parts["loc_col"] < h) and np.all(parts["nl_col"] >= h)
        got[r0:r1] = oracle.spmv_split(parts, Bp)
        received[p] = halo
        # what this share sends: its rows with an entry outside its own columns
        sent[p] = oracle.send_list_symmetric(rp, col, h) + r0
    assert np.array_equal(got, full)
    # for a symmetric matrix, what share q sends is what the other shares receive from it
    for q in range(P):
        r0, r1 = int(cuts[q]), int(cuts[q + 1])
        wanted = np.unique(np.concatenate([received[p][(received[p] >= r0) & (received[p] < r1)]
                                           for p in range(P) if p != q] + [np.zeros(0, np.int64)]))
        assert np.array_equal(sent[q], wanted)
