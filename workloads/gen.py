"""Seeded generators for the CRS matrices and vectors used by tests and bench.

Every array produced here is a plain host array in the CRS layout of the
paper (Sect. 1.2, "Sparse matrix-vector multiplication and node-level
performance model"): ``row_ptr`` (N_r+1 row starts), ``col_idx`` (original
column of each stored entry) and ``val`` (entries row by row), here 0-based
with int32 indices and float64 values.

The workload recipes stand in for the paper's test matrices, which are not
available (Sect. 1.3.1): a 2D 5-point Laplacian (small correctness case), a 3D
27-point stencil (regular, N_nzr ~ 27, the bandwidth case), an irregular
banded symmetric matrix with geometric row lengths (stand-in for the
Holstein-Hubbard matrix HMeP, N_nzr ~ 15), and batches of 2D 5-point / 3D
7-point stencils (stand-in for the sAMG Poisson matrix, N_nzr ~ 7).

Randomness: every generator takes a ``numpy.random.Generator``; the canonical
seeds are ``rng_for(config, part)`` built from ``SeedSequence([1106, config,
part])``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ROOT_SEED = 1106

# part identifiers for rng_for(); fixed so every consumer draws the same arrays
PART_MATRIX = 0
PART_X = 1
PART_C0 = 2
PART_HALO = 3
PART_BLOCK = 4
PART_BATCH = 5


def rng_for(config: int, part: int, extra: int = 0) -> np.random.Generator:
    """PCG64 generator for (config, part[, extra]) under the root seed 1106."""
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, config, part, extra]))


@dataclasses.dataclass
class CRS:
    """A CRS matrix on the host: 0-based int32 indices, float64 values."""

    n_rows: int
    n_cols: int
    row_ptr: np.ndarray  # int32 [n_rows+1]
    col_idx: np.ndarray  # int32 [nnz]
    val: np.ndarray      # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def stats(self) -> dict:
        rl = self.row_lengths()
        return {
            "n_rows": self.n_rows,
            "n_cols": self.n_cols,
            "nnz": self.nnz,
            "mean": float(rl.mean()) if rl.size else 0.0,
            "max": int(rl.max()) if rl.size else 0,
            "p50": float(np.percentile(rl, 50)) if rl.size else 0.0,
            "p99": float(np.percentile(rl, 99)) if rl.size else 0.0,
        }


def _finish(n_rows, n_cols, counts, cols, vals) -> CRS:
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32")
    return CRS(n_rows, n_cols, row_ptr.astype(np.int32),
               np.ascontiguousarray(cols, dtype=np.int32),
               np.ascontiguousarray(vals, dtype=np.float64))


# --------------------------------------------------------------------------
# Structured stencils (Dirichlet boundaries: missing neighbours are dropped)
# --------------------------------------------------------------------------

def _stencil_from_coords(coords, dims, offsets, n_points, diag, off, perturb, rng):
    """Build a stencil matrix on the first ``n_points`` points of a
    lexicographic grid (x fastest).  ``coords`` is a list of per-axis index
    arrays for the points, ``offsets`` a list of per-axis offset tuples sorted
    so that the linear column index increases with the offset.  Neighbours
    outside the grid or with linear index >= n_points are dropped."""
    ndim = len(dims)
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    lin = np.arange(n_points, dtype=np.int64)
    cols_all = []
    mask_all = []
    for o in offsets:
        ok = np.ones(n_points, dtype=bool)
        step = 0
        for a in range(ndim):
            if o[a]:
                c = coords[a] + o[a]
                ok &= (c >= 0) & (c < dims[a])
            step += o[a] * strides[a]
        col = lin + step
        ok &= (col >= 0) & (col < n_points)
        cols_all.append(col)
        mask_all.append(ok)
    cols2 = np.stack(cols_all, axis=1)
    mask2 = np.stack(mask_all, axis=1)
    is_diag = np.array([all(v == 0 for v in o) for o in offsets])
    vals2 = np.where(is_diag[None, :], diag, off)
    counts = mask2.sum(axis=1)
    cols = cols2[mask2]
    vals = np.broadcast_to(vals2, mask2.shape)[mask2].astype(np.float64)
    if perturb:
        vals = vals + rng.uniform(-perturb, perturb, size=vals.size)
    return _finish(n_points, n_points, counts, cols, vals)


def _offsets(ndim, reach_full):
    """Offsets of a (2*1+1)^ndim box (reach_full) or of the 2*ndim+1 star,
    ordered by increasing linear index (slowest axis first)."""
    out = []
    rng_ = (-1, 0, 1)
    if ndim == 2:
        for dy in rng_:
            for dx in rng_:
                if reach_full or (abs(dx) + abs(dy) <= 1):
                    out.append((dx, dy))
    else:
        for dz in rng_:
            for dy in rng_:
                for dx in rng_:
                    if reach_full or (abs(dx) + abs(dy) + abs(dz) <= 1):
                        out.append((dx, dy, dz))
    return out


def laplace_5pt_2d(nx: int, ny: int | None = None, n_points: int | None = None,
                   diag: float = 4.0, off: float = -1.0) -> CRS:
    """2D 5-point Laplacian (4 on the diagonal, -1 on the neighbours) on an
    nx x ny grid, optionally truncated to the first ``n_points`` points."""
    ny = nx if ny is None else ny
    n = nx * ny if n_points is None else n_points
    k = np.arange(n, dtype=np.int64)
    coords = [k % nx, k // nx]
    return _stencil_from_coords(coords, (nx, ny), _offsets(2, False), n, diag, off, 0.0, None)


def laplace_7pt_3d(nx: int, ny: int | None = None, nz: int | None = None,
                   n_points: int | None = None, diag: float = 6.0, off: float = -1.0) -> CRS:
    """3D 7-point Laplacian (6 / -1), optionally truncated to ``n_points``."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz if n_points is None else n_points
    k = np.arange(n, dtype=np.int64)
    coords = [k % nx, (k // nx) % ny, k // (nx * ny)]
    return _stencil_from_coords(coords, (nx, ny, nz), _offsets(3, False), n, diag, off, 0.0, None)


def stencil_27pt_3d(n: int, diag: float = 26.0, off: float = -1.0,
                    perturb: float = 0.0, rng: np.random.Generator | None = None) -> CRS:
    """3D 27-point stencil on an n^3 grid: ``diag`` on the diagonal, ``off``
    elsewhere, each stored entry (diagonal included) plus an independent
    U[-perturb, perturb] draw when ``perturb`` > 0."""
    N = n * n * n
    k = np.arange(N, dtype=np.int64)
    coords = [k % n, (k // n) % n, k // (n * n)]
    return _stencil_from_coords(coords, (n, n, n), _offsets(3, True), N, diag, off, perturb, rng)


def truncated_stencil(n_points: int, three_d: bool) -> CRS:
    """Stencil on a truncated lexicographic grid: 2D 5-point with
    nx = ceil(sqrt(N)), or 3D 7-point with nx = ny = ceil(cbrt(N)); the first
    N points are kept and neighbours with index >= N are dropped."""
    if three_d:
        nx = int(math.ceil(round(n_points ** (1.0 / 3.0), 9)))
        while nx ** 3 < n_points:
            nx += 1
        while (nx - 1) ** 3 >= n_points:
            nx -= 1
        nz = -(-n_points // (nx * nx))
        return laplace_7pt_3d(nx, nx, nz, n_points=n_points)
    nx = math.isqrt(n_points)
    if nx * nx < n_points:
        nx += 1
    ny = -(-n_points // nx)
    return laplace_5pt_2d(nx, ny, n_points=n_points)


# --------------------------------------------------------------------------
# Irregular banded symmetric matrix (Hamiltonian stand-in)
# --------------------------------------------------------------------------

C3_P = 0.138      # Geom0(p) upper-half count; calibrated for mean row length ~13
C3_UMAX = 31


def irregular_symmetric(N: int, W: int, rng: np.random.Generator,
                        p: float = C3_P, umax: int = C3_UMAX) -> CRS:
    """Exactly symmetric banded matrix with geometric row lengths.

    Row i draws u_i = min(Geom0(p), umax) upper entries at columns uniform in
    (i, i+W]; columns >= N are dropped and duplicates merged.  Every upper
    entry (i, j) is mirrored to (j, i) with the same N(0,1) value; the
    diagonal is always stored with its own N(0,1) value.  Columns within each
    row come out sorted."""
    u = rng.geometric(p, size=N).astype(np.int64) - 1
    np.minimum(u, umax, out=u)
    rows = np.repeat(np.arange(N, dtype=np.int64), u)
    cols = rows + rng.integers(1, W + 1, size=rows.size, dtype=np.int64)
    keep = cols < N
    key = np.unique(rows[keep] * N + cols[keep])  # sorted by (row, col), merged
    del rows, cols, keep
    urow = key // N
    ucol = key - urow * N
    del key
    uval = rng.standard_normal(urow.size)
    dval = rng.standard_normal(N)
    # mirrored entries grouped by their new row; stable order keeps cols sorted
    order = np.argsort(ucol, kind="stable")
    lrow = ucol[order]
    lcol = urow[order]
    lval = uval[order]
    del order
    cnt_up = np.bincount(urow, minlength=N)
    cnt_lo = np.bincount(lrow, minlength=N)
    counts = cnt_lo + 1 + cnt_up
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    if nnz > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32")
    col_idx = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    # lower part: positions row_ptr[r] + rank within the row's lower group
    lo_start = np.cumsum(cnt_lo) - cnt_lo
    pos = row_ptr[lrow] + (np.arange(lrow.size, dtype=np.int64) - lo_start[lrow])
    col_idx[pos] = lcol
    val[pos] = lval
    del pos, lrow, lcol, lval
    # diagonal
    dpos = row_ptr[:-1] + cnt_lo
    col_idx[dpos] = np.arange(N, dtype=np.int32)
    val[dpos] = dval
    # upper part
    up_start = np.cumsum(cnt_up) - cnt_up
    pos = dpos[urow] + 1 + (np.arange(urow.size, dtype=np.int64) - up_start[urow])
    col_idx[pos] = ucol
    val[pos] = uval
    return CRS(N, N, row_ptr.astype(np.int32), col_idx, val)


def upper_triangle(A: CRS) -> CRS:
    """The entries of A with column >= row, in A's order (input of the
    symmetric-storage handle)."""
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(A.row_ptr))
    keep = A.col_idx.astype(np.int64) >= rows
    counts = np.bincount(rows[keep], minlength=A.n_rows)
    return _finish(A.n_rows, A.n_cols, counts, A.col_idx[keep], A.val[keep])


# --------------------------------------------------------------------------
# Tiny random CRS (brute-force pins and edge cases)
# --------------------------------------------------------------------------

def random_crs(n_rows: int, n_cols: int, rng: np.random.Generator, max_len: int = 8,
               empty_frac: float = 0.2, dup_frac: float = 0.2, sort_cols: bool = False,
               integer_values: bool = False, vmax: int = 8) -> CRS:
    """Small random CRS with empty rows, duplicate and unsorted columns."""
    counts = rng.integers(0, max_len + 1, size=n_rows)
    counts[rng.random(n_rows) < empty_frac] = 0
    if n_cols == 0:
        counts[:] = 0
    nnz = int(counts.sum())
    cols = rng.integers(0, max(n_cols, 1), size=nnz)
    # duplicate some entries of the same row
    rp = np.concatenate([[0], np.cumsum(counts)])
    for i in range(n_rows):
        a, b = rp[i], rp[i + 1]
        if b - a >= 2 and rng.random() < dup_frac:
            cols[b - 1] = cols[a]
        if sort_cols:
            cols[a:b] = np.sort(cols[a:b])
    if integer_values:
        vals = rng.integers(-vmax, vmax + 1, size=nnz).astype(np.float64)
    else:
        vals = rng.standard_normal(nnz)
    return _finish(n_rows, n_cols, counts, cols, vals)


def uniform_vector(n: int, rng: np.random.Generator, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return rng.uniform(lo, hi, size=n)


def integer_vector(n: int, rng: np.random.Generator, vmax: int = 16) -> np.ndarray:
    return rng.integers(-vmax, vmax + 1, size=n).astype(np.float64)


# --------------------------------------------------------------------------
# Named workloads (sizes of the benchmark configurations)
# --------------------------------------------------------------------------

C1_N = 64                    # 2D 5-point, 64 x 64
C2_N = 160                   # 3D 27-point, 160^3
C3_ROWS = 8_000_000          # irregular symmetric, band N/16
C3_HALO_FRAC = 0.06          # last 6% of columns are halo
C5_COUNT = 512
C5_NMIN, C5_NMAX = 1000, 250_000
BLOCK_KS = (4, 8, 16)


def workload_c1():
    """2D 5-point Laplacian, 64 x 64, x ~ U[-1,1], C0 = 0."""
    A = laplace_5pt_2d(C1_N)
    x = uniform_vector(A.n_cols, rng_for(1, PART_X))
    return A, x


def workload_c2(n: int = C2_N, perturb: float = 0.01):
    """3D 27-point stencil on n^3 (26 / -1) with U[-0.01,0.01] perturbation
    on every stored entry, x ~ U[-1,1]."""
    A = stencil_27pt_3d(n, perturb=perturb, rng=rng_for(2, PART_MATRIX, n))
    x = uniform_vector(A.n_cols, rng_for(2, PART_X, n))
    return A, x


def workload_c3(N: int = C3_ROWS):
    """Irregular symmetric matrix, band W = N/16, geometric row lengths."""
    A = irregular_symmetric(N, max(N // 16, 1), rng_for(3, PART_MATRIX, N))
    x = uniform_vector(A.n_cols, rng_for(3, PART_X, N))
    return A, x


def halo_begin(n_cols: int, frac: float = C3_HALO_FRAC) -> int:
    """First halo column: the last ``frac`` of the columns are halo."""
    return n_cols - int(round(frac * n_cols))


def block_rhs(n: int, k: int, config: int = 5, extra: int = 0) -> np.ndarray:
    """Row-major n x k block of right-hand sides, U[-1,1]."""
    return rng_for(config, PART_BLOCK, k * 1000 + extra).uniform(-1.0, 1.0, size=(n, k))


def batch_sizes(count: int = C5_COUNT, nmin: int = C5_NMIN, nmax: int = C5_NMAX, seed_extra: int = 0):
    """Sizes and kinds of the batched stencils: N ~ U{nmin..nmax},
    kind ~ Bernoulli(1/2) (True = 3D 7-point, False = 2D 5-point)."""
    rng = rng_for(5, PART_BATCH, seed_extra)
    sizes = rng.integers(nmin, nmax + 1, size=count)
    kinds = rng.random(count) < 0.5
    return sizes, kinds


def workload_c5_batch(count: int = C5_COUNT, nmin: int = C5_NMIN, nmax: int = C5_NMAX, seed_extra: int = 0):
    """List of (CRS, x) for the batched stencils."""
    sizes, kinds = batch_sizes(count, nmin, nmax, seed_extra)
    out = []
    for m, (n, three_d) in enumerate(zip(sizes, kinds)):
        A = truncated_stencil(int(n), bool(three_d))
        x = uniform_vector(A.n_cols, rng_for(5, PART_X, seed_extra * 100000 + m))
        out.append((A, x))
    return out


__all__ = [n for n in dir() if not n.startswith("_")]
