"""Pins of the CPU oracle against facts that do not come from the oracle.

Each ``check_*`` function takes a bound oracle (``oracle.Oracle``) and raises
AssertionError when the oracle disagrees with something the paper or the
mathematics fixes: closed forms of stencil operators, exact rational
arithmetic on tiny matrices, hand-worked split examples and exhaustive
enumerations of the rounding targets.  ``run_all`` runs every check; the
test suite runs it against the real oracle and against altered copies of it
(each must fail at least one check).
"""
from __future__ import annotations

import math
import os
import sys
from fractions import Fraction

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from workloads import gen  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U = 2.0 ** -53


def gamma(n: int) -> float:
    """Higham's gamma_n = n u / (1 - n u) for binary64."""
    return n * U / (1 - n * U)


def read_golden(name: str) -> dict:
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            out[key] = vals
    return out


# ----------------------------------------------------------------------------
# P1: row sums of stencils on a vector of ones (closed-form classes)
# ----------------------------------------------------------------------------

def _neighbour_count(coords, dims, full):
    """Number of in-grid neighbours of each point (box or star stencil)."""
    nd = len(dims)
    count = np.zeros(coords[0].size, dtype=np.int64)
    rng = (-1, 0, 1)
    import itertools
    for off in itertools.product(rng, repeat=nd):
        if all(o == 0 for o in off):
            continue
        if not full and sum(abs(o) for o in off) != 1:
            continue
        ok = np.ones(coords[0].size, dtype=bool)
        for a in range(nd):
            c = coords[a] + off[a]
            ok &= (c >= 0) & (c < dims[a])
        count += ok
    return count


def check_rowsums(O):
    # 2D 5-point, 64 x 64 (4 / -1): interior 0 (3844 rows), edge 1 (248), corner 2 (4)
    A = gen.laplace_5pt_2d(64)
    r = O.spmv(A.row_ptr, A.col_idx, A.val, np.ones(A.n_cols))
    assert A.nnz == 5 * 4096 - 4 * 64
    assert (r == 0).sum() == 62 * 62 and (r == 1).sum() == 4 * 62 and (r == 2).sum() == 4
    assert r.sum() == 256.0
    # 3D 27-point (26 / -1) on 6^3: interior 0, face 9, edge 15, corner 19
    n = 6
    A = gen.stencil_27pt_3d(n)
    r = O.spmv(A.row_ptr, A.col_idx, A.val, np.ones(A.n_cols))
    k = np.arange(n ** 3)
    ix, iy, iz = k % n, (k // n) % n, k // (n * n)
    nb = sum(((c == 0) | (c == n - 1)).astype(int) for c in (ix, iy, iz))  # boundary axes
    expect = np.select([nb == 0, nb == 1, nb == 2, nb == 3], [0.0, 9.0, 15.0, 19.0])
    assert np.array_equal(r, expect)
    assert [(r == v).sum() for v in (0, 9, 15, 19)] == [(n - 2) ** 3, 6 * (n - 2) ** 2, 12 * (n - 2), 8]
    # 3D 7-point (6 / -1) on 5 x 4 x 3: row sum = number of missing neighbours
    A = gen.laplace_7pt_3d(5, 4, 3)
    r = O.spmv(A.row_ptr, A.col_idx, A.val, np.ones(A.n_cols))
    k = np.arange(60)
    coords = [k % 5, (k // 5) % 4, k // 20]
    assert np.array_equal(r, 6.0 - _neighbour_count(coords, (5, 4, 3), False))


# ----------------------------------------------------------------------------
# P2: integer quadratics -- exact interior value plus ghost contributions
# ----------------------------------------------------------------------------

def _ghost_sum(coords, dims, full, p):
    """Sum of p over the neighbours that fall outside the grid."""
    import itertools
    nd = len(dims)
    s = np.zeros(coords[0].size, dtype=np.int64)
    for off in itertools.product((-1, 0, 1), repeat=nd):
        if all(o == 0 for o in off):
            continue
        if not full and sum(abs(o) for o in off) != 1:
            continue
        g = [coords[a] + off[a] for a in range(nd)]
        outside = np.zeros(coords[0].size, dtype=bool)
        for a in range(nd):
            outside |= (g[a] < 0) | (g[a] >= dims[a])
        s += np.where(outside, p(*g), 0)
    return s


def check_quadratics(O):
    # 2D 5-point on 7 x 5: p = i^2 + j^2 -> interior -4; p = i*j -> interior 0
    nx, ny = 7, 5
    A = gen.laplace_5pt_2d(nx, ny)
    k = np.arange(nx * ny)
    c = [k % nx, k // nx]
    for p, interior in ((lambda i, j: i * i + j * j, -4), (lambda i, j: i * j, 0),
                        (lambda i, j: 3 * i - 2 * j + 5, 0)):
        x = p(*c).astype(np.float64)
        r = O.spmv(A.row_ptr, A.col_idx, A.val, x)
        assert np.array_equal(r, interior + _ghost_sum(c, (nx, ny), False, p).astype(np.float64))
    # 3D 7-point on 4 x 5 x 6: p = i^2 + j^2 + k^2 -> interior -6
    dims = (4, 5, 6)
    A = gen.laplace_7pt_3d(*dims)
    k = np.arange(np.prod(dims))
    c = [k % 4, (k // 4) % 5, k // 20]
    p = lambda i, j, l: i * i + j * j + l * l  # noqa: E731
    r = O.spmv(A.row_ptr, A.col_idx, A.val, p(*c).astype(np.float64))
    assert np.array_equal(r, -6 + _ghost_sum(c, dims, False, p).astype(np.float64))
    # 3D 27-point (26 / -1) on 5^3: A = 27 I - T(x)T(x)T with T = tridiag(1,1,1);
    # p = i^2 + j^2 + k^2 -> interior -54, p = i*j*k -> interior 0
    n = 5
    A = gen.stencil_27pt_3d(n)
    k = np.arange(n ** 3)
    c = [k % n, (k // n) % n, k // (n * n)]
    for p, interior in ((lambda i, j, l: i * i + j * j + l * l, -54), (lambda i, j, l: i * j * l, 0)):
        r = O.spmv(A.row_ptr, A.col_idx, A.val, p(*c).astype(np.float64))
        assert np.array_equal(r, interior + _ghost_sum(c, (n, n, n), True, p).astype(np.float64))


# ----------------------------------------------------------------------------
# P3: Dirichlet sine modes are eigenvectors with closed-form eigenvalues
# ----------------------------------------------------------------------------

def check_sine_modes(O):
    def mode(dims, ps):
        # 1-based grid coordinates i_d = 1..n_d; x fastest
        grids = np.meshgrid(*[np.arange(1, d + 1) for d in dims], indexing="ij")
        x = np.ones(grids[0].shape)
        for g, d, p in zip(grids, dims, ps):
            x = x * np.sin(np.pi * p * g / (d + 1))
        # meshgrid with 'ij' gives axis 0 = x; flatten so that x is fastest
        return x.transpose(*reversed(range(len(dims)))).ravel()

    cases = []
    dims = (64, 64)
    for ps in ((1, 1), (3, 7), (64, 2)):
        lam = 4 - sum(2 * math.cos(math.pi * p / (d + 1)) for p, d in zip(ps, dims))
        cases.append((gen.laplace_5pt_2d(*dims), mode(dims, ps), lam))
    dims = (9, 8, 7)
    for ps in ((1, 1, 1), (2, 5, 7)):
        lam = 6 - sum(2 * math.cos(math.pi * p / (d + 1)) for p, d in zip(ps, dims))
        cases.append((gen.laplace_7pt_3d(*dims), mode(dims, ps), lam))
    n = 7
    for ps in ((1, 1, 1), (2, 4, 6), (7, 1, 3)):
        lam = 27 - math.prod(1 + 2 * math.cos(math.pi * p / (n + 1)) for p in ps)
        cases.append((gen.stencil_27pt_3d(n), mode((n, n, n), ps), lam))
    for A, x, lam in cases:
        r = O.spmv(A.row_ptr, A.col_idx, A.val, x)
        denom = np.abs(A.val).max() * np.abs(x).max() * np.diff(A.row_ptr).max() + abs(lam) * np.abs(x)
        assert np.all(np.abs(r - lam * x) <= 1e-13 * denom), (lam, np.abs(r - lam * x).max())


# ----------------------------------------------------------------------------
# P4: exact rational brute force on tiny random matrices
# ----------------------------------------------------------------------------

def _dense_exact(A, x, c0):
    """Exact C0 + A x with a dense matrix of Fractions (duplicates summed)."""
    D = [[Fraction(0)] * A.n_cols for _ in range(A.n_rows)]
    for i in range(A.n_rows):
        for j in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i][int(A.col_idx[j])] += Fraction(float(A.val[j]))
    out = []
    for i in range(A.n_rows):
        s = Fraction(float(c0[i]))
        for col in range(A.n_cols):
            if D[i][col]:
                s += D[i][col] * Fraction(float(x[col]))
        out.append(s)
    return out


def _abs_exact(A, x, c0):
    out = []
    for i in range(A.n_rows):
        s = abs(Fraction(float(c0[i])))
        for j in range(A.row_ptr[i], A.row_ptr[i + 1]):
            s += abs(Fraction(float(A.val[j]))) * abs(Fraction(float(x[int(A.col_idx[j])])))
        out.append(s)
    return out


def _tiny_cases():
    rng = gen.rng_for(900, 0)
    shapes = [(1, 1), (5, 5), (7, 13), (13, 7), (16, 16), (32, 9), (3, 0), (0, 4), (0, 0), (24, 31)]
    cases = []
    for t, (m, n) in enumerate(shapes):
        for integer in (False, True):
            A = gen.random_crs(m, n, rng, max_len=9, integer_values=integer)
            if integer:
                x = rng.integers(-9, 10, size=n).astype(np.float64)
                c0 = rng.integers(-9, 10, size=m).astype(np.float64)
            else:
                x = rng.standard_normal(n)
                c0 = rng.standard_normal(m)
            cases.append((A, x, c0, integer))
    return cases


def check_bruteforce(O):
    for A, x, c0, integer in _tiny_cases():
        exact = _dense_exact(A, x, c0)
        mag = _abs_exact(A, x, c0)
        for base in (0, 1):
            r = O.spmv(A.row_ptr + base, A.col_idx + base, A.val, x, c0, base=base)
            assert r.shape == (A.n_rows,)
            for i in range(A.n_rows):
                err = abs(Fraction(float(r[i])) - exact[i])
                if integer:
                    assert err == 0, (i, r[i], exact[i])
                else:
                    ln = int(A.row_ptr[i + 1] - A.row_ptr[i])
                    assert err <= Fraction(gamma(ln + 1)) * mag[i], (i, float(err))
        # denominators of the normalised error, exact on integers
        d = O.abs_spmv(A.row_ptr, A.col_idx, A.val, x, c0)
        for i in range(A.n_rows):
            if integer:
                assert Fraction(float(d[i])) == mag[i]
            else:
                ln = int(A.row_ptr[i + 1] - A.row_ptr[i])
                assert abs(Fraction(float(d[i])) - mag[i]) <= Fraction(gamma(ln + 1)) * mag[i]


def check_rows(O):
    for A, x, c0, integer in _tiny_cases():
        if not integer or A.n_rows == 0:
            continue
        exact = _dense_exact(A, x, c0)
        rng = np.random.default_rng(A.n_rows * 31 + A.n_cols)
        rows = rng.integers(0, A.n_rows, size=min(A.n_rows, 6))
        r = O.spmv_rows(rows, A.row_ptr, A.col_idx, A.val, x, c0[rows])
        assert [Fraction(float(v)) for v in r] == [exact[i] for i in rows]


def check_block(O):
    rng = gen.rng_for(901, 0)
    for (m, n, k) in ((9, 11, 3), (16, 16, 4), (5, 2, 2), (12, 7, 1)):
        A = gen.random_crs(m, n, rng, max_len=6, integer_values=True)
        X = rng.integers(-7, 8, size=(n, k)).astype(np.float64)
        C0 = rng.integers(-7, 8, size=(m, k)).astype(np.float64)
        r = O.spmv_block(A.row_ptr, A.col_idx, A.val, X, C0)
        for t in range(k):
            exact = _dense_exact(A, X[:, t], C0[:, t])
            assert [Fraction(float(v)) for v in r[:, t]] == exact, t
        # 1-based arrays give the same block product
        r1 = O.spmv_block(A.row_ptr + 1, A.col_idx + 1, A.val, X, C0, base=1)
        assert np.array_equal(r, r1)


# ----------------------------------------------------------------------------
# Split (Sect. 3.4): hand-worked example and structural invariants
# ----------------------------------------------------------------------------

def check_split(O):
    g = read_golden("split_small.txt")
    iv = lambda k: np.array([int(v) for v in g[k]], dtype=np.int32)  # noqa: E731
    fv = lambda k: np.array([float(v) for v in g[k]])  # noqa: E731
    h = int(g["h"][0])
    for base in (0, 1):
        parts = O.split(iv("row_ptr") + base, iv("col_idx") + base, fv("val"), h, base=base)
        for key in ("loc_row_ptr", "loc_col", "nl_rows", "nl_ptr", "nl_col"):
            assert np.array_equal(parts[key], iv(key)), key
        for key in ("loc_val", "nl_val"):
            assert np.array_equal(parts[key], fv(key)), key
    c = O.spmv_split(parts, fv("B"))
    assert np.array_equal(c, fv("C"))
    loc_only = O.spmv(parts["loc_row_ptr"], parts["loc_col"], parts["loc_val"], fv("B"))
    assert np.array_equal(loc_only, fv("C_local"))

    # random matrices: the two parts partition the stored entries
    rng = gen.rng_for(902, 0)
    for (m, n) in ((40, 40), (17, 60), (60, 17), (1, 5)):
        A = gen.random_crs(m, n, rng, max_len=10, integer_values=True)
        for h in (0, 1, n // 2, n - 1, n):
            p = O.split(A.row_ptr, A.col_idx, A.val, h)
            assert p["loc_row_ptr"][0] == 0 and p["loc_row_ptr"][-1] == p["loc_col"].size
            assert np.all(p["loc_col"] < h) and np.all(p["nl_col"] >= h)
            lrp = p["loc_row_ptr"]
            R = p["nl_rows"].size
            assert np.all(np.diff(p["nl_rows"]) > 0) and np.all(np.diff(p["nl_ptr"]) > 0)
            nl_of = {int(p["nl_rows"][r]): (int(p["nl_ptr"][r]), int(p["nl_ptr"][r + 1])) for r in range(R)}
            for i in range(m):
                cols = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
                vals = A.val[A.row_ptr[i]:A.row_ptr[i + 1]]
                loc = cols < h
                assert np.array_equal(p["loc_col"][lrp[i]:lrp[i + 1]], cols[loc])
                assert np.array_equal(p["loc_val"][lrp[i]:lrp[i + 1]], vals[loc])
                if (~loc).any():
                    a, b = nl_of[i]
                    assert np.array_equal(p["nl_col"][a:b], cols[~loc])
                    assert np.array_equal(p["nl_val"][a:b], vals[~loc])
                else:
                    assert i not in nl_of
            x = rng.integers(-9, 10, size=n).astype(np.float64)
            c0 = rng.integers(-9, 10, size=m).astype(np.float64)
            exact = _dense_exact(A, x, c0)
            cs = O.spmv_split(p, x, c0)
            assert [Fraction(float(v)) for v in cs] == exact


# ----------------------------------------------------------------------------
# Send side of the exchange (Sect. 3.3): hand-worked lists, the transposed
# definition on random symmetric structures, bitwise gathers
# ----------------------------------------------------------------------------

def _grid5_structure(nx: int, ny: int):
    """CRS structure of the 5-point stencil on an nx x ny grid, row x + nx*y,
    built here from the neighbour description (no library code)."""
    rp, ci = [0], []
    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            nb = [i]
            if x > 0:
                nb.append(i - 1)
            if x < nx - 1:
                nb.append(i + 1)
            if y > 0:
                nb.append(i - nx)
            if y < ny - 1:
                nb.append(i + nx)
            ci.extend(sorted(nb))
            rp.append(len(ci))
    return np.array(rp, np.int32), np.array(ci, np.int32)


def check_send(O):
    g = read_golden("send_small.txt")
    rp, ci = _grid5_structure(3, 3)
    for h, key in ((6, "send_h6"), (4, "send_h4"), (9, "send_h9"), (0, "send_h0")):
        for base in (0, 1):
            got = O.send_list_symmetric(rp + base, ci + base, h, base=base)
            assert got.tolist() == [int(v) for v in g[key]], (h, base)
    out = O.pack([int(v) for v in g["pack_idx"]], [float(v) for v in g["pack_B"]])
    assert out.tolist() == [float(v) for v in g["pack_out"]]

    rng = gen.rng_for(903, 0)
    # the send list equals the columns below h used by the rows at or above h
    for n in (1, 2, 7, 40, 97):
        for density in (0.05, 0.3):
            S = rng.random((n, n)) < density
            S = S | S.T
            rows, cols = [0], []
            for i in range(n):
                c = np.flatnonzero(S[i])
                rng.shuffle(c)  # storage order need not be sorted
                cols.extend(c.tolist())
                rows.append(len(cols))
            rp2, ci2 = np.array(rows, np.int32), np.array(cols, np.int32)
            for h in sorted({0, 1, n // 3, n // 2, n - 1, n}):
                want = [j for j in range(h) if S[h:, j].any()]
                assert O.send_list_symmetric(rp2, ci2, h).tolist() == want, (n, h)

    # the gather copies bits: signed zeros and NaN payloads survive
    B = rng.standard_normal(64)
    B[3] = -0.0
    B[7] = np.array([0x7FF8DEADBEEF0001], dtype=np.uint64).view(np.float64)[0]
    B[9] = np.inf
    ident = O.pack(np.arange(64), B)
    assert np.array_equal(ident.view(np.uint64), B.view(np.uint64))
    perm = rng.permutation(64)
    back = np.empty(64)
    back[perm] = O.pack(perm, B)
    assert np.array_equal(back.view(np.uint64), B.view(np.uint64))
    rep = O.pack(np.full(5, 7), B)
    assert np.all(rep.view(np.uint64) == B[7:8].view(np.uint64))
    assert O.pack(np.zeros(0, np.int32), B).size == 0


# ----------------------------------------------------------------------------
# Chebyshev moments: exact sequences and the spectral closed form of the
# Dirichlet Laplacian (eigenvectors are sine modes)
# ----------------------------------------------------------------------------

def _cheb(m: int, t: np.ndarray) -> np.ndarray:
    return np.cos(m * np.arccos(np.clip(t, -1.0, 1.0)))


def check_kpm(O):
    # 1 x 1 matrix [0.5], v0 = 1: v_m = T_m(1/2) = cos(m pi / 3), every step exact
    one = O.kpm_moments(np.array([0, 1], np.int32), np.array([0], np.int32), np.array([0.5]),
                        np.ones((1, 1)), 13)
    assert one[:, 0].tolist() == [[1.0, 0.5, -0.5, -1.0, -0.5, 0.5][m % 6] for m in range(13)]
    # 1 x 1 matrix [-1], v0 = 3: mu_m = 9 (-1)^m; index base 1
    neg = O.kpm_moments(np.array([1, 2], np.int32), np.array([1], np.int32), np.array([-1.0]),
                        np.full((1, 1), 3.0), 6, base=1)
    assert neg[:, 0].tolist() == [9.0 * (-1) ** m for m in range(6)]

    # H = (L - 4 I) / 4.25 for the 5-point Laplacian L (4 / -1) on an n x n grid:
    # eigenvalues -(2 cos(j pi/(n+1)) + 2 cos(k pi/(n+1))) / 4.25 with
    # orthonormal eigenvectors s_j(x) s_k(y), s_j(x) = sqrt(2/(n+1)) sin(j pi (x+1)/(n+1))
    n = 12
    rp, ci = _grid5_structure(n, n)
    rows = np.repeat(np.arange(n * n), np.diff(rp))
    val = np.where(ci == rows, 0.0, -1.0 / 4.25)
    rng = gen.rng_for(904, 0)
    R, M = 3, 40
    V0 = rng.standard_normal((n * n, R))
    mu = O.kpm_moments(rp, ci, val, V0, M)
    idx = np.arange(1, n + 1)
    S = np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(idx, idx) / (n + 1))  # S[j-1, x]
    lam = 2.0 * np.cos(idx * np.pi / (n + 1))
    theta = -(lam[:, None] + lam[None, :]) / 4.25  # [k-1 (y), j-1 (x)]
    for r in range(R):
        c = S @ V0[:, r].reshape(n, n) @ S.T  # [k-1, j-1]: coefficient of mode (j, k)
        norm2 = float(V0[:, r] @ V0[:, r])
        for m in range(M):
            want = float(np.sum(c * c * _cheb(m, theta)))
            assert abs(mu[m, r] - want) <= 1e-12 * norm2, (r, m, mu[m, r], want)
    # the moments of a start vector that is one eigenvector are T_m(theta) exactly in form
    e = (S[2][:, None] * S[4][None, :]).T.reshape(-1)  # mode j = 3 (x), k = 5 (y)
    mu_e = O.kpm_moments(rp, ci, val, e[:, None], 25)
    th = -(lam[2] + lam[4]) / 4.25
    assert np.allclose(mu_e[:, 0], _cheb(np.arange(25), th), rtol=0, atol=1e-13)


# ----------------------------------------------------------------------------
# Lanczos: a matrix already in Lanczos form, the Gram-polynomial recurrence,
# and termination on an invariant subspace of the Dirichlet Laplacian
# ----------------------------------------------------------------------------

def _laplace_1d(n):
    rp, ci, vv = [0], [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                ci.append(j)
                vv.append(v)
        rp.append(len(ci))
    return np.array(rp, np.int32), np.array(ci, np.int32), np.array(vv)


def check_lanczos(O):
    # tridiag(-1, 2, -1) from e_1 is its own Lanczos matrix: alpha = 2, beta = 1
    # (every operation exact), in both index bases
    rp, ci, vv = _laplace_1d(50)
    q = np.zeros(50)
    q[0] = 3.0
    for base in (0, 1):
        a, b = O.lanczos(rp + base, ci + base, vv, q, 20, base=base)
        assert a.tolist() == [2.0] * 20 and b.tolist() == [1.0] * 20
    # diag(0, 1, ..., N-1) from the vector of ones: the recurrence of the
    # discrete Chebyshev (Gram) polynomials, alpha_j = (N-1)/2 and
    # beta_j^2 = j^2 (N^2 - j^2) / (4 (4 j^2 - 1))
    N = 30
    a, b = O.lanczos(np.arange(N + 1, dtype=np.int32), np.arange(N, dtype=np.int32),
                     np.arange(N, dtype=np.float64), np.ones(N), N - 1)
    j = np.arange(1, N)
    assert np.allclose(a, (N - 1) / 2, rtol=0, atol=1e-12)
    assert np.allclose(b, np.sqrt(j * j * (N * N - j * j) / (4.0 * (4 * j * j - 1))), rtol=0, atol=1e-12)
    # q in the span of k sine modes of the 12 x 12 Dirichlet 5-point Laplacian:
    # after k steps beta_k vanishes and T_k has exactly those k eigenvalues
    n = 12
    rp2, ci2 = _grid5_structure(n, n)
    rows = np.repeat(np.arange(n * n), np.diff(rp2))
    val = np.where(ci2 == rows, 4.0, -1.0)
    idx = np.arange(1, n + 1)
    S = np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(idx, idx) / (n + 1))
    lam = 2.0 - 2.0 * np.cos(idx * np.pi / (n + 1))
    modes = [(1, 1), (2, 5), (7, 3), (12, 12)]
    q = np.zeros(n * n)
    for t, (jx, ky) in enumerate(modes):
        q += (t + 1.0) * np.outer(S[ky - 1], S[jx - 1]).reshape(-1)  # [y, x] layout
    k = len(modes)
    a, b = O.lanczos(rp2, ci2, val, q, k)
    assert abs(b[k - 1]) <= 1e-12 * 8
    T = np.diag(a) + np.diag(b[:k - 1], 1) + np.diag(b[:k - 1], -1)
    want = sorted(lam[jx - 1] + lam[ky - 1] for jx, ky in modes)
    assert np.allclose(np.linalg.eigvalsh(T), want, rtol=0, atol=1e-12)


# ----------------------------------------------------------------------------
# Rounding to the storage precisions: exhaustive enumeration of the targets
# ----------------------------------------------------------------------------

def _bf16_values():
    """All bfloat16 codes and their values, decoded through binary32 (a
    bfloat16 code is the upper half of a binary32 pattern)."""
    codes = np.arange(65536, dtype=np.uint32)
    with np.errstate(invalid="ignore"):
        vals = (codes << 16).view(np.float32).astype(np.float64)
    return codes.astype(np.uint16), vals


def _nearest_even(x, codes, vals, inf_code):
    """Brute-force nearest representable value, ties to the even code."""
    finite = np.isfinite(vals)
    pos = finite & (np.signbit(vals) == False)  # noqa: E712
    pc, pv = codes[pos], vals[pos]
    order = np.argsort(pv, kind="stable")
    pc, pv = pc[order], pv[order]
    # drop -0 duplicates etc: +0 is code 0 (first)
    out = np.empty(x.size, dtype=np.int64)
    a = np.abs(x)
    idx = np.searchsorted(pv, a, side="left")
    for t in range(x.size):
        if np.isnan(x[t]):
            out[t] = -1
            continue
        s = 1 if np.signbit(x[t]) else 0
        i = idx[t]
        if i < pv.size and pv[i] == a[t]:
            c = pc[i]
        elif i >= pv.size:
            # beyond the largest finite value: halfway point to 2^emax+1 decides
            top = pv[-1]
            half = (top + (top - pv[-2]) / 2)
            c = inf_code if a[t] >= half else pc[-1]
        else:
            lo, hi = pv[i - 1], pv[i]
            if a[t] - lo < hi - a[t]:
                c = pc[i - 1]
            elif a[t] - lo > hi - a[t]:
                c = pc[i]
            else:
                c = pc[i - 1] if pc[i - 1] % 2 == 0 else pc[i]
        out[t] = int(c) | (s << 15)
    return out


def _rounding_inputs(vals):
    rng = np.random.default_rng(7)
    fin = vals[np.isfinite(vals)]
    fin = fin[fin > 0]
    fin = np.unique(fin)
    # exact representable values, midpoints (ties), and near-midpoints
    mids = (fin[:-1] + fin[1:]) / 2
    xs = [fin[::37], mids[::29], np.nextafter(mids[::31], 0), np.nextafter(mids[::31], np.inf)]
    xs.append(rng.standard_normal(3000) * 10.0 ** rng.integers(-45, 39, size=3000))
    xs.append(np.array([0.0, 5e-324, 1e-300, 1e300, fin[-1] * (1 + 2.0 ** -9), fin[-1] * 1.01]))
    x = np.concatenate(xs)
    return np.concatenate([x, -x, [np.nan, -np.nan, np.inf, -np.inf, -0.0]])


def check_round_bf16(O):
    codes, vals = _bf16_values()
    x = _rounding_inputs(vals)
    got = O.round_bf16(x).astype(np.int64)
    exp = _nearest_even(x, codes, vals, 0x7F80).astype(np.int64)
    nan = np.isnan(x)
    assert np.array_equal(got[~nan], exp[~nan]), np.flatnonzero(got[~nan] != exp[~nan])[:5]
    assert np.all((got[nan] & 0x7FFF) == 0x7FC0)
    # decoding every code is exact (NaN codes decode to NaN)
    dec = O.bf16_to_f64(codes)
    same = (dec == vals) | (np.isnan(dec) & np.isnan(vals))
    assert same.all()
    assert np.array_equal(np.signbit(dec[~np.isnan(dec)]), np.signbit(vals[~np.isnan(vals)]))


def check_round_f32(O):
    rng = np.random.default_rng(11)
    f = rng.standard_normal(4000).astype(np.float32) * np.float32(2.0) ** rng.integers(-150, 127, size=4000).astype(np.float32)
    f = f[np.isfinite(f) & (f != 0)]
    lo = f.astype(np.float64)
    hi = np.nextafter(f, np.float32(np.inf) * np.sign(f)).astype(np.float64)
    mid = (lo + hi) / 2
    x = np.concatenate([lo, mid, np.nextafter(mid, 0), np.nextafter(mid, np.inf) * 1.0])
    got = O.round_f32(x)
    for t in range(x.size):
        a = np.float32(x[t])  # candidate; checked against both neighbours below
        d = np.float64(x[t])
        below = np.nextafter(np.float32(d), np.float32(-np.inf))
        above = np.nextafter(np.float32(d), np.float32(np.inf))
        cands = [np.float32(c) for c in (below, a, above) if np.isfinite(c)]
        best = min(abs(np.float64(c) - d) for c in cands)
        nearest = [c for c in cands if abs(np.float64(c) - d) == best]
        if len(nearest) > 1:
            nearest = [c for c in nearest if (np.array(c).view(np.uint32) & 1) == 0]
        assert got[t] == nearest[0], (t, d, got[t], nearest)
    assert np.isnan(O.round_f32(np.array([np.nan]))[0])
    assert O.round_f32(np.array([1e39, -1e39])).tolist() == [np.inf, -np.inf]


ALL_CHECKS = [check_rowsums, check_quadratics, check_sine_modes, check_bruteforce, check_rows,
              check_block, check_split, check_send, check_kpm, check_lanczos, check_round_bf16,
              check_round_f32]


def run_all(O) -> list:
    """Run every check; return the names of those that failed."""
    failed = []
    for chk in ALL_CHECKS:
        try:
            chk(O)
        except AssertionError:
            failed.append(chk.__name__)
    return failed


if __name__ == "__main__":
    # usage: python pins.py <path to liboracle build>
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import oracle as _oracle

    bad = run_all(_oracle.Oracle(sys.argv[1]))
    print("FAILED:" + ",".join(bad) if bad else "ALL-PASS")
    sys.exit(1 if bad else 0)
