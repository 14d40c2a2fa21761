/*
 * spmv_oracle -- plain, sequential, FP64 CPU reference for the CRS spMV path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the yardstick the GPU library is
 * checked against; it is used by the test suite, by the package's smoke check
 * and by the benchmark's CPU-baseline leg, and by nothing else.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 *   (no FMA contraction and no reassociation: every multiply and add below is
 *   one IEEE-754 binary64 operation rounded to nearest-even, in the order
 *   written).
 *
 * Source of truth: Schubert, Fehske, Hager, Wellein, "Hybrid-parallel sparse
 * matrix-vector multiplication with explicit communication overlap on current
 * multicore-based systems" (2011).
 *   - CRS storage: Sect. 1.2 (val row by row, row_ptr row starts, col_idx the
 *     original column of each entry).
 *   - The kernel: Listing 1, C(i) = C(i) + val(j) * B(col_idx(j)), rows in
 *     order, entries of a row in storage order.
 *   - Local / nonlocal split: Sect. 3.4 (first the part that uses local RHS
 *     elements only, then the remaining part once the halo has arrived; the
 *     result vector is updated twice).
 *   - Send buffer: Sect. 3.3 (the elements other processes need, gathered
 *     into one contiguous buffer).
 *   - Chebyshev moments: the polynomial-expansion methods named in Sect. 1.3,
 *     from the three-term recursion of the Chebyshev polynomials.
 *   - Lanczos: the eigensolver named in Sect. 1.3, plain three-term form.
 *
 * Index base: Listing 1 is written with 1-based (Fortran) indices.  Every
 * function takes `base` (0 or 1) and subtracts it from row_ptr and col_idx
 * entries, so the same arrays can be passed in either convention.
 *
 * Parity pins: the test suite checks these functions against closed forms
 * (row sums of stencils on a vector of ones, integer quadratics, Dirichlet
 * sine modes), exact rational brute force on tiny random matrices, and
 * invariants of the split; the rounding helpers are checked against an
 * exhaustive enumeration of the bfloat16 / binary32 value sets.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Listing 1 over all rows: C[i] <- C[i] + sum_j val[j] * B[col_idx[j]]. */
void oracle_spmv(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                 const double *val, int32_t base, const double *B, double *C)
{
    for (int64_t i = 0; i < n_rows; ++i) {
        double c = C[i];
        int64_t begin = (int64_t)row_ptr[i] - base;
        int64_t end = (int64_t)row_ptr[i + 1] - base;
        for (int64_t j = begin; j < end; ++j) {
            double prod = val[j] * B[(int64_t)col_idx[j] - base];
            c = c + prod;
        }
        C[i] = c;
    }
}

/* Listing 1 restricted to the rows listed in `rows` (0-based row numbers):
 * out[s] <- out[s] + sum over row rows[s].  Used to check single entries of
 * very large products one by one. */
void oracle_spmv_rows(int64_t n_sel, const int64_t *rows, const int32_t *row_ptr,
                      const int32_t *col_idx, const double *val, int32_t base,
                      const double *B, double *out)
{
    for (int64_t s = 0; s < n_sel; ++s) {
        int64_t i = rows[s];
        double c = out[s];
        int64_t begin = (int64_t)row_ptr[i] - base;
        int64_t end = (int64_t)row_ptr[i + 1] - base;
        for (int64_t j = begin; j < end; ++j) {
            double prod = val[j] * B[(int64_t)col_idx[j] - base];
            c = c + prod;
        }
        out[s] = c;
    }
}

/* Listing 1 applied to each of k right-hand sides stored row-major:
 * column t of B is B[r*ldb + t], column t of C is C[r*ldc + t]. */
void oracle_spmv_block(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                       const double *val, int32_t base, int32_t k,
                       const double *B, int64_t ldb, double *C, int64_t ldc)
{
    for (int32_t t = 0; t < k; ++t) {
        for (int64_t i = 0; i < n_rows; ++i) {
            double c = C[i * ldc + t];
            int64_t begin = (int64_t)row_ptr[i] - base;
            int64_t end = (int64_t)row_ptr[i + 1] - base;
            for (int64_t j = begin; j < end; ++j) {
                double prod = val[j] * B[((int64_t)col_idx[j] - base) * ldb + t];
                c = c + prod;
            }
            C[i * ldc + t] = c;
        }
    }
}

/* Denominator of the normalised componentwise error:
 * D[i] = |C0[i]| + sum_j |val[j]| * |B[col_idx[j]]|  (rows in order). */
void oracle_abs_spmv(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                     const double *val, int32_t base, const double *B,
                     const double *C0, double *D)
{
    for (int64_t i = 0; i < n_rows; ++i) {
        double d = fabs(C0[i]);
        int64_t begin = (int64_t)row_ptr[i] - base;
        int64_t end = (int64_t)row_ptr[i + 1] - base;
        for (int64_t j = begin; j < end; ++j)
            d = d + fabs(val[j]) * fabs(B[(int64_t)col_idx[j] - base]);
        D[i] = d;
    }
}

/* ---------------------------------------------------------------------------
 * Local / nonlocal split of one process's share (Sect. 3.4).
 *
 * Columns [0, h) are the locally owned RHS elements, columns [h, n_cols) the
 * halo received from other processes.  The local part keeps every stored
 * entry with column < h in a CRS with the full n_rows+1 row_ptr.  The
 * nonlocal part keeps the entries with column >= h, only for the rows that
 * have at least one of them: nl_rows[r] is the r-th such row (ascending) and
 * nl_ptr[r]..nl_ptr[r+1]-1 its entries.  Entries keep their storage order and
 * their original (global, 0-based) column.  All outputs are 0-based.
 * ------------------------------------------------------------------------- */

/* First pass: sizes of the two parts. */
void oracle_split_count(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                        int32_t base, int64_t h, int64_t *nnz_loc, int64_t *nnz_nl,
                        int64_t *n_nl_rows)
{
    int64_t nl = 0, loc = 0, rows = 0;
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t here = 0;
        for (int64_t j = (int64_t)row_ptr[i] - base; j < (int64_t)row_ptr[i + 1] - base; ++j) {
            if ((int64_t)col_idx[j] - base < h)
                ++loc;
            else
                ++here;
        }
        nl += here;
        if (here > 0)
            ++rows;
    }
    *nnz_loc = loc;
    *nnz_nl = nl;
    *n_nl_rows = rows;
}

/* Second pass: fill both parts (arrays sized by oracle_split_count). */
void oracle_split_fill(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                       const double *val, int32_t base, int64_t h,
                       int32_t *loc_row_ptr, int32_t *loc_col, double *loc_val,
                       int32_t *nl_rows, int32_t *nl_ptr, int32_t *nl_col, double *nl_val)
{
    int64_t loc = 0, nl = 0, r = 0;
    loc_row_ptr[0] = 0;
    nl_ptr[0] = 0;
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t nl_before = nl;
        for (int64_t j = (int64_t)row_ptr[i] - base; j < (int64_t)row_ptr[i + 1] - base; ++j) {
            int64_t c = (int64_t)col_idx[j] - base;
            if (c < h) {
                loc_col[loc] = (int32_t)c;
                loc_val[loc] = val[j];
                ++loc;
            } else {
                nl_col[nl] = (int32_t)c;
                nl_val[nl] = val[j];
                ++nl;
            }
        }
        loc_row_ptr[i + 1] = (int32_t)loc;
        if (nl > nl_before) {
            nl_rows[r] = (int32_t)i;
            nl_ptr[r + 1] = (int32_t)nl;
            ++r;
        }
    }
}

/* The split product: local part over all rows, then the nonlocal part over
 * the listed rows (both 0-based, as produced by oracle_split_fill). */
void oracle_spmv_split(int64_t n_rows, const int32_t *loc_row_ptr, const int32_t *loc_col,
                       const double *loc_val, int64_t n_nl_rows, const int32_t *nl_rows,
                       const int32_t *nl_ptr, const int32_t *nl_col, const double *nl_val,
                       const double *B, double *C)
{
    oracle_spmv(n_rows, loc_row_ptr, loc_col, loc_val, 0, B, C);
    for (int64_t r = 0; r < n_nl_rows; ++r) {
        int64_t i = nl_rows[r];
        double c = C[i];
        for (int64_t j = nl_ptr[r]; j < nl_ptr[r + 1]; ++j) {
            double prod = nl_val[j] * B[nl_col[j]];
            c = c + prod;
        }
        C[i] = c;
    }
}

/* ---------------------------------------------------------------------------
 * Chebyshev moments of the kernel polynomial method (the polynomial-expansion
 * methods for spectral properties the paper lists among the applications of
 * spMVM, Sect. 1.3), by the plain definition: for each start vector v0 (column
 * r of the row-major block V0, n_rows x R),
 *   v_1 = H v0,  v_{m+1} = 2 H v_m - v_{m-1},  mu_m = v0 . v_m,
 * with every product H v computed by the Listing 1 loop from a zero vector
 * and every dot product summed in index order.  Returns 0, or -1 if memory
 * for the three work vectors cannot be allocated.
 * ------------------------------------------------------------------------- */
int oracle_kpm_moments(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                       const double *val, int32_t base, int32_t R, int32_t M,
                       const double *V0, double *mu)
{
    size_t n = (size_t)(n_rows > 0 ? n_rows : 1);
    double *prev = calloc(n, sizeof(double));
    double *cur = calloc(n, sizeof(double));
    double *hv = calloc(n, sizeof(double));
    if (!prev || !cur || !hv) {
        free(prev); free(cur); free(hv);
        return -1;
    }
    for (int32_t r = 0; r < R; ++r) {
        for (int64_t i = 0; i < n_rows; ++i)
            cur[i] = V0[i * R + r];
        for (int32_t m = 0; m < M; ++m) {
            double d = 0.0;
            for (int64_t i = 0; i < n_rows; ++i)
                d = d + V0[i * R + r] * cur[i];
            mu[(int64_t)m * R + r] = d;
            if (m + 1 == M)
                break;
            for (int64_t i = 0; i < n_rows; ++i)
                hv[i] = 0.0;
            oracle_spmv(n_rows, row_ptr, col_idx, val, base, cur, hv);
            for (int64_t i = 0; i < n_rows; ++i) {
                double next = (m == 0) ? hv[i] : 2.0 * hv[i] - prev[i];
                prev[i] = cur[i];
                cur[i] = next;
            }
        }
    }
    free(prev); free(cur); free(hv);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Lanczos (the iterative eigensolver the paper names first among the
 * algorithms whose time goes into spMVM, Sect. 1.3), without
 * reorthogonalisation: v_1 = q / |q|, beta_0 = 0, and for j = 1 .. m
 *   w = H v_j - beta_{j-1} v_{j-1},  alpha_j = w . v_j,
 *   w = w - alpha_j v_j,             beta_j = |w|,
 *   v_{j+1} = w / beta_j  (0 if beta_j = 0: the Krylov space is invariant).
 * alpha[j-1] = alpha_j and beta[j-1] = beta_j; the tridiagonal matrix of the
 * first m steps has diagonal alpha[0..m-1] and off-diagonal beta[0..m-2].
 * Products by the Listing 1 loop from a zero vector; dot products and norms
 * summed in index order.  Returns 0, or -1 if work memory cannot be
 * allocated.
 * ------------------------------------------------------------------------- */
int oracle_lanczos(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                   const double *val, int32_t base, int32_t m, const double *q,
                   double *alpha, double *beta)
{
    size_t n = (size_t)(n_rows > 0 ? n_rows : 1);
    double *prev = calloc(n, sizeof(double));
    double *cur = calloc(n, sizeof(double));
    double *w = calloc(n, sizeof(double));
    if (!prev || !cur || !w) {
        free(prev); free(cur); free(w);
        return -1;
    }
    double nq = 0.0;
    for (int64_t i = 0; i < n_rows; ++i)
        nq = nq + q[i] * q[i];
    nq = sqrt(nq);
    for (int64_t i = 0; i < n_rows; ++i)
        cur[i] = nq > 0.0 ? q[i] / nq : 0.0;
    double b_prev = 0.0;
    for (int32_t j = 0; j < m; ++j) {
        for (int64_t i = 0; i < n_rows; ++i)
            w[i] = 0.0;
        oracle_spmv(n_rows, row_ptr, col_idx, val, base, cur, w);
        for (int64_t i = 0; i < n_rows; ++i)
            w[i] = w[i] - b_prev * prev[i];
        double a = 0.0;
        for (int64_t i = 0; i < n_rows; ++i)
            a = a + w[i] * cur[i];
        for (int64_t i = 0; i < n_rows; ++i)
            w[i] = w[i] - a * cur[i];
        double b = 0.0;
        for (int64_t i = 0; i < n_rows; ++i)
            b = b + w[i] * w[i];
        b = sqrt(b);
        alpha[j] = a;
        beta[j] = b;
        for (int64_t i = 0; i < n_rows; ++i) {
            prev[i] = cur[i];
            cur[i] = b > 0.0 ? w[i] / b : 0.0;
        }
        b_prev = b;
    }
    free(prev); free(cur); free(w);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Send side of the exchange (Sect. 3.3: the RHS elements another process
 * needs are gathered into one contiguous send buffer before they are
 * communicated).
 * ------------------------------------------------------------------------- */

/* The send buffer: out[k] = B[idx[k]] for k < n (0-based positions). */
void oracle_pack(int64_t n, const int32_t *idx, const double *B, double *out)
{
    for (int64_t k = 0; k < n; ++k)
        out[k] = B[idx[k]];
}

/* The send list of a structurally symmetric matrix whose columns [h, n_cols)
 * belong to another process: every row i < h that holds at least one entry
 * with column >= h, ascending.  An entry (i, j) with i < h <= j means, by
 * symmetry, that the other process's row j uses column i, i.e. needs B[i].
 * out has room for n_rows entries; *count receives the list length. */
void oracle_send_list_symmetric(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                                int32_t base, int64_t h, int32_t *out, int64_t *count)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n_rows && i < h; ++i) {
        int needed = 0;
        for (int64_t j = (int64_t)row_ptr[i] - base; j < (int64_t)row_ptr[i + 1] - base; ++j)
            if ((int64_t)col_idx[j] - base >= h)
                needed = 1;
        if (needed)
            out[m++] = (int32_t)i;
    }
    *count = m;
}

/* ---------------------------------------------------------------------------
 * Storage-precision encodings of the values, each a single rounding of the
 * binary64 input to nearest, ties to even.
 * ------------------------------------------------------------------------- */

/* binary64 -> binary32: the C conversion, which rounds to nearest-even in the
 * default rounding mode; NaN stays NaN, overflow gives +-Inf. */
void oracle_round_f32(int64_t n, const double *in, float *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = (float)in[i];
}

/* binary64 -> bfloat16 (1 sign bit, 8 exponent bits with bias 127, 7 stored
 * fraction bits), by arithmetic on the value rather than on its bits:
 * find the spacing of bfloat16 numbers at |x| (2^(E-7) for a normal number
 * with leading exponent E >= -126, 2^-133 below that), round |x|/spacing to
 * the nearest integer with ties to even, and encode the result.  NaN becomes
 * the quiet NaN 0x7FC0 with the input's sign; results of magnitude >= 2^128
 * become +-Inf. */
void oracle_round_bf16(int64_t n, const double *in, uint16_t *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double x = in[i];
        uint16_t sign = signbit(x) ? 0x8000u : 0u;
        if (isnan(x)) {
            out[i] = (uint16_t)(sign | 0x7FC0u);
            continue;
        }
        double a = fabs(x);
        if (isinf(a)) {
            out[i] = (uint16_t)(sign | 0x7F80u);
            continue;
        }
        if (a == 0.0) {
            out[i] = sign;
            continue;
        }
        int ex;
        (void)frexp(a, &ex);            /* a = m * 2^ex, m in [0.5, 1) */
        int E = ex - 1;                 /* a in [2^E, 2^(E+1)) */
        int qexp = (E < -126) ? -133 : E - 7;
        double q = ldexp(a, -qexp);     /* exact: scaling by a power of two */
        double r = nearbyint(q);        /* round to nearest, ties to even */
        double v = ldexp(r, qexp);
        if (v >= ldexp(1.0, 128)) {
            out[i] = (uint16_t)(sign | 0x7F80u);
            continue;
        }
        uint16_t bits;
        if (v < ldexp(1.0, -126)) {
            bits = (uint16_t)r;         /* subnormal: fraction field = v / 2^-133 */
        } else {
            int vex;
            double vm = frexp(v, &vex); /* v = vm * 2^vex, vm in [0.5, 1) */
            int VE = vex - 1;
            double frac = ldexp(vm, 1) - 1.0;        /* in [0, 1) */
            uint16_t f = (uint16_t)ldexp(frac, 7);   /* exact: 7 fraction bits */
            bits = (uint16_t)(((uint16_t)(VE + 127) << 7) | f);
        }
        out[i] = (uint16_t)(sign | bits);
    }
}

/* bfloat16 code -> exact binary64 value. */
void oracle_bf16_to_f64(int64_t n, const uint16_t *in, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        uint16_t b = in[i];
        double s = (b & 0x8000u) ? -1.0 : 1.0;
        int e = (b >> 7) & 0xFF;
        int f = b & 0x7F;
        double v;
        if (e == 0xFF)
            v = f ? NAN : INFINITY;
        else if (e == 0)
            v = ldexp((double)f, -133);
        else
            v = ldexp(1.0 + ldexp((double)f, -7), e - 127);
        out[i] = s * v;
    }
}
