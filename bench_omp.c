/* Host-CPU reference point for the benchmark: the CRS product as the paper
 * runs it on a multicore node, plus the triad that measures the node's
 * memory bandwidth.
 *
 * CRS (Listing 1, storage of Sect. 1.2): one OpenMP loop over the rows with
 * a static schedule.  All arrays are copied into memory that is first
 * touched under that same schedule, so each thread's rows, entries and
 * vector slices lie in memory local to it (the placement the paper uses for
 * its node-level runs, Sect. 2).
 *
 * Triad a = b + s*c (the STREAM triad of Sect. 2), same first-touch
 * placement; bytes counted as 24 per element (add 1/3 for the
 * write-allocate transfer of a).
 *
 * Not part of the GPU library and not the oracle: a plain C baseline that
 * bench.py loads with ctypes.  Build: gcc -O3 -fopenmp -shared -fPIC.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double now(void) { return omp_get_wtime(); }

static int cmp_double(const void *a, const void *b) {
  const double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/* Copies the CRS matrix and x into first-touched memory, runs `reps` products
 * y = y + A x starting from y = 0 (one extra untimed call first), returns
 * the median seconds per call and leaves the first call's y in y_out (n_rows
 * entries).  threads_out receives the thread count.  Returns a negative
 * value when memory cannot be allocated. */
double omp_crs_bench(int64_t n_rows, int64_t n_cols, const int32_t *row_ptr, const int32_t *col,
                     const double *val, const double *x, int reps, double *y_out,
                     int *threads_out) {
  const int64_t nnz = row_ptr[n_rows];
  int32_t *rp = malloc(sizeof(int32_t) * (size_t)(n_rows + 1));
  int32_t *c = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  double *v = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  double *xx = malloc(sizeof(double) * (size_t)(n_cols > 0 ? n_cols : 1));
  double *y = malloc(sizeof(double) * (size_t)(n_rows > 0 ? n_rows : 1));
  double *times = malloc(sizeof(double) * (size_t)(reps > 0 ? reps : 1));
  if (!rp || !c || !v || !xx || !y || !times) {
    free(rp); free(c); free(v); free(xx); free(y); free(times);
    return -1.0;
  }
  int nt = 1;
#pragma omp parallel
  {
#pragma omp single
    nt = omp_get_num_threads();
  }
  /* first touch under the product's schedule */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_rows; ++i) {
    rp[i] = row_ptr[i];
    y[i] = 0.0;
    for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
      c[j] = col[j];
      v[j] = val[j];
    }
  }
  rp[n_rows] = row_ptr[n_rows];
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_cols; ++i) xx[i] = x[i];

  for (int r = -1; r < reps; ++r) {
    const double t0 = now();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
      double acc = y[i];
      for (int32_t j = rp[i]; j < rp[i + 1]; ++j) acc += v[j] * xx[c[j]];
      y[i] = acc;
    }
    const double t1 = now();
    if (r == -1) memcpy(y_out, y, sizeof(double) * (size_t)n_rows);
    if (r >= 0) times[r] = t1 - t0;
  }
  qsort(times, (size_t)reps, sizeof(double), cmp_double);
  const double med = reps > 0 ? times[reps / 2] : 0.0;
  free(rp); free(c); free(v); free(xx); free(y); free(times);
  if (threads_out) *threads_out = nt;
  return med;
}

/* Triad over n doubles per array, best of `reps`; returns GB/s counted as
 * 24 bytes per element, or a negative value when memory cannot be
 * allocated. */
double omp_triad_bench(int64_t n, int reps, int *threads_out) {
  double *a = malloc(sizeof(double) * (size_t)n);
  double *b = malloc(sizeof(double) * (size_t)n);
  double *c = malloc(sizeof(double) * (size_t)n);
  if (!a || !b || !c) {
    free(a); free(b); free(c);
    return -1.0;
  }
  int nt = 1;
#pragma omp parallel
  {
#pragma omp single
    nt = omp_get_num_threads();
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    a[i] = 0.0;
    b[i] = 1.0;
    c[i] = 2.0;
  }
  double best = 1e30;
  const double s = 0.5;
  for (int r = 0; r < reps; ++r) {
    const double t0 = now();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) a[i] = b[i] + s * c[i];
    const double t = now() - t0;
    if (t < best) best = t;
  }
  volatile double sink = a[n / 2];
  (void)sink;
  free(a); free(b); free(c);
  if (threads_out) *threads_out = nt;
  return 24.0 * (double)n / best / 1e9;
}
