// Device-side bookkeeping of the local / nonlocal split (Sect. 3.4 of
// Schubert, Fehske, Hager, Wellein 2011; done once per partition as in
// Sect. 3.2).  Columns [0, h) are locally owned, columns [h, n_cols) the
// halo.  Three passes over the rows:
//   1. count: per row, entries with column < h, entries with column >= h,
//      and whether the row has any of the latter;
//   2. exclusive scans of the three counts (row starts of the local part,
//      offsets of the nonlocal entries, positions in the nonlocal row list);
//   3. fill: every row copies its entries, in storage order, to the two
//      parts and, if it has halo entries, records itself in the row list.
#include <hip/hip_runtime.h>

#include "spmv_internal.h"

namespace spmv {
namespace {

constexpr int SCAN_WG = 256;
constexpr int SCAN_PER = 8;
constexpr int SCAN_CHUNK = SCAN_WG * SCAN_PER;

// Work layout: three int32 arrays of n_rows + 1 entries each.  Entry n_rows
// is a zero pad so the exclusive scan leaves the total there.
__global__ void k_split_count(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                              int64_t n, int32_t h, int32_t *__restrict__ w_loc,
                              int32_t *__restrict__ w_nl, int32_t *__restrict__ w_flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == n) {
    w_loc[n] = 0;
    w_nl[n] = 0;
    w_flag[n] = 0;
    return;
  }
  int loc = 0, nl = 0;
  for (int j = rp[i]; j < rp[i + 1]; ++j) {
    if (col[j] < h) ++loc;
    else ++nl;
  }
  w_loc[i] = loc;
  w_nl[i] = nl;
  w_flag[i] = nl > 0 ? 1 : 0;
}

// Exclusive scan of the 256 per-thread values of a workgroup; returns this
// thread's prefix and writes the workgroup total to *total.
__device__ int block_exclusive_scan(int v, int *s_wave, int *total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  int wave_prefix = 0, sum = 0;
  for (int w = 0; w < SCAN_WG / 64; ++w) {
    if (w < wave) wave_prefix += s_wave[w];
    sum += s_wave[w];
  }
  __syncthreads();
  *total = sum;
  return wave_prefix + incl - v;
}

__global__ __launch_bounds__(SCAN_WG) void k_scan_reduce(const int32_t *__restrict__ in, int64_t n,
                                                         int32_t *__restrict__ partial) {
  __shared__ int s_wave[SCAN_WG / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
  int s = 0;
#pragma unroll
  for (int e = 0; e < SCAN_PER; ++e)
    if (base + e < n) s += in[base + e];
  int total;
  (void)block_exclusive_scan(s, s_wave, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of the chunk totals, in place.
__global__ __launch_bounds__(SCAN_WG) void k_scan_partials(int32_t *partial, int64_t nb) {
  __shared__ int s_wave[SCAN_WG / 64];
  int carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += SCAN_WG) {
    const int64_t b = b0 + threadIdx.x;
    const int v = b < nb ? partial[b] : 0;
    int total;
    const int ex = block_exclusive_scan(v, s_wave, &total);
    if (b < nb) partial[b] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(SCAN_WG) void k_scan_apply(const int32_t *in, int32_t *out, int64_t n,
                                                        const int32_t *__restrict__ partial) {
  __shared__ int s_wave[SCAN_WG / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
  int v[SCAN_PER];
  int s = 0;
#pragma unroll
  for (int e = 0; e < SCAN_PER; ++e) {
    v[e] = base + e < n ? in[base + e] : 0;
    s += v[e];
  }
  int total;
  int run = block_exclusive_scan(s, s_wave, &total) + partial[blockIdx.x];
#pragma unroll
  for (int e = 0; e < SCAN_PER; ++e) {
    if (base + e < n) out[base + e] = run;
    run += v[e];
  }
}

// In-place exclusive scan of n int32 values (n >= 1).
hipError_t scan_exclusive(int32_t *data, int64_t n, int32_t *tmp, hipStream_t s) {
  const int64_t nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_WG), 0, s, data, n, tmp);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_WG), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_WG), 0, s, data, data, n, tmp);
  return hipGetLastError();
}

template <class T>
__global__ void k_split_fill(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                             const T *__restrict__ val, int64_t n, int32_t h,
                             const int32_t *__restrict__ w_loc, const int32_t *__restrict__ w_nl,
                             const int32_t *__restrict__ w_flag, int32_t *__restrict__ loc_row_ptr,
                             int32_t *__restrict__ loc_col, T *__restrict__ loc_val,
                             int32_t *__restrict__ nl_rows, int32_t *__restrict__ nl_ptr,
                             int32_t *__restrict__ nl_col, T *__restrict__ nl_val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    loc_row_ptr[n] = w_loc[n];
    nl_ptr[w_flag[n]] = w_nl[n];
  }
  if (i >= n) return;
  int lo = w_loc[i];
  int no = w_nl[i];
  loc_row_ptr[i] = lo;
  const int pos = w_flag[i];
  if (w_flag[i + 1] > pos) {
    nl_rows[pos] = (int32_t)i;
    nl_ptr[pos] = no;
  }
  for (int j = rp[i]; j < rp[i + 1]; ++j) {
    const int c = col[j];
    if (c < h) {
      loc_col[lo] = c;
      loc_val[lo] = val[j];
      ++lo;
    } else {
      nl_col[no] = c;
      nl_val[no] = val[j];
      ++no;
    }
  }
}

// ---- diagonal panels --------------------------------------------------------
// Panel of an entry: its offset d = col - row placed in one of K equal
// slices of [dmin, dmin + span).
__device__ __forceinline__ int panel_of(int64_t d, int64_t dmin, int64_t span, int K) {
  const int64_t q = ((d - dmin) * K) / span;
  return (int)(q < 0 ? 0 : (q >= K ? K - 1 : q));
}

__global__ void k_d_range(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t n,
                          int64_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  if (i < n)
    for (int j = rp[i]; j < rp[i + 1]; ++j) {
      const int64_t d = (int64_t)col[j] - i;
      lo = d < lo ? d : lo;
      hi = d > hi ? d : hi;
    }
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t a = __shfl_xor(lo, off), b = __shfl_xor(hi, off);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  if ((threadIdx.x & 63) == 0 && lo <= hi) {
    atomicMin((unsigned long long *)&out[0], (unsigned long long)(lo + ((int64_t)1 << 40)));
    atomicMax((unsigned long long *)&out[1], (unsigned long long)(hi + ((int64_t)1 << 40)));
  }
}

// counts: K arrays of n + 1 entries (entry n is a zero pad for the scan)
__global__ void k_panel_count(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                              int64_t n, int64_t dmin, int64_t span, int K,
                              int32_t *__restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  int c[PANEL_MAX] = {0};
  if (i < n)
    for (int j = rp[i]; j < rp[i + 1]; ++j) ++c[panel_of((int64_t)col[j] - i, dmin, span, K)];
  for (int k = 0; k < K; ++k) counts[(int64_t)k * (n + 1) + i] = c[k];
}

template <class T>
__global__ void k_panel_fill(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                             const T *__restrict__ val, int64_t n, int64_t dmin, int64_t span, int K,
                             const int32_t *__restrict__ starts, PanelOut out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int pos[PANEL_MAX];
  for (int k = 0; k < K; ++k) pos[k] = starts[(int64_t)k * (n + 1) + i];
  for (int j = rp[i]; j < rp[i + 1]; ++j) {
    const int k = panel_of((int64_t)col[j] - i, dmin, span, K);
    out.col[k][pos[k]] = col[j];
    static_cast<T *>(out.val[k])[pos[k]] = val[j];
    ++pos[k];
  }
}

}  // namespace

hipError_t panel_d_range(const int32_t *row_ptr, const int32_t *col, int64_t n_rows, int64_t *dev2,
                         int64_t *dmin, int64_t *dmax, hipStream_t s) {
  const int64_t init[2] = {INT64_MAX, 0};
  hipError_t e = hipMemcpyAsync(dev2, init, sizeof(init), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  if (n_rows > 0)
    hipLaunchKernelGGL(k_d_range, dim3((unsigned)((n_rows + 255) / 256)), dim3(256), 0, s, row_ptr,
                       col, n_rows, dev2);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t r[2];
  e = hipMemcpyAsync(r, dev2, sizeof(r), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if (r[0] == INT64_MAX) {  // no entries
    *dmin = 0;
    *dmax = 0;
  } else {
    *dmin = r[0] - ((int64_t)1 << 40);
    *dmax = r[1] - ((int64_t)1 << 40);
  }
  return hipSuccess;
}

hipError_t panel_count(const int32_t *row_ptr, const int32_t *col, int64_t n_rows, int64_t dmin,
                       int64_t span, int K, int32_t *counts, int32_t *scan_tmp, hipStream_t s) {
  const int64_t m = n_rows + 1;
  hipLaunchKernelGGL(k_panel_count, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, row_ptr, col,
                     n_rows, dmin, span, K, counts);
  hipError_t e = hipGetLastError();
  for (int k = 0; k < K && e == hipSuccess; ++k) e = scan_exclusive(counts + (int64_t)k * m, m, scan_tmp, s);
  return e;
}

hipError_t panel_fill(int prec, const int32_t *row_ptr, const int32_t *col, const void *val,
                      int64_t n_rows, int64_t dmin, int64_t span, int K, const int32_t *starts,
                      const PanelOut &out, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((n_rows + 255) / 256);
  switch (val_bytes(prec)) {
    case 8:
      hipLaunchKernelGGL(k_panel_fill<uint64_t>, dim3(nb), dim3(256), 0, s, row_ptr, col,
                         static_cast<const uint64_t *>(val), n_rows, dmin, span, K, starts, out);
      break;
    case 4:
      hipLaunchKernelGGL(k_panel_fill<uint32_t>, dim3(nb), dim3(256), 0, s, row_ptr, col,
                         static_cast<const uint32_t *>(val), n_rows, dmin, span, K, starts, out);
      break;
    default:
      hipLaunchKernelGGL(k_panel_fill<uint16_t>, dim3(nb), dim3(256), 0, s, row_ptr, col,
                         static_cast<const uint16_t *>(val), n_rows, dmin, span, K, starts, out);
      break;
  }
  return hipGetLastError();
}

int64_t split_work_elems(int64_t n_rows) { return 3 * (n_rows + 1); }
int64_t scan_tmp_elems(int64_t n) { return (n + SCAN_CHUNK - 1) / SCAN_CHUNK + 1; }

hipError_t split_count(const int32_t *row_ptr, const int32_t *col, int64_t n_rows, int32_t h,
                       int32_t *work, int32_t *scan_tmp, int64_t *nnz_loc, int64_t *nnz_nl,
                       int64_t *n_nl_rows, hipStream_t s) {
  const int64_t m = n_rows + 1;
  int32_t *w_loc = work, *w_nl = work + m, *w_flag = work + 2 * m;
  const int64_t nb = (m + 255) / 256;
  hipLaunchKernelGGL(k_split_count, dim3((unsigned)nb), dim3(256), 0, s, row_ptr, col, n_rows, h,
                     w_loc, w_nl, w_flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int32_t *a : {w_loc, w_nl, w_flag}) {
    e = scan_exclusive(a, m, scan_tmp, s);
    if (e != hipSuccess) return e;
  }
  int32_t tot[3];
  for (int q = 0; q < 3; ++q) {
    e = hipMemcpyAsync(&tot[q], work + q * m + n_rows, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  *nnz_loc = tot[0];
  *nnz_nl = tot[1];
  *n_nl_rows = tot[2];
  return hipSuccess;
}

hipError_t split_fill(int prec, const int32_t *row_ptr, const int32_t *col, const void *val,
                      int64_t n_rows, int32_t h, const int32_t *work, int64_t, int64_t,
                      const SplitOut &o, hipStream_t s) {
  const int64_t m = n_rows + 1;
  const int32_t *w_loc = work, *w_nl = work + m, *w_flag = work + 2 * m;
  const int64_t nb = (n_rows > 0 ? n_rows + 255 : 256) / 256;
  switch (val_bytes(prec)) {
    case 8:
      hipLaunchKernelGGL(k_split_fill<uint64_t>, dim3((unsigned)nb), dim3(256), 0, s, row_ptr, col,
                         static_cast<const uint64_t *>(val), n_rows, h, w_loc, w_nl, w_flag,
                         o.loc_row_ptr, o.loc_col, static_cast<uint64_t *>(o.loc_val), o.nl_rows,
                         o.nl_ptr, o.nl_col, static_cast<uint64_t *>(o.nl_val));
      break;
    case 4:
      hipLaunchKernelGGL(k_split_fill<uint32_t>, dim3((unsigned)nb), dim3(256), 0, s, row_ptr, col,
                         static_cast<const uint32_t *>(val), n_rows, h, w_loc, w_nl, w_flag,
                         o.loc_row_ptr, o.loc_col, static_cast<uint32_t *>(o.loc_val), o.nl_rows,
                         o.nl_ptr, o.nl_col, static_cast<uint32_t *>(o.nl_val));
      break;
    default:
      hipLaunchKernelGGL(k_split_fill<uint16_t>, dim3((unsigned)nb), dim3(256), 0, s, row_ptr, col,
                         static_cast<const uint16_t *>(val), n_rows, h, w_loc, w_nl, w_flag,
                         o.loc_row_ptr, o.loc_col, static_cast<uint16_t *>(o.loc_val), o.nl_rows,
                         o.nl_ptr, o.nl_col, static_cast<uint16_t *>(o.nl_val));
      break;
  }
  return hipGetLastError();
}

}  // namespace spmv
