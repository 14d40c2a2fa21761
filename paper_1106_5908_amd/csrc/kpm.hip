// Vector kernels of the Chebyshev-moment loop of the kernel polynomial method
// (the polynomial-expansion methods for spectral properties that Schubert,
// Fehske, Hager, Wellein 2011 name as an application whose cost is the
// spMV, Sect. 1.3).  The product itself is the block kernel; these kernels
// do the O(N) work between products.
//
// The loop keeps z_n = c_n v_n with c_n = 1, 1, -1, -1, 1, 1, ... (period
// four), for which the three-term recursion becomes one in-place product
// z_{n+1} = z_{n-1} + 2 (c_{n+1}/c_n) H z_n.  Then |z_n|^2 = |v_n|^2 and
// <v_{n+1}|v_n> = (c_{n+1}/c_n) <z_{n+1}|z_n>, with c_{n+1}/c_n = +1 for n
// even and -1 for n odd.
//
// Vectors are blocks of R columns stored row-major (element (i, r) at
// i*R + r), R a power of two <= 64, as the block product reads and writes
// them.  Every dot product is reduced in a fixed order (per-thread partial
// sums, a per-workgroup tree, then one pass over the workgroups), so results
// are reproducible from run to run.
#include <hip/hip_runtime.h>

#include "spmv_internal.h"

namespace spmv {
namespace {

constexpr int WG = 256;

// Thread t of the grid touches elements t, t + S, t + 2S, ... with the grid
// size S a multiple of R, so all of them lie in column t % R.
__device__ __forceinline__ void wg_column_sums(double a, double b, int R, double *s_a, double *s_b,
                                               double *out_a, double *out_b) {
  const int tid = threadIdx.x;
  s_a[tid] = a;
  s_b[tid] = b;
  __syncthreads();
  for (int off = WG / 2; off >= R; off >>= 1) {
    if (tid < off) {
      s_a[tid] += s_a[tid + off];
      s_b[tid] += s_b[tid + off];
    }
    __syncthreads();
  }
  if (tid < R) {
    out_a[(int64_t)blockIdx.x * R + tid] = s_a[tid];
    out_b[(int64_t)blockIdx.x * R + tid] = s_b[tid];
  }
}

// First step: with W1 = H v0 = z1 (v0 = V0), partial sums of <v0|v0> and
// <W1|v0> per column, and W2 = v0 = z0, the vector the next product
// accumulates onto (V0 itself stays untouched).
__global__ __launch_bounds__(WG) void k_kpm_first(const double *__restrict__ V0,
                                                  const double *__restrict__ W1,
                                                  double *__restrict__ W2, int64_t n, int R,
                                                  double *__restrict__ part_a,
                                                  double *__restrict__ part_b) {
  __shared__ double s_a[WG], s_b[WG];
  const int64_t stride = (int64_t)gridDim.x * WG;
  double a = 0.0, b = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < n; e += stride) {
    const double v = V0[e];
    a += v * v;
    b += W1[e] * v;
    W2[e] = v;
  }
  wg_column_sums(a, b, R, s_a, s_b, part_a, part_b);
}

// Step n >= 1: X = z_n, P = z_{n+1}.  Partial sums of <z_n|z_n> and
// <z_{n+1}|z_n>; nothing is written back.
__global__ __launch_bounds__(WG) void k_kpm_step(const double *__restrict__ X,
                                                 const double *__restrict__ P, int64_t n, int R,
                                                 double *__restrict__ part_a,
                                                 double *__restrict__ part_b) {
  __shared__ double s_a[WG], s_b[WG];
  const int64_t stride = (int64_t)gridDim.x * WG;
  double a = 0.0, b = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < n; e += stride) {
    const double x = X[e];
    a += x * x;
    b += P[e] * x;
  }
  wg_column_sums(a, b, R, s_a, s_b, part_a, part_b);
}

// Sums the per-workgroup partials of each column and writes the moments:
// first step (first != 0): mu[0] = <v0|v0>, mu[1] = <v1|v0>; step n:
// mu[2n] = 2 <v_n|v_n> - mu[0], mu[2n+1] = 2 <v_{n+1}|v_n> - mu[1], the dot
// products taken from those of z (see above); moments at or past M are not
// written.  One workgroup: thread t sums column t % R
// over the partials t / R, t / R + WG / R, ... (each pass of the workgroup
// reads WG consecutive doubles), then a fixed tree over the WG / R groups.
__global__ __launch_bounds__(WG) void k_kpm_finish(const double *__restrict__ part_a,
                                                   const double *__restrict__ part_b, int n_parts,
                                                   int R, int first, int step, int M,
                                                   double *__restrict__ mu) {
  __shared__ double s_a[WG], s_b[WG];
  const int tid = threadIdx.x;
  const int groups = WG / R;
  double a = 0.0, b = 0.0;
  for (int w = tid / R; w < n_parts; w += groups) {
    a += part_a[(int64_t)w * R + tid % R];
    b += part_b[(int64_t)w * R + tid % R];
  }
  s_a[tid] = a;
  s_b[tid] = b;
  __syncthreads();
  for (int off = WG / 2; off >= R; off >>= 1) {
    if (tid < off) {
      s_a[tid] += s_a[tid + off];
      s_b[tid] += s_b[tid + off];
    }
    __syncthreads();
  }
  if (tid >= R) return;
  const int r = tid;
  a = s_a[r];
  b = s_b[r];
  if (first) {
    mu[r] = a;
    if (M > 1) mu[(int64_t)R + r] = b;
  } else {
    const int m0 = 2 * step, m1 = 2 * step + 1;
    if (m0 < M) mu[(int64_t)m0 * R + r] = 2.0 * a - mu[r];
    const double sgn = (step % 2 == 0) ? 1.0 : -1.0;  // c_{n+1} / c_n
    if (m1 < M) mu[(int64_t)m1 * R + r] = 2.0 * (sgn * b) - mu[(int64_t)R + r];
  }
}

__global__ __launch_bounds__(WG) void k_zero(double *__restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * WG;
  for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < n; e += stride) p[e] = 0.0;
}

unsigned grid_for(int64_t n) {
  const int64_t want = (n + WG - 1) / WG;
  return (unsigned)(want < KPM_GRID ? (want > 0 ? want : 1) : KPM_GRID);
}

}  // namespace

hipError_t launch_kpm_zero(double *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(WG), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_kpm_first(const double *V0, const double *W1, double *W2, int64_t n_rows, int R,
                            double *part, int M, double *mu, hipStream_t s) {
  const int64_t n = n_rows * R;
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(k_kpm_first, dim3(g), dim3(WG), 0, s, V0, W1, W2, n, R, part,
                     part + (int64_t)KPM_GRID * R);
  hipLaunchKernelGGL(k_kpm_finish, dim3(1), dim3(WG), 0, s, part, part + (int64_t)KPM_GRID * R,
                     (int)g, R, 1, 0, M, mu);
  return hipGetLastError();
}

hipError_t launch_kpm_step(const double *X, const double *P, int64_t n_rows, int R, double *part,
                           int step, int M, double *mu, hipStream_t s) {
  const int64_t n = n_rows * R;
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(k_kpm_step, dim3(g), dim3(WG), 0, s, X, P, n, R, part,
                     part + (int64_t)KPM_GRID * R);
  hipLaunchKernelGGL(k_kpm_finish, dim3(1), dim3(WG), 0, s, part, part + (int64_t)KPM_GRID * R,
                     (int)g, R, 0, step, M, mu);
  return hipGetLastError();
}

}  // namespace spmv
