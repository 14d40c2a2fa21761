// Vector kernels of the Lanczos iteration (the eigensolver that Schubert,
// Fehske, Hager, Wellein 2011 name first among the algorithms whose time goes
// into the spMV, Sect. 1.3).  The product is the library's CRS kernel; these
// kernels do the O(N) work of a step with the scalars alpha_j and beta_j kept
// in device memory, so a whole run of m steps is enqueued without the host
// waiting for any of them.
//
// Every dot product and norm is reduced in a fixed order (per-thread sums over
// a fixed grid, a per-workgroup tree, then one workgroup over the partials),
// so repeated runs give identical coefficients.
#include <hip/hip_runtime.h>

#include <math.h>

#include "spmv_internal.h"

namespace spmv {
namespace {

constexpr int WG = 256;

unsigned grid_for(int64_t n) {
  const int64_t want = (n + WG - 1) / WG;
  return (unsigned)(want < KPM_GRID ? (want > 0 ? want : 1) : KPM_GRID);
}

__device__ __forceinline__ void wg_sum(double a, double *s, double *out) {
  const int tid = threadIdx.x;
  s[tid] = a;
  __syncthreads();
  for (int off = WG / 2; off > 0; off >>= 1) {
    if (tid < off) s[tid] += s[tid + off];
    __syncthreads();
  }
  if (tid == 0) out[blockIdx.x] = s[0];
}

// Sum of the n_parts partials in a fixed order; sqrt of it if `root`.
__global__ __launch_bounds__(WG) void k_lz_finish(const double *__restrict__ part, int n_parts,
                                                  int root, double *__restrict__ out) {
  __shared__ double s[WG];
  double a = 0.0;
  for (int w = threadIdx.x; w < n_parts; w += WG) a += part[w];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int off = WG / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = root ? sqrt(s[0]) : s[0];
}

// partials of q.q
__global__ __launch_bounds__(WG) void k_lz_sq(const double *__restrict__ q, int64_t n,
                                              double *__restrict__ part) {
  __shared__ double s[WG];
  const int64_t stride = (int64_t)gridDim.x * WG;
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) a += q[i] * q[i];
  wg_sum(a, s, part);
}

// V = q / |q| (0 if q = 0)
__global__ __launch_bounds__(WG) void k_lz_start(const double *__restrict__ q,
                                                 double *__restrict__ V, int64_t n,
                                                 const double *__restrict__ norm) {
  const double nq = *norm;
  const int64_t stride = (int64_t)gridDim.x * WG;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride)
    V[i] = nq > 0.0 ? q[i] / nq : 0.0;
}

// partials of W.V
__global__ __launch_bounds__(WG) void k_lz_dot(const double *__restrict__ W,
                                               const double *__restrict__ V, int64_t n,
                                               double *__restrict__ part) {
  __shared__ double s[WG];
  const int64_t stride = (int64_t)gridDim.x * WG;
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) a += W[i] * V[i];
  wg_sum(a, s, part);
}

// W = W - alpha V and partials of W.W
__global__ __launch_bounds__(WG) void k_lz_update(double *__restrict__ W,
                                                  const double *__restrict__ V, int64_t n,
                                                  const double *__restrict__ alpha,
                                                  double *__restrict__ part) {
  __shared__ double s[WG];
  const double al = *alpha;
  const int64_t stride = (int64_t)gridDim.x * WG;
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
    const double w = W[i] - al * V[i];
    W[i] = w;
    a += w * w;
  }
  wg_sum(a, s, part);
}

// W = W / beta (0 if beta = 0): the next Lanczos vector; V = -beta V: the
// term the next product accumulates onto.
__global__ __launch_bounds__(WG) void k_lz_next(double *__restrict__ W, double *__restrict__ V,
                                                int64_t n, const double *__restrict__ beta) {
  const double b = *beta;
  const int64_t stride = (int64_t)gridDim.x * WG;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
    W[i] = b > 0.0 ? W[i] / b : 0.0;
    V[i] = -(b * V[i]);
  }
}

}  // namespace

hipError_t launch_lz_start(const double *q, double *V, int64_t n, double *part, hipStream_t s) {
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(k_lz_sq, dim3(g), dim3(WG), 0, s, q, n, part);
  hipLaunchKernelGGL(k_lz_finish, dim3(1), dim3(WG), 0, s, part, (int)g, 1, part + KPM_GRID);
  hipLaunchKernelGGL(k_lz_start, dim3(g), dim3(WG), 0, s, q, V, n, part + KPM_GRID);
  return hipGetLastError();
}

hipError_t launch_lz_step(double *W, double *V, int64_t n, double *part, double *alpha,
                          double *beta, hipStream_t s) {
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(k_lz_dot, dim3(g), dim3(WG), 0, s, W, V, n, part);
  hipLaunchKernelGGL(k_lz_finish, dim3(1), dim3(WG), 0, s, part, (int)g, 0, alpha);
  hipLaunchKernelGGL(k_lz_update, dim3(g), dim3(WG), 0, s, W, V, n, alpha, part);
  hipLaunchKernelGGL(k_lz_finish, dim3(1), dim3(WG), 0, s, part, (int)g, 1, beta);
  hipLaunchKernelGGL(k_lz_next, dim3(g), dim3(WG), 0, s, W, V, n, beta);
  return hipGetLastError();
}

}  // namespace spmv
