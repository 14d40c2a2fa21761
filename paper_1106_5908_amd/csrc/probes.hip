// Measurement probes.
//   copy / triad: the bandwidth ceiling the spMV is compared with, in the
//     role the STREAM triad plays in Sect. 2 of Schubert, Fehske, Hager,
//     Wellein 2011 (GPU stores do not write-allocate, so no 4/3 scaling);
//   spin: a workgroup that stays busy for a given time without touching
//     memory, the device-side "do_work" of the asynchrony test of Listing 2
//     (Sect. 3.1), used to check that a host-to-device copy on another stream
//     really proceeds while a kernel runs.
#include <hip/hip_runtime.h>

#include "spmv_internal.h"

namespace spmv {
namespace {

constexpr int WG = 256;
constexpr int PER = 4;  // double2 per thread

__global__ __launch_bounds__(WG) void k_copy(double2 *__restrict__ dst,
                                             const double2 *__restrict__ src, int64_t n2) {
  const int64_t base = ((int64_t)blockIdx.x * WG * PER) + threadIdx.x;
  double2 v[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t i = base + (int64_t)e * WG;
    if (i < n2) v[e] = src[i];
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t i = base + (int64_t)e * WG;
    if (i < n2) dst[i] = v[e];
  }
}

__global__ __launch_bounds__(WG) void k_triad(double2 *__restrict__ a,
                                              const double2 *__restrict__ b,
                                              const double2 *__restrict__ c, double s, int64_t n2) {
  const int64_t base = ((int64_t)blockIdx.x * WG * PER) + threadIdx.x;
  double2 vb[PER], vc[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t i = base + (int64_t)e * WG;
    if (i < n2) {
      vb[e] = b[i];
      vc[e] = c[i];
    }
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t i = base + (int64_t)e * WG;
    if (i < n2) a[i] = make_double2(vb[e].x + s * vc[e].x, vb[e].y + s * vc[e].y);
  }
}

// Scalar tail for odd n (element n-1).
__global__ void k_copy_tail(double *dst, const double *src, int64_t i) {
  if (threadIdx.x == 0) dst[i] = src[i];
}
__global__ void k_triad_tail(double *a, const double *b, const double *c, double s, int64_t i) {
  if (threadIdx.x == 0) a[i] = b[i] + s * c[i];
}

// Busy-waits until `ticks` ticks of the constant-rate wall clock have passed.
__global__ void k_spin(int64_t ticks) {
  const int64_t t0 = wall_clock64();
  while (wall_clock64() - t0 < ticks) {
    __builtin_amdgcn_s_sleep(1);
  }
}

}  // namespace

hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t s) {
  const int64_t n2 = n / 2;
  if (n2 > 0) {
    const int64_t nb = (n2 + WG * PER - 1) / (WG * PER);
    hipLaunchKernelGGL(k_copy, dim3((unsigned)nb), dim3(WG), 0, s,
                       reinterpret_cast<double2 *>(dst), reinterpret_cast<const double2 *>(src), n2);
  }
  if (n % 2) hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, s, dst, src, n - 1);
  return hipGetLastError();
}

hipError_t launch_triad(double *a, const double *b, const double *c, double sc, int64_t n,
                        hipStream_t s) {
  const int64_t n2 = n / 2;
  if (n2 > 0) {
    const int64_t nb = (n2 + WG * PER - 1) / (WG * PER);
    hipLaunchKernelGGL(k_triad, dim3((unsigned)nb), dim3(WG), 0, s, reinterpret_cast<double2 *>(a),
                       reinterpret_cast<const double2 *>(b), reinterpret_cast<const double2 *>(c),
                       sc, n2);
  }
  if (n % 2) hipLaunchKernelGGL(k_triad_tail, dim3(1), dim3(64), 0, s, a, b, c, sc, n - 1);
  return hipGetLastError();
}

hipError_t launch_spin(int64_t nanoseconds, hipStream_t s) {
  int dev = 0, rate_khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return e;
  const int64_t ticks = nanoseconds * (int64_t)rate_khz / 1000000;
  hipLaunchKernelGGL(k_spin, dim3(1), dim3(64), 0, s, ticks);
  return hipGetLastError();
}

}  // namespace spmv
