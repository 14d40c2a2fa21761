// Measurement probes.
//   copy / triad / read: the bandwidth ceilings the spMV is compared with, in the
//     role the STREAM triad plays in Sect. 2 of Schubert, Fehske, Hager,
//     Wellein 2011 (GPU stores do not write-allocate, so no 4/3 scaling);
//   atomic: throughput of FP64 atomic adds into HBM, coalesced or scattered
//     (what a scatter into C, such as the transposed half of a symmetric
//     product, would pay per contribution);
//   gather: the indexed loads of B alone -- a stream of int32 indices read
//     with coalesced loads and, for each index, W consecutive doubles gathered
//     from B (W = 1 for one right-hand side, W = k for a row-major block) --
//     the part of the spMV whose extra traffic the paper calls kappa
//     (Sect. 1.2, Eq. (1)); fed with a matrix's own col_idx it gives the rate
//     the product's gathers alone reach, with random indices in a window of
//     chosen size the rate of the cache level that window fits;
//   spin: a workgroup that stays busy for a given time without touching
//     memory, the device-side "do_work" of the asynchrony test of Listing 2
//     (Sect. 3.1), used to check that a host-to-device copy on another stream
//     really proceeds while a kernel runs.
#include <hip/hip_runtime.h>

#include "spmv_internal.h"

namespace spmv {
namespace {

constexpr int WG = 256;
constexpr int PER = 4;  // 16-byte elements per thread

typedef double dv2 __attribute__((ext_vector_type(2)));

// Copy and triad use nontemporal loads and stores (the fastest of the
// variants measured on MI355X), four 16-byte elements per thread.
__global__ __launch_bounds__(WG) void k_copy(dv2 *__restrict__ dst, const dv2 *__restrict__ src,
                                             int64_t n2) {
  const int64_t base = ((int64_t)blockIdx.x * WG * PER) + threadIdx.x;
  dv2 v[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t i = base + (int64_t)e * WG;
    if (i < n2) v[e] = __builtin_nontemporal_load(src + i);
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t i = base + (int64_t)e * WG;
    if (i < n2) __builtin_nontemporal_store(v[e], dst + i);
  }
}

__global__ __launch_bounds__(WG) void k_triad(dv2 *__restrict__ a, const dv2 *__restrict__ b,
                                              const dv2 *__restrict__ c, double s, int64_t n2) {
  const int64_t base = ((int64_t)blockIdx.x * WG * PER) + threadIdx.x;
  dv2 vb[PER], vc[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t i = base + (int64_t)e * WG;
    if (i < n2) {
      vb[e] = __builtin_nontemporal_load(b + i);
      vc[e] = __builtin_nontemporal_load(c + i);
    }
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t i = base + (int64_t)e * WG;
    if (i < n2) __builtin_nontemporal_store(vb[e] + s * vc[e], a + i);
  }
}

// Read-only stream: sums the input; one value per workgroup is written.
__global__ __launch_bounds__(WG) void k_read(const dv2 *__restrict__ src, int64_t n2,
                                             double *__restrict__ sums) {
  __shared__ double s_red[WG];
  const int64_t base = ((int64_t)blockIdx.x * WG * PER) + threadIdx.x;
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t i = base + (int64_t)e * WG;
    if (i < n2) {
      const dv2 v = __builtin_nontemporal_load(src + i);
      acc += v.x + v.y;
    }
  }
  s_red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = WG / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s_red[threadIdx.x] += s_red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = s_red[0];
}

// Scalar tail for odd n (element n-1).
__global__ void k_copy_tail(double *dst, const double *src, int64_t i) {
  if (threadIdx.x == 0) dst[i] = src[i];
}
__global__ void k_triad_tail(double *a, const double *b, const double *c, double s, int64_t i) {
  if (threadIdx.x == 0) a[i] = b[i] + s * c[i];
}

// FP64 atomic adds of 1.0 into C[0, n) (n a power of two): each thread adds
// `iters` times, at position (wave-block * 64 + lane) for the coalesced
// pattern (a wave's 64 lanes hit 512 consecutive bytes) or at a hashed
// position for the scattered one.  Vector global atomics only.
__device__ __forceinline__ uint32_t mix32(uint32_t a) {
  a ^= a >> 16;
  a *= 0x7feb352du;
  a ^= a >> 15;
  a *= 0x846ca68bu;
  a ^= a >> 16;
  return a;
}

__global__ __launch_bounds__(WG) void k_atomic(double *__restrict__ C, uint32_t mask, int scattered,
                                               int iters) {
  const uint32_t g = blockIdx.x * (uint32_t)WG + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u, wave = g >> 6;
  for (int i = 0; i < iters; ++i) {
    const uint32_t idx = scattered ? (mix32(g * 1009u + (uint32_t)i) & mask)
                                   : (((wave * 977u + (uint32_t)i * 131u) * 64u + lane) & mask);
    unsafeAtomicAdd(C + idx, 1.0);
  }
}

// Gathers: lane group g of L = max(1, W/2) lanes takes indices
// base + e*NI + g (e < GE, NI = 256 / L indices per pass), loads all GE indices
// first (coalesced, streaming hint), then gathers row idx of src (W doubles,
// 16 bytes per lane, or 8 bytes for W = 1).  Indices are clamped into
// [0, n_rows) so no load leaves src.  Workgroups are placed on the XCDs as
// the stream kernel places its tiles (contiguous ranges per XCD when remap
// is set).  Each workgroup writes the sum of what it gathered.
constexpr int GE = 8;

__device__ __forceinline__ int64_t probe_tile(int64_t bid, int64_t n, int remap) {
  if (!remap) return bid;
  const int64_t x = bid % 8, i = bid / 8;
  const int64_t q = n / 8, r = n % 8;
  return x * q + (x < r ? x : r) + i;
}

template <int W>
__global__ __launch_bounds__(WG) void k_gather(const double *__restrict__ src, int64_t n_rows,
                                               const int32_t *__restrict__ idx, int64_t n,
                                               int remap, double *__restrict__ sums) {
  constexpr int L = W >= 2 ? W / 2 : 1;
  constexpr int NI = WG / L;
  __shared__ double s_red[WG];
  const int64_t b = probe_tile(blockIdx.x, gridDim.x, remap);
  const int64_t base = b * NI * GE;
  const int g = (int)threadIdx.x / L, lane = (int)threadIdx.x % L;
  int64_t c[GE];
#pragma unroll
  for (int e = 0; e < GE; ++e) {
    const int64_t j = base + (int64_t)e * NI + g;
    const int64_t v = j < n ? (int64_t)__builtin_nontemporal_load(idx + j) : 0;
    c[e] = v < 0 ? 0 : (v >= n_rows ? n_rows - 1 : v);
  }
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < GE; ++e) {
    const bool in = base + (int64_t)e * NI + g < n;
    if constexpr (W == 1) {
      const double v = src[c[e]];
      acc += in ? v : 0.0;
    } else {
      const dv2 v = *reinterpret_cast<const dv2 *>(src + c[e] * W + 2 * lane);
      acc += in ? v.x + v.y : 0.0;
    }
  }
  s_red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = WG / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s_red[threadIdx.x] += s_red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = s_red[0];
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
    hipLaunchKernelGGL(k_copy, dim3((unsigned)nb), dim3(WG), 0, s, reinterpret_cast<dv2 *>(dst),
                       reinterpret_cast<const dv2 *>(src), n2);
  }
  if (n % 2) hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, s, dst, src, n - 1);
  return hipGetLastError();
}

hipError_t launch_triad(double *a, const double *b, const double *c, double sc, int64_t n,
                        hipStream_t s) {
  const int64_t n2 = n / 2;
  if (n2 > 0) {
    const int64_t nb = (n2 + WG * PER - 1) / (WG * PER);
    hipLaunchKernelGGL(k_triad, dim3((unsigned)nb), dim3(WG), 0, s, reinterpret_cast<dv2 *>(a),
                       reinterpret_cast<const dv2 *>(b), reinterpret_cast<const dv2 *>(c), sc, n2);
  }
  if (n % 2) hipLaunchKernelGGL(k_triad_tail, dim3(1), dim3(64), 0, s, a, b, c, sc, n - 1);
  return hipGetLastError();
}

int64_t read_sums_needed(int64_t n) { return (n / 2 + WG * PER - 1) / (WG * PER) + 1; }

hipError_t launch_read(const double *src, int64_t n, double *sums, hipStream_t s) {
  const int64_t n2 = n / 2;
  if (n2 > 0) {
    const int64_t nb = (n2 + WG * PER - 1) / (WG * PER);
    hipLaunchKernelGGL(k_read, dim3((unsigned)nb), dim3(WG), 0, s,
                       reinterpret_cast<const dv2 *>(src), n2, sums);
  }
  return hipGetLastError();
}

hipError_t launch_atomic(double *C, int64_t n, int scattered, int iters, hipStream_t s) {
  hipLaunchKernelGGL(k_atomic, dim3(ATOMIC_BLOCKS), dim3(WG), 0, s, C, (uint32_t)(n - 1),
                     scattered, iters);
  return hipGetLastError();
}

int64_t gather_sums_needed(int64_t n, int width) {
  const int64_t per = (int64_t)(WG / (width >= 2 ? width / 2 : 1)) * GE;
  return n > 0 ? (n + per - 1) / per : 0;
}

template <int W>
static void gather_w(const double *src, int64_t n_rows, const int32_t *idx, int64_t n, int remap,
                     double *sums, hipStream_t s) {
  const int64_t nb = gather_sums_needed(n, W);
  hipLaunchKernelGGL(k_gather<W>, dim3((unsigned)nb), dim3(WG), 0, s, src, n_rows, idx, n, remap,
                     sums);
}

hipError_t launch_gather(const double *src, int64_t n_rows, const int32_t *idx, int64_t n,
                         int width, int remap, double *sums, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (width) {
    case 1: gather_w<1>(src, n_rows, idx, n, remap, sums, s); break;
    case 2: gather_w<2>(src, n_rows, idx, n, remap, sums, s); break;
    case 4: gather_w<4>(src, n_rows, idx, n, remap, sums, s); break;
    case 8: gather_w<8>(src, n_rows, idx, n, remap, sums, s); break;
    case 16: gather_w<16>(src, n_rows, idx, n, remap, sums, s); break;
    default: return hipErrorInvalidValue;
  }
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
