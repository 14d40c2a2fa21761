// Send side of the halo exchange of Schubert, Fehske, Hager, Wellein 2011:
// the elements of B that another process needs are gathered into one
// contiguous send buffer (Sect. 3.3) before they are communicated; in task
// mode (Sect. 3.5) this gather runs beside the local part of the product.
//
// The gather moves bits, not numbers: elements are copied as 4- or 8-byte
// words, so NaN payloads and signed zeros arrive unchanged.
#include <hip/hip_runtime.h>

#include "spmv_internal.h"

namespace spmv {
namespace {

constexpr int WG = 256;

// out[k] = B[idx[k]] for k < n.  Grid-stride: the grid is capped and every
// thread walks k, k + stride, ... so any n up to 2^31 - 1 is covered.
template <class W>
__global__ __launch_bounds__(WG) void k_pack(const W *__restrict__ B, const int32_t *__restrict__ idx,
                                             int64_t n, W *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * WG;
  for (int64_t k = (int64_t)blockIdx.x * WG + threadIdx.x; k < n; k += stride) out[k] = B[idx[k]];
}

}  // namespace

hipError_t launch_pack(int word_bytes, const void *B, const int32_t *idx, int64_t n, void *out,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + WG - 1) / WG;
  const unsigned grid = (unsigned)(want < 8192 ? want : 8192);
  if (word_bytes == 8)
    hipLaunchKernelGGL(k_pack<uint64_t>, dim3(grid), dim3(WG), 0, s,
                       static_cast<const uint64_t *>(B), idx, n, static_cast<uint64_t *>(out));
  else
    hipLaunchKernelGGL(k_pack<uint32_t>, dim3(grid), dim3(WG), 0, s,
                       static_cast<const uint32_t *>(B), idx, n, static_cast<uint32_t *>(out));
  return hipGetLastError();
}

}  // namespace spmv
