// libspmv runtime, solver unit: the two loops of the paper's application
// context that drive the product (Sect. 1.3): the Chebyshev moments of the
// kernel polynomial method (block products) and the Lanczos iteration (one
// product per step), and the Lanczos loop in a form that allocates nothing.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "runtime.h"

using namespace spmv;
using namespace spmv::rt;

// ==== Chebyshev moments (kernel polynomial method) ======================================================

extern "C" spmv_status_t spmv_kpm_moments(spmv_handle_t h_, int32_t R, int32_t M, const double *V0,
                                          double *W1, double *W2, double *mu, void *stream) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    if (h->kind != SPMV_KIND_PLAIN)
      fail(SPMV_ERR_UNSUPPORTED, "spmv_kpm_moments serves plain handles only");
    if (h->prec != P_F64) fail(SPMV_ERR_UNSUPPORTED, "spmv_kpm_moments needs an SPMV_PREC_F64 handle");
    if (h->n_rows != h->n_cols) fail(SPMV_ERR_INVALID_ARG, "the matrix must be square");
    if (R < 1 || R > 64 || (R & (R - 1)) != 0)
      fail(SPMV_ERR_INVALID_ARG, "R must be a power of two in [1, 64]");
    if (M < 1 || M > (1 << 20)) fail(SPMV_ERR_INVALID_ARG, "M must be in [1, 2^20]");
    if (!mu) fail(SPMV_ERR_INVALID_ARG, "mu is null");
    if (h->n_rows > 0 && (!V0 || !W1 || !W2)) fail(SPMV_ERR_INVALID_ARG, "V0, W1 or W2 is null");
    if (h->n_rows > 0 && (V0 == W1 || V0 == W2 || W1 == W2))
      fail(SPMV_ERR_INVALID_ARG, "V0, W1 and W2 must be distinct");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard dg(h->device);
    const size_t need = size_t(2) * KPM_GRID * size_t(R) * sizeof(double);
    if (h->kpm_part.bytes < need) {
      hip_ok(hipDeviceSynchronize(), "synchronize before growing the moment scratch");
      h->kpm_part.alloc(need, "moment partial sums");
    }
    double *part = h->kpm_part.as<double>();
    const int64_t n = h->n_rows;
    // The recursion v_{n+1} = 2 H v_n - v_{n-1} runs on z_n = c_n v_n with
    // c = 1, 1, -1, -1, 1, 1, ...: then z_{n+1} = z_{n-1} + 2 (c_{n+1}/c_n) H z_n,
    // one product accumulating in place onto the older vector with the exact
    // scale +2 (n even) or -2 (n odd), and no pass to negate or halve it.
    hip_ok(launch_kpm_zero(W1, n * R, s), "zero fill");
    block_product(h, R, V0, R, W1, R, s);  // W1 = H v0 = v1 = z1
    hip_ok(launch_kpm_first(V0, W1, W2, n, R, part, M, mu, s), "moment kernels");  // W2 = z0
    double *X = W1, *P = W2;  // X = z_n, P = z_{n-1}
    for (int step = 1; 2 * step < M; ++step) {
      block_product(h, R, X, R, P, R, s, step % 2 == 0 ? 2.0 : -2.0);  // P = z_{n+1}
      hip_ok(launch_kpm_step(X, P, n, R, part, step, M, mu, s), "moment kernels");
      std::swap(X, P);
    }
  });
}

// ==== Lanczos =========================================================================================

extern "C" spmv_status_t spmv_lanczos(spmv_handle_t h_, int32_t m, const double *q, double *V1,
                                      double *V2, double *alpha, double *beta, void *stream) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    if (h->kind != SPMV_KIND_PLAIN) fail(SPMV_ERR_UNSUPPORTED, "spmv_lanczos serves plain handles only");
    if (h->prec != P_F64) fail(SPMV_ERR_UNSUPPORTED, "spmv_lanczos needs an SPMV_PREC_F64 handle");
    if (h->n_rows != h->n_cols) fail(SPMV_ERR_INVALID_ARG, "the matrix must be square");
    if (m < 1 || m > (1 << 20)) fail(SPMV_ERR_INVALID_ARG, "m must be in [1, 2^20]");
    if (!alpha || !beta) fail(SPMV_ERR_INVALID_ARG, "alpha or beta is null");
    if (h->n_rows > 0 && (!q || !V1 || !V2)) fail(SPMV_ERR_INVALID_ARG, "q, V1 or V2 is null");
    if (h->n_rows > 0 && (q == V1 || q == V2 || V1 == V2))
      fail(SPMV_ERR_INVALID_ARG, "q, V1 and V2 must be distinct");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard dg(h->device);
    const size_t need = size_t(2) * KPM_GRID * sizeof(double);
    if (h->kpm_part.bytes < need) {
      hip_ok(hipDeviceSynchronize(), "synchronize before growing the reduction scratch");
      h->kpm_part.alloc(need, "reduction partial sums");
    }
    double *part = h->kpm_part.as<double>();
    const int64_t n = h->n_rows;
    hip_ok(launch_lz_start(q, V1, n, part, s), "Lanczos kernels");
    hip_ok(launch_kpm_zero(V2, n, s), "zero fill");
    double *V = V1, *W = V2;  // V = v_j, W = -beta_{j-1} v_{j-1}
    for (int j = 0; j < m; ++j) {
      run_part(h, h->main, V, W, s);  // W = H v_j - beta_{j-1} v_{j-1}
      hip_ok(launch_lz_step(W, V, n, part, alpha + j, beta + j, s), "Lanczos kernels");
      std::swap(V, W);
    }
  });
}

// ==== Lanczos without allocation =========================================================================

namespace {

// Partial sums of the Lanczos reductions for spmv_lanczos_noalloc.  The
// reduction kernels use at most KPM_GRID workgroups whatever n is, so their
// partials and the one finished scalar (KPM_GRID + 1 doubles) always fit.
// Each device holds its own copy of this array, at its own address, for the
// life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (lz_scratch), never through the
// symbol itself.
constexpr int64_t kLzScratchDoubles = 2 * KPM_GRID;
static __device__ __align__(256) double scratch[kLzScratchDoubles];

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_at;  // device -> address of `scratch` there

// Address of `scratch` on device `dev`, which must be current; looked up
// once per device.
double *lz_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_at.find(dev);
  if (it != g_scratch_at.end()) return it->second;
  void *p = nullptr;
  hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
  if (!p) fail(SPMV_ERR_HIP, "scratch address: null");
  g_scratch_at.emplace(dev, static_cast<double *>(p));
  return static_cast<double *>(p);
}

}  // namespace

extern "C" spmv_status_t spmv_lanczos_noalloc(spmv_handle_t h_, int32_t m, const double *q,
                                              double *V1, double *V2, double *alpha,
                                              double *beta, void *stream) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    if (h->kind != SPMV_KIND_PLAIN)
      fail(SPMV_ERR_UNSUPPORTED, "spmv_lanczos_noalloc serves plain handles only");
    if (h->prec != P_F64)
      fail(SPMV_ERR_UNSUPPORTED, "spmv_lanczos_noalloc needs an SPMV_PREC_F64 handle");
    if (h->n_rows != h->n_cols) fail(SPMV_ERR_INVALID_ARG, "the matrix must be square");
    if (m < 1 || m > (1 << 20)) fail(SPMV_ERR_INVALID_ARG, "m must be in [1, 2^20]");
    if (!alpha || !beta) fail(SPMV_ERR_INVALID_ARG, "alpha or beta is null");
    if (h->n_rows > 0 && (!q || !V1 || !V2)) fail(SPMV_ERR_INVALID_ARG, "q, V1 or V2 is null");
    if (h->n_rows > 0 && (q == V1 || q == V2 || V1 == V2))
      fail(SPMV_ERR_INVALID_ARG, "q, V1 and V2 must be distinct");
    // what the reductions need of the scratch array, whatever n is
    const int64_t need = int64_t(KPM_GRID) + 1;
    if (need > kLzScratchDoubles)
      fail(SPMV_ERR_UNSUPPORTED, "the reductions need " + std::to_string(need) +
                                     " doubles of scratch, more than the " +
                                     std::to_string(kLzScratchDoubles) + " the library holds");
    // The product must only enqueue work: its tiles, run tables and panels
    // were built when the plan was chosen; anything missing would need an
    // allocation, so it is an error here.
    if (!part_prepared(h->main, vec_bytes(h->prec)))
      fail(SPMV_ERR_STATE, "the handle's plan is not prepared (spmv_set_plan or spmv_tune "
                           "prepares it)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard dg(h->device);
    double *part = lz_scratch(h->device);
    const int64_t n = h->n_rows;
    hip_ok(launch_lz_start(q, V1, n, part, s), "Lanczos kernels");
    hip_ok(launch_kpm_zero(V2, n, s), "zero fill");
    double *V = V1, *W = V2;  // V = v_j, W = -beta_{j-1} v_{j-1}
    for (int j = 0; j < m; ++j) {
      run_part(h, h->main, V, W, s);  // W = H v_j - beta_{j-1} v_{j-1}
      hip_ok(launch_lz_step(W, V, n, part, alpha + j, beta + j, s), "Lanczos kernels");
      std::swap(V, W);
    }
  });
}
