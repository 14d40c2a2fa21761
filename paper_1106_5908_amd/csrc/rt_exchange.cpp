// libspmv runtime, exchange unit: the send side of one process's exchange
// (Sect. 3.3: the elements another process needs gathered into one
// contiguous buffer; Sect. 3.5: in task mode the gather and the local part
// run while the communication proceeds), and the per-phase timing of split
// handles (the breakdown of Fig. 5).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.h"

using namespace spmv;

namespace spmv {
namespace rt {

namespace {

bool is_pinned_host(const void *p) {
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  const hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeHost;
}

}  // namespace

void mark(spmv_handle_s *h, int i, hipStream_t s) {
  if (h->timing) hip_ok(hipEventRecord(h->tev[i], s), "timing event");
}

void begin_timed_call(spmv_handle_s *h, hipStream_t s) {
  if (!h->timing) return;
  for (bool &r : h->tran) r = false;
  mark(h, T_START, s);
}

void require_pinned(const spmv_handle_s *h, const void *p, const char *what) {
  if (!(h->flags & SPMV_FLAG_ALLOW_PAGEABLE_HALO) && !is_pinned_host(p))
    fail(SPMV_ERR_INVALID_ARG,
         std::string(what) + " is not pinned host memory (a pageable copy cannot overlap); "
         "allocate it with hipHostMalloc or create the handle with SPMV_FLAG_ALLOW_PAGEABLE_HALO");
}

// ==== send side of the exchange (Sect. 3.3, 3.5) =======================================================

namespace {

void set_send_list(spmv_handle_s *h, const int32_t *idx, int64_t n) {
  // the previous list may still be read by a call in flight
  hip_ok(hipDeviceSynchronize(), "synchronize before replacing the send list");
  h->send_idx.release();
  h->send_buf.release();
  h->n_send = 0;
  if (n == 0) return;
  const size_t vb = size_t(vec_bytes(h->prec));
  upload(h->send_idx, idx, size_t(n) * 4, "send list");
  h->send_buf.alloc(size_t(n) * vb, "send buffer");
  h->n_send = n;
}

spmv_handle_s *split_handle(spmv_handle_t h_, const char *fn) {
  spmv_handle_s *h = live(h_);
  if (h->kind != SPMV_KIND_SPLIT) fail(SPMV_ERR_UNSUPPORTED, std::string(fn) + " needs a split handle");
  return h;
}

}  // namespace

}  // namespace rt
}  // namespace spmv

using namespace spmv::rt;

extern "C" spmv_status_t spmv_set_send_list(spmv_handle_t h_, const int32_t *send_idx,
                                            int64_t n_send) {
  return guarded([&] {
    spmv_handle_s *h = split_handle(h_, "spmv_set_send_list");
    if (n_send < 0) fail(SPMV_ERR_INVALID_ARG, "n_send is negative");
    if (n_send > 0 && !send_idx) fail(SPMV_ERR_INVALID_ARG, "send_idx is null");
    if (n_send > INT32_MAX) fail(SPMV_ERR_INVALID_ARG, "n_send exceeds 2^31 - 1");
    for (int64_t k = 0; k < n_send; ++k)
      if (send_idx[k] < 0 || int64_t(send_idx[k]) >= h->halo_begin)
        fail(SPMV_ERR_INVALID_ARG, "send_idx[" + std::to_string(k) + "] = " +
                                       std::to_string(send_idx[k]) + " outside [0, " +
                                       std::to_string(h->halo_begin) + ")");
    DeviceGuard dg(h->device);
    set_send_list(h, send_idx, n_send);
  });
}

extern "C" spmv_status_t spmv_send_list_symmetric(spmv_handle_t h_, int64_t *n_send) {
  return guarded([&] {
    spmv_handle_s *h = split_handle(h_, "spmv_send_list_symmetric");
    if (!n_send) fail(SPMV_ERR_INVALID_ARG, "n_send is null");
    DeviceGuard dg(h->device);
    // The nonlocal rows are ascending, so the rows below h are a prefix.
    std::vector<int32_t> rows(size_t(h->nl.n_rows));
    if (!rows.empty())
      hip_ok(hipMemcpy(rows.data(), h->nl.row_ids.p, rows.size() * 4, hipMemcpyDeviceToHost),
             "nonlocal rows readback");
    const int64_t m = std::lower_bound(rows.begin(), rows.end(), int64_t(h->halo_begin),
                                       [](int32_t r, int64_t v) { return int64_t(r) < v; }) -
                      rows.begin();
    set_send_list(h, rows.data(), m);
    *n_send = m;
  });
}

extern "C" spmv_status_t spmv_run_exchange(spmv_handle_t h_, const void *B, void *C,
                                           const void *B_halo_host, void *send_host,
                                           void *stream) {
  return guarded([&] {
    spmv_handle_s *h = split_handle(h_, "spmv_run_exchange");
    if ((!B && h->n_cols > 0) || (!C && h->n_rows > 0)) fail(SPMV_ERR_INVALID_ARG, "B or C is null");
    if (B && C && B == C) fail(SPMV_ERR_INVALID_ARG, "C must not alias B");
    const int64_t ns = h->n_send;
    if (ns > 0 && !send_host)
      fail(SPMV_ERR_INVALID_ARG, "send_host is null but the send list has " + std::to_string(ns) +
                                     " entries");
    if (ns > 0) require_pinned(h, send_host, "send_host");
    const int64_t n_halo = h->n_cols - h->halo_begin;
    const size_t vb = size_t(vec_bytes(h->prec));
    void *recv = static_cast<char *>(const_cast<void *>(B)) + size_t(h->halo_begin) * vb;
    const bool copy = B_halo_host && n_halo > 0;
    if (copy) require_pinned(h, B_halo_host, "B_halo_host");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard dg(h->device);
    begin_timed_call(h, s);
    h->tran[0] = copy;
    h->tran[1] = h->tran[2] = true;
    h->tran[3] = ns > 0;
    if (h->schedule == SPMV_SCHEDULE_SERIAL) {
      if (ns > 0) {
        mark(h, T_SEND, s);
        hip_ok(launch_pack(int(vb), B, h->send_idx.as<int32_t>(), ns, h->send_buf.p, s), "pack");
        hip_ok(hipMemcpyAsync(send_host, h->send_buf.p, size_t(ns) * vb, hipMemcpyDeviceToHost, s),
               "send copy");
        mark(h, T_SEND + 1, s);
      }
      if (copy) {
        mark(h, T_COPY, s);
        hip_ok(hipMemcpyAsync(recv, B_halo_host, size_t(n_halo) * vb, hipMemcpyHostToDevice, s),
               "halo copy");
        mark(h, T_COPY + 1, s);
      }
      split_compute(h, B, C, nullptr, SPMV_SCHEDULE_SERIAL, s);
      return;
    }
    hip_ok(hipEventRecord(h->ev_start, s), "event record");
    if (ns > 0) {
      hip_ok(hipStreamWaitEvent(h->send_stream, h->ev_start, 0), "stream wait");
      mark(h, T_SEND, h->send_stream);
      hip_ok(launch_pack(int(vb), B, h->send_idx.as<int32_t>(), ns, h->send_buf.p, h->send_stream),
             "pack");
      hip_ok(hipMemcpyAsync(send_host, h->send_buf.p, size_t(ns) * vb, hipMemcpyDeviceToHost,
                            h->send_stream),
             "send copy");
      mark(h, T_SEND + 1, h->send_stream);
      hip_ok(hipEventRecord(h->ev_sent, h->send_stream), "event record");
    }
    if (copy) {
      hip_ok(hipStreamWaitEvent(h->copy_stream, h->ev_start, 0), "stream wait");
      mark(h, T_COPY, h->copy_stream);
      hip_ok(hipMemcpyAsync(recv, B_halo_host, size_t(n_halo) * vb, hipMemcpyHostToDevice,
                            h->copy_stream),
             "halo copy");
      mark(h, T_COPY + 1, h->copy_stream);
      hip_ok(hipEventRecord(h->ev_copied, h->copy_stream), "event record");
    }
    split_compute(h, B, C, copy ? h->ev_copied : h->ev_start, h->schedule, s);
    if (ns > 0) hip_ok(hipStreamWaitEvent(s, h->ev_sent, 0), "stream wait");
  });
}

// ==== phase timing of split handles ====================================================================

extern "C" spmv_status_t spmv_set_phase_timing(spmv_handle_t h_, int32_t on) {
  return guarded([&] {
    spmv_handle_s *h = split_handle(h_, "spmv_set_phase_timing");
    DeviceGuard dg(h->device);
    if (on && !h->tev[0])
      for (hipEvent_t &e : h->tev) hip_ok(hipEventCreate(&e), "timing event");
    h->timing = on != 0;
    for (bool &r : h->tran) r = false;
  });
}

extern "C" spmv_status_t spmv_phase_times(spmv_handle_t h_, double *t) {
  return guarded([&] {
    spmv_handle_s *h = split_handle(h_, "spmv_phase_times");
    if (!t) fail(SPMV_ERR_INVALID_ARG, "t is null");
    if (!h->timing) fail(SPMV_ERR_STATE, "phase timing is off (spmv_set_phase_timing)");
    if (!h->tran[1]) fail(SPMV_ERR_STATE, "no call has run since phase timing was switched on");
    DeviceGuard dg(h->device);
    for (int i = 0; i < 8; ++i) t[i] = -1.0;
    for (int p = 0; p < 4; ++p) {
      if (!h->tran[p]) continue;
      for (int j = 0; j < 2; ++j) {
        hipEvent_t e = h->tev[1 + 2 * p + j];
        hip_ok(hipEventSynchronize(e), "timing event");
        float ms = 0.f;
        hip_ok(hipEventElapsedTime(&ms, h->tev[T_START], e), "timing event");
        t[2 * p + j] = double(ms);
      }
    }
  });
}
