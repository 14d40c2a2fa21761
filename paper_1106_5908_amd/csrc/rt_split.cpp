// libspmv runtime, split unit: the local / nonlocal split of one process's
// share (Sect. 3.4; the bookkeeping is done once, Sect. 3.2) and the
// diagonal panels of a part, both built on the device.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include "runtime.h"

using namespace spmv;

namespace spmv {
namespace rt {

// Diagonal panels of a part without a row list: entries grouped by their
// offset d = col - row into K equal slices of the part's offset range, each
// slice a CRS over all rows (built on the device; synchronous).
std::vector<std::unique_ptr<Part>> &build_panels(spmv_handle_s *h, Part &p, int K) {
  auto found = p.panel_sets.find(K);
  if (found != p.panel_sets.end()) return found->second;
  if (K <= 1) fail(SPMV_ERR_INVALID_ARG, "panel count must exceed 1");
  if (p.row_ids.p) fail(SPMV_ERR_UNSUPPORTED, "diagonal panels need a part that covers all rows");
  hipStream_t s = nullptr;
  hip_ok(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
  struct StreamCloser {
    hipStream_t s;
    ~StreamCloser() { (void)hipStreamDestroy(s); }
  } closer{s};
  const int64_t n = p.n_rows, m = n + 1;
  DevBuf d2, counts, tmp;
  d2.alloc(16, "panel range");
  hip_ok(panel_d_range(p.row_ptr.as<int32_t>(), p.col.as<int32_t>(), n, d2.as<int64_t>(), &p.d_min,
                       &p.d_max, s),
         "panel range");
  const int64_t span = p.d_max - p.d_min + 1;
  counts.alloc(size_t(K) * size_t(m) * 4, "panel counts");
  tmp.alloc(size_t(scan_tmp_elems(m)) * 4, "scan scratch");
  hip_ok(panel_count(p.row_ptr.as<int32_t>(), p.col.as<int32_t>(), n, p.d_min, span, K,
                     counts.as<int32_t>(), tmp.as<int32_t>(), s),
         "panel count");
  const int vb = val_bytes(h->prec);
  PanelOut out{};
  std::vector<std::unique_ptr<Part>> ps;
  for (int k = 0; k < K; ++k) {
    std::unique_ptr<Part> q(new Part());
    q->n_rows = n;
    q->cut_row = p.cut_row;
    q->h_row_ptr.resize(size_t(m));
    hip_ok(hipMemcpyAsync(q->h_row_ptr.data(), counts.as<int32_t>() + int64_t(k) * m, size_t(m) * 4,
                          hipMemcpyDeviceToHost, s),
           "panel row_ptr readback");
    ps.push_back(std::move(q));
  }
  hip_ok(hipStreamSynchronize(s), "panels");
  for (int k = 0; k < K; ++k) {
    Part &q = *ps[size_t(k)];
    q.nnz = q.h_row_ptr[size_t(n)];
    upload(q.row_ptr, q.h_row_ptr.data(), size_t(m) * 4, "panel row_ptr");
    q.col.alloc(size_t(q.nnz) * 4, "panel col_idx");
    q.val.alloc(size_t(q.nnz) * vb, "panel val");
    q.stats = row_stats(q.h_row_ptr.data(), n);
    out.col[k] = q.col.as<int32_t>();
    out.val[k] = q.val.p;
  }
  hip_ok(panel_fill(h->prec, p.row_ptr.as<int32_t>(), p.col.as<int32_t>(), p.val.p, n, p.d_min,
                    span, K, counts.as<int32_t>(), out, s),
         "panel fill");
  hip_ok(hipStreamSynchronize(s), "panels");
  return p.panel_sets.emplace(K, std::move(ps)).first->second;
}

void prune_panels(Part &p, const std::vector<int> &keep) {
  for (auto it = p.panel_sets.begin(); it != p.panel_sets.end();) {
    if (std::find(keep.begin(), keep.end(), it->first) == keep.end())
      it = p.panel_sets.erase(it);
    else
      ++it;
  }
}

}  // namespace rt
}  // namespace spmv

using namespace spmv::rt;

// ==== a2: split bookkeeping =================================================================

extern "C" spmv_status_t spmv_split_local_nonlocal(spmv_handle_t a_, int64_t halo_begin_col,
                                                   spmv_handle_t *out_split) {
  return guarded([&] {
    if (!out_split) fail(SPMV_ERR_INVALID_ARG, "out_split is null");
    *out_split = nullptr;
    spmv_handle_s *a = live(a_);
    if (a->kind != SPMV_KIND_PLAIN)
      fail(SPMV_ERR_UNSUPPORTED, "only a plain handle can be split");
    if (halo_begin_col < 0 || halo_begin_col > a->n_cols)
      fail(SPMV_ERR_INVALID_ARG, "halo_begin_col " + std::to_string(halo_begin_col) +
                                     " outside [0, " + std::to_string(a->n_cols) + "]");
    DeviceGuard dg(a->device);
    std::unique_ptr<spmv_handle_s> h(new spmv_handle_s());
    h->device = a->device;
    h->prec = a->prec;
    h->flags = a->flags;
    h->kind = SPMV_KIND_SPLIT;
    h->n_rows = a->n_rows;
    h->n_cols = a->n_cols;
    h->nnz = a->nnz;
    h->halo_begin = halo_begin_col;
    const int64_t n = a->n_rows;
    hipStream_t s = nullptr;
    hip_ok(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
    struct StreamCloser {
      hipStream_t s;
      ~StreamCloser() { (void)hipStreamDestroy(s); }
    } closer{s};
    DevBuf work, tmp;
    work.alloc(size_t(split_work_elems(n)) * 4, "split work");
    tmp.alloc(size_t(scan_tmp_elems(n + 1)) * 4, "scan scratch");
    int64_t nnz_loc = 0, nnz_nl = 0, R = 0;
    hip_ok(split_count(a->main.row_ptr.as<int32_t>(), a->main.col.as<int32_t>(), n,
                       int32_t(halo_begin_col), work.as<int32_t>(), tmp.as<int32_t>(), &nnz_loc,
                       &nnz_nl, &R, s),
           "split count");
    Part &L = h->main;
    Part &N = h->nl;
    const int vb = val_bytes(h->prec);
    L.n_rows = n;
    L.nnz = nnz_loc;
    L.row_ptr.alloc(size_t(n + 1) * 4, "local row_ptr");
    L.col.alloc(size_t(nnz_loc) * 4, "local col_idx");
    L.val.alloc(size_t(nnz_loc) * vb, "local val");
    N.n_rows = R;
    N.nnz = nnz_nl;
    N.row_ids.alloc(size_t(R) * 4, "nonlocal rows");
    N.row_ptr.alloc(size_t(R + 1) * 4, "nonlocal row_ptr");
    N.col.alloc(size_t(nnz_nl) * 4, "nonlocal col_idx");
    N.val.alloc(size_t(nnz_nl) * vb, "nonlocal val");
    SplitOut o;
    o.loc_row_ptr = L.row_ptr.as<int32_t>();
    o.loc_col = L.col.as<int32_t>();
    o.loc_val = L.val.p;
    o.nl_rows = N.row_ids.as<int32_t>();
    o.nl_ptr = N.row_ptr.as<int32_t>();
    o.nl_col = N.col.as<int32_t>();
    o.nl_val = N.val.p;
    hip_ok(split_fill(h->prec, a->main.row_ptr.as<int32_t>(), a->main.col.as<int32_t>(),
                      a->main.val.p, n, int32_t(halo_begin_col), work.as<int32_t>(), nnz_nl, R, o,
                      s),
           "split fill");
    L.h_row_ptr.resize(size_t(n + 1));
    N.h_row_ptr.resize(size_t(R + 1));
    hip_ok(hipMemcpyAsync(L.h_row_ptr.data(), L.row_ptr.p, size_t(n + 1) * 4,
                          hipMemcpyDeviceToHost, s),
           "row_ptr readback");
    hip_ok(hipMemcpyAsync(N.h_row_ptr.data(), N.row_ptr.p, size_t(R + 1) * 4,
                          hipMemcpyDeviceToHost, s),
           "nl_ptr readback");
    hip_ok(hipStreamSynchronize(s), "split");
    L.stats = row_stats(L.h_row_ptr.data(), n);
    N.stats = row_stats(N.h_row_ptr.data(), R);
    // The local part is tiled in two halves, cut at the first row that has a
    // nonlocal entry, so that under SPMV_SCHEDULE_OVERLAP_NONLOCAL the rows
    // above it can run beside the nonlocal part.
    if (R > 0) {
      int32_t first = 0;
      hip_ok(hipMemcpy(&first, N.row_ids.p, 4, hipMemcpyDeviceToHost), "nonlocal rows readback");
      L.cut_row = first;
    }
    choose_plan(h.get(), L, "local");
    choose_plan(h.get(), N, "nonlocal");
    hip_ok(hipStreamCreateWithFlags(&h->copy_stream, hipStreamNonBlocking), "copy stream");
    hip_ok(hipEventCreateWithFlags(&h->ev_start, hipEventDisableTiming), "event");
    hip_ok(hipEventCreateWithFlags(&h->ev_copied, hipEventDisableTiming), "event");
    hip_ok(hipStreamCreateWithFlags(&h->send_stream, hipStreamNonBlocking), "send stream");
    hip_ok(hipEventCreateWithFlags(&h->ev_sent, hipEventDisableTiming), "event");
    hip_ok(hipStreamCreateWithFlags(&h->nl_stream, hipStreamNonBlocking), "nonlocal stream");
    hip_ok(hipEventCreateWithFlags(&h->ev_nl_done, hipEventDisableTiming), "event");
    register_handle(h.get());
    *out_split = h.release();
  });
}
