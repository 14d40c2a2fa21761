// libspmv runtime, run unit: C = C + A*B (Listing 1) for plain, split
// (Sect. 3.4 / 3.5), symmetric-storage and batch handles, and the block of
// right-hand sides.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <string>

#include "runtime.h"

using namespace spmv;

namespace spmv {
namespace rt {

void run_sym(spmv_handle_s *h, const void *B, void *C, hipStream_t s) {
  const Part &p = h->main;
  if (p.n_rows == 0 || p.nnz == 0) return;
  hip_ok(launch_spmv_sym(p.dev(), p.plan.lanes, p.plan.nontemporal, p.plan.xcd_remap,
                         static_cast<const double *>(B), static_cast<double *>(C), s),
         "symmetric kernel launch");
}

int default_kt(int k) {
  if (k <= 4) return 4;
  if (k <= 8) return 8;
  return 16;
}

// The panels are shared with the single-vector plan.
void run_block_part(spmv_handle_s *h, Part &p, int kt, int nt, int remap, int panels, int k,
                    const void *B, int64_t ldb, void *C, int64_t ldc, hipStream_t s,
                    double scale, bool fused, int sorted_items) {
  if (p.n_rows == 0 || p.nnz == 0) return;
  if (sorted_items > 0) {
    // one pass over the layout per kt columns of B and C
    const SortedDev S = sorted_dev(h, p, sorted_items, kt);
    for (int j0 = 0; j0 < k; j0 += kt)
      hip_ok(launch_spmv_sorted_block(h->prec, S, sorted_items, kt, remap, B, ldb, j0,
                                      std::min(kt, k - j0), C, ldc, scale, s),
             "block kernel launch");
    return;
  }
  if (fused) {
    // 8 entries per lane are staged per panel: rows per workgroup sized so a
    // panel's entries in a block fit them
    const PanelSetDev S = panel_set_dev(h, p, panels);
    const int want = fused_rows_for(h, p, panels, kWG * 8);
    hip_ok(launch_spmv_block_fused(h->prec, S, want, nt, remap, kt, k, B, ldb, C, ldc, scale, s),
           "block kernel launch");
    return;
  }
  if (panels > 1) {
    for (auto &q : build_panels(h, p, panels))
      run_block_part(h, *q, kt, nt, remap, 1, k, B, ldb, C, ldc, s, scale);
    return;
  }
  auto t = p.tiles_for(4);
  hip_ok(launch_spmv_block(h->prec, p.dev(), t.first, t.second, 4, nt, remap, kt, k, B, ldb, C,
                           ldc, scale, s),
         "block kernel launch");
}

spmv_plan_t block_plan(spmv_handle_s *h, int k) {
  Part &p = h->main;
  auto it = h->block_plans.find(k);
  if (it != h->block_plans.end()) return it->second;
  spmv_plan_t c = p.plan;
  // a sorted-block plan serves blocks only with block_kt set; otherwise
  // blocks use the block kernel
  if (c.kernel == SPMV_KERNEL_SORTED_BLOCKS && c.block_kt == 0) {
    c.kernel = SPMV_KERNEL_STREAM;
    c.tile_items = 4;
  }
  if (p.plan.block_kt != 0) return c;  // set through spmv_set_plan
  c.block_kt = default_kt(k);
  // the cache file is read once per k and handle, not on every product
  if (!(h->flags & SPMV_FLAG_NO_TUNE_CACHE) && !h->block_cache_read[k]) {
    h->block_cache_read[k] = true;
    spmv_plan_t cached;
    if (cache_lookup(tune_key(h->device, h->prec, k, "block", p.n_rows, p.stats), &cached) &&
        cached.block_kt) {
      h->block_plans[k] = cached;
      return cached;
    }
  }
  return c;
}

void block_product(spmv_handle_s *h, int k, const void *B, int64_t ldb, void *C, int64_t ldc,
                   hipStream_t s, double scale) {
  const spmv_plan_t c = block_plan(h, k);
  run_block_part(h, h->main, c.block_kt, c.nontemporal, c.xcd_remap, c.panels, k, B, ldb, C, ldc,
                 s, scale, c.kernel == SPMV_KERNEL_FUSED_PANELS,
                 c.kernel == SPMV_KERNEL_SORTED_BLOCKS ? c.tile_items : 0);
}

void split_compute(spmv_handle_s *h, const void *B, void *C, hipEvent_t nl_after, int schedule,
                   hipStream_t s) {
  const SortedSet *T = nullptr;
  if (schedule == SPMV_SCHEDULE_OVERLAP_MERGED && h->main.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS &&
      h->main.n_rows > 0 && h->main.nnz > 0)
    T = merged_tail_for(h, h->main.plan.tile_items);
  if (T) {
    // The first blocks run from the local layout; the rest, from the merged
    // layout over their rows' local and nonlocal entries, once the halo is
    // in.  No separate nonlocal kernel runs.  When the first blocks are
    // whole rounds (one block per CU), the rest follow on s as one launch,
    // so that every round sweeps B as in the unsplit product; otherwise
    // they run on the nonlocal stream, on the CUs the first blocks leave
    // free.
    mark(h, T_LOCAL, s);
    SortedDev u = sorted_dev(h, h->main, h->main.plan.tile_items);
    u.b1 = T->b_first;
    hip_ok(launch_spmv_sorted(h->prec, u, h->main.plan.tile_items, h->main.plan.nontemporal,
                              h->main.plan.xcd_remap, B, C, s),
           "kernel launch");
    const bool ordered = T->after_rounds;
    hipStream_t t = ordered ? s : h->nl_stream;
    if (!ordered) hip_ok(hipStreamWaitEvent(t, h->ev_start, 0), "stream wait");
    if (nl_after && nl_after != h->ev_start)
      hip_ok(hipStreamWaitEvent(t, nl_after, 0), "stream wait");
    mark(h, T_NONLOCAL, t);
    SortedDev d;
    d.cs = T->cs.as<const int64_t>();
    d.col = T->col.as<const int32_t>();
    d.val = T->val.p;
    d.row = T->row.as<const uint16_t>();
    d.n_rows = h->main.n_rows;
    d.n_blocks = T->n_blocks;
    d.R = T->R;
    d.q = T->Q;
    d.b0 = T->b_first;
    d.b1 = T->n_blocks;
    hip_ok(launch_spmv_sorted(h->prec, d, h->main.plan.tile_items, h->main.plan.nontemporal,
                              h->main.plan.xcd_remap, B, C, t),
           "kernel launch");
    mark(h, T_NONLOCAL + 1, t);
    if (!ordered) {
      hip_ok(hipEventRecord(h->ev_nl_done, t), "event record");
      hip_ok(hipStreamWaitEvent(s, h->ev_nl_done, 0), "stream wait");
    }
    mark(h, T_LOCAL + 1, s);
    return;
  }
  const bool beside = schedule == SPMV_SCHEDULE_OVERLAP_NONLOCAL;
  if (beside && part_runs_halves(h->main) && h->nl.n_rows > 0 && h->nl.nnz > 0 &&
      h->main.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS) {
    // Sorted blocks run one workgroup per CU, in rounds.  The blocks above
    // the first nonlocal row start on s; on the nonlocal stream the
    // nonlocal part runs beside them as soon as the halo is in, and then
    // the blocks that hold nonlocal rows, which take the CUs the first
    // blocks leave free in their last round.
    mark(h, T_LOCAL, s);
    run_part_half(h, h->main, 0, B, C, s);
    hip_ok(hipStreamWaitEvent(h->nl_stream, h->ev_start, 0), "stream wait");
    if (nl_after && nl_after != h->ev_start)
      hip_ok(hipStreamWaitEvent(h->nl_stream, nl_after, 0), "stream wait");
    mark(h, T_NONLOCAL, h->nl_stream);
    run_part(h, h->nl, B, C, h->nl_stream);
    mark(h, T_NONLOCAL + 1, h->nl_stream);
    run_part_half(h, h->main, 1, B, C, h->nl_stream);
    hip_ok(hipEventRecord(h->ev_nl_done, h->nl_stream), "event record");
    hip_ok(hipStreamWaitEvent(s, h->ev_nl_done, 0), "stream wait");
    mark(h, T_LOCAL + 1, s);
    return;
  }
  if (beside && part_runs_halves(h->main) && h->nl.n_rows > 0 && h->nl.nnz > 0) {
    // rows above the first nonlocal row on s, the nonlocal part beside them
    // on its own stream once the halo is in, then the remaining local rows
    mark(h, T_LOCAL, s);
    run_part_half(h, h->main, 0, B, C, s);
    hip_ok(hipStreamWaitEvent(h->nl_stream, nl_after, 0), "stream wait");
    mark(h, T_NONLOCAL, h->nl_stream);
    run_part(h, h->nl, B, C, h->nl_stream);
    mark(h, T_NONLOCAL + 1, h->nl_stream);
    hip_ok(hipEventRecord(h->ev_nl_done, h->nl_stream), "event record");
    hip_ok(hipStreamWaitEvent(s, h->ev_nl_done, 0), "stream wait");
    run_part_half(h, h->main, 1, B, C, s);
    mark(h, T_LOCAL + 1, s);
    return;
  }
  mark(h, T_LOCAL, s);
  run_part(h, h->main, B, C, s);
  mark(h, T_LOCAL + 1, s);
  if (nl_after && nl_after != h->ev_start) hip_ok(hipStreamWaitEvent(s, nl_after, 0), "stream wait");
  mark(h, T_NONLOCAL, s);
  run_part(h, h->nl, B, C, s);
  mark(h, T_NONLOCAL + 1, s);
}

void split_run(spmv_handle_s *h, const void *B, void *C, const void *B_halo_host, hipStream_t s) {
  const int64_t n_halo = h->n_cols - h->halo_begin;
  const size_t vb = size_t(vec_bytes(h->prec));
  void *recv = static_cast<char *>(const_cast<void *>(B)) + size_t(h->halo_begin) * vb;
  const bool copy = B_halo_host && n_halo > 0;
  if (copy) require_pinned(h, B_halo_host, "B_halo_host");
  begin_timed_call(h, s);
  if (h->schedule == SPMV_SCHEDULE_SERIAL) {
    if (copy) {
      mark(h, T_COPY, s);
      hip_ok(hipMemcpyAsync(recv, B_halo_host, size_t(n_halo) * vb, hipMemcpyHostToDevice, s),
             "halo copy");
      mark(h, T_COPY + 1, s);
    }
    split_compute(h, B, C, nullptr, SPMV_SCHEDULE_SERIAL, s);
  } else {
    hip_ok(hipEventRecord(h->ev_start, s), "event record");
    hipEvent_t after = h->ev_start;
    if (copy) {
      hip_ok(hipStreamWaitEvent(h->copy_stream, h->ev_start, 0), "stream wait");
      mark(h, T_COPY, h->copy_stream);
      hip_ok(hipMemcpyAsync(recv, B_halo_host, size_t(n_halo) * vb, hipMemcpyHostToDevice,
                            h->copy_stream),
             "halo copy");
      mark(h, T_COPY + 1, h->copy_stream);
      hip_ok(hipEventRecord(h->ev_copied, h->copy_stream), "event record");
      after = h->ev_copied;
    }
    split_compute(h, B, C, after, h->schedule, s);
  }
  h->tran[0] = copy;
  h->tran[1] = h->tran[2] = true;
  h->tran[3] = false;
}

}  // namespace rt
}  // namespace spmv

using namespace spmv::rt;

// ==== a3-a7, a9: C = C + A*B ========================================================================

extern "C" spmv_status_t spmv_run(spmv_handle_t h_, const void *B, void *C,
                                  const void *B_halo_host, void *stream) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    if ((!B && h->n_cols > 0) || (!C && h->n_rows > 0)) fail(SPMV_ERR_INVALID_ARG, "B or C is null");
    if (B && C && B == C) fail(SPMV_ERR_INVALID_ARG, "C must not alias B");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard dg(h->device);
    if (h->kind != SPMV_KIND_SPLIT) {
      if (B_halo_host) fail(SPMV_ERR_INVALID_ARG, "B_halo_host is only accepted by split handles");
      if (h->kind == SPMV_KIND_PLAIN)
        run_part(h, h->main, B, C, s);
      else if (h->kind == SPMV_KIND_SYMMETRIC)
        run_sym(h, B, C, s);
      else
        batch_run(h, B, C, s);
      return;
    }
    // split handle: local part, halo arrival, nonlocal part (Sect. 3.4 / 3.5)
    split_run(h, B, C, B_halo_host, s);
  });
}

extern "C" spmv_status_t spmv_run_block(spmv_handle_t h_, int32_t k, const void *B, int64_t ldb,
                                        void *C, int64_t ldc, void *stream) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    if (h->kind != SPMV_KIND_PLAIN)
      fail(SPMV_ERR_UNSUPPORTED, "spmv_run_block serves plain handles only");
    if (k < 1 || k > 64) fail(SPMV_ERR_INVALID_ARG, "k must be in [1, 64]");
    if (ldb < k || ldc < k) fail(SPMV_ERR_INVALID_ARG, "ldb and ldc must be >= k");
    if ((!B && h->n_cols > 0) || (!C && h->n_rows > 0)) fail(SPMV_ERR_INVALID_ARG, "B or C is null");
    if (B && C && B == C) fail(SPMV_ERR_INVALID_ARG, "C must not alias B");
    DeviceGuard dg(h->device);
    block_product(h, k, B, ldb, C, ldc, static_cast<hipStream_t>(stream));
  });
}

extern "C" spmv_status_t spmv_get_block_plan(spmv_handle_t h_, int32_t k, spmv_plan_t *plan) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    if (h->kind != SPMV_KIND_PLAIN)
      fail(SPMV_ERR_UNSUPPORTED, "block products serve plain handles only");
    if (k < 1 || k > 64) fail(SPMV_ERR_INVALID_ARG, "k must be in [1, 64]");
    if (!plan) fail(SPMV_ERR_INVALID_ARG, "plan is null");
    *plan = block_plan(h, k);
  });
}
