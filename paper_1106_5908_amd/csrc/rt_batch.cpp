// libspmv runtime, batch unit: many independent products C_m = C_m + A_m B_m
// in one launch -- the members pooled in one allocation, their tiles in
// per-XCD queues or one grid, the launch captured in a HIP graph and
// replayed.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "runtime.h"

using namespace spmv;
using namespace spmv::rt;

// ==== a9: batch setup ========================================================================

extern "C" spmv_status_t spmv_create_batch(int32_t count, const int64_t *n_rows,
                                           const int64_t *n_cols, const int64_t *nnz,
                                           const int32_t *const *row_ptr,
                                           const int32_t *const *col_idx,
                                           const double *const *val, int32_t index_base,
                                           int32_t prec, uint32_t flags,
                                           spmv_handle_t *out) {
  return guarded([&] {
    if (!out) fail(SPMV_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (count < 1) fail(SPMV_ERR_INVALID_ARG, "count must be >= 1");
    if (!n_rows || !n_cols || !nnz || !row_ptr || !col_idx || !val)
      fail(SPMV_ERR_INVALID_ARG, "null member array");
    const int p = check_prec(prec);
    int64_t tot_rp = 0, tot_nz = 0, tot_x = 0, tot_y = 0;
    for (int32_t m = 0; m < count; ++m) {
      validate_crs(n_rows[m], n_cols[m], nnz[m], row_ptr[m], col_idx[m], val[m], index_base,
                   "member " + std::to_string(m) + ": ");
      tot_rp += n_rows[m] + 1;
      tot_nz += nnz[m];
      tot_x += n_cols[m];
      tot_y += n_rows[m];
    }
    if (tot_nz > int64_t(INT32_MAX) * 4)
      fail(SPMV_ERR_INVALID_ARG, "batch too large");
    std::unique_ptr<spmv_handle_s> h(new spmv_handle_s());
    h->device = current_device();
    h->prec = p;
    h->flags = flags;
    h->kind = SPMV_KIND_BATCH;
    h->count = count;
    h->n_rows = tot_y;
    h->n_cols = tot_x;
    h->nnz = tot_nz;
    h->halo_begin = tot_x;
    const int vb = val_bytes(p);
    std::vector<int32_t> rp_all(static_cast<size_t>(tot_rp));
    std::vector<int32_t> col_all(static_cast<size_t>(tot_nz));
    std::vector<uint8_t> val_all(static_cast<size_t>(tot_nz) * vb);
    h->h_desc.resize(size_t(count));
    int64_t orp = 0, onz = 0, ox = 0, oy = 0;
    double sum = 0, sq = 0;
    int64_t mx = 0;
    for (int32_t m = 0; m < count; ++m) {
      Encoded enc;
      encode(n_rows[m], nnz[m], row_ptr[m], col_idx[m], val[m], index_base, p, enc);
      std::memcpy(rp_all.data() + orp, enc.rp.data(), enc.rp.size() * 4);
      std::memcpy(col_all.data() + onz, enc.col_ptr, size_t(nnz[m]) * 4);
      std::memcpy(val_all.data() + size_t(onz) * vb, enc.val_ptr, size_t(nnz[m]) * vb);
      h->h_desc[size_t(m)] = BatchDesc{orp, onz, ox, oy};
      for (int64_t i = 0; i < n_rows[m]; ++i) {
        const int64_t l = int64_t(enc.rp[size_t(i + 1)]) - enc.rp[size_t(i)];
        sum += double(l);
        sq += double(l) * double(l);
        mx = std::max(mx, l);
      }
      h->m_rows.push_back(n_rows[m]);
      h->m_cols.push_back(n_cols[m]);
      orp += n_rows[m] + 1;
      onz += nnz[m];
      ox += n_cols[m];
      oy += n_rows[m];
    }
    Part &M = h->main;
    M.n_rows = tot_y;
    M.nnz = tot_nz;
    if (tot_y > 0) {
      M.stats.mean = sum / double(tot_y);
      M.stats.cv = M.stats.mean > 0
                       ? std::sqrt(std::max(0.0, sq / double(tot_y) - M.stats.mean * M.stats.mean)) /
                             M.stats.mean
                       : 0.0;
      M.stats.max = mx;
    }
    M.h_row_ptr = std::move(rp_all);  // pooled, member-local values
    {
      SetupStream up;
      upload(M.row_ptr, M.h_row_ptr.data(), M.h_row_ptr.size() * 4, "batch row_ptr", up.s);
      upload(M.col, col_all.data(), col_all.size() * 4, "batch col_idx", up.s);
      upload(M.val, val_all.data(), val_all.size(), "batch val", up.s);
      h->b_counter.alloc(NXCD_QUEUES * QUEUE_STRIDE * sizeof(int32_t), "batch queue counters", up.s);
      up.sync();
    }
    choose_plan(h.get(), M, "batch");
    hip_ok(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking), "capture stream");
    register_handle(h.get());
    *out = h.release();
  });
}

namespace spmv {
namespace rt {

namespace {
void batch_runs(spmv_handle_s *h);
}  // namespace

// Tile queue of a batch for the current tile size.
void batch_prepare(spmv_handle_s *h) {
  const int items = h->main.plan.tile_items;
  if (h->b_tiles_items == items && h->b_tiles.p) {
    if (h->main.plan.kernel == SPMV_KERNEL_STAGED && h->b_runs_items != items) batch_runs(h);
    return;
  }
  std::vector<BatchTile> tl;
  for (int32_t m = 0; m < h->count; ++m) {
    const BatchDesc &d = h->h_desc[size_t(m)];
    std::vector<int32_t> t =
        make_tiles(h->main.h_row_ptr.data() + d.rp_off, h->m_rows[size_t(m)], int64_t(kWG) * items);
    const int32_t *mrp = h->main.h_row_ptr.data() + d.rp_off;
    for (size_t i = 0; i + 1 < t.size(); ++i)
      tl.push_back(BatchTile{m, t[i], t[i + 1], mrp[t[i]], mrp[t[i + 1]], 0, d.rp_off, d.nz_off,
                             d.x_off, d.y_off});
  }
  if (int64_t(tl.size()) >= int64_t(INT32_MAX) - (int64_t(1) << 20))
    fail(SPMV_ERR_UNSUPPORTED, "too many tiles");
  upload(h->b_tiles, tl.data(), tl.size() * sizeof(BatchTile), "batch tiles");
  h->b_ntiles = int64_t(tl.size());
  h->b_tiles_items = items;
  h->b_grid = batch_persistent_grid(h->prec, items, h->device);
  h->h_btiles = std::move(tl);
  if (h->main.plan.kernel == SPMV_KERNEL_STAGED) batch_runs(h);
}

namespace {

// Run table of the batch tiles for the staged kernel, from a copy of the
// pooled (member-local) col_idx read back once.
void batch_runs(spmv_handle_s *h) {
  const int items = h->b_tiles_items;
  const Part &M = h->main;
  std::vector<int32_t> hc(static_cast<size_t>(M.nnz));
  if (M.nnz > 0)
    hip_ok(hipMemcpy(hc.data(), M.col.p, size_t(M.nnz) * 4, hipMemcpyDeviceToHost), "col readback");
  const int64_t nt = int64_t(h->h_btiles.size());
  std::vector<int32_t> table(size_t(nt) * RUN_WORDS, 0);
  const int64_t budget = RUN_STAGE_BYTES / vec_bytes(h->prec);
  parallel_for(
      nt,
      [&](int64_t b, int64_t e) {
        std::vector<int32_t> cs;
        for (int64_t t = b; t < e; ++t) {
          const BatchTile &T = h->h_btiles[size_t(t)];
          run_row(hc.data() + T.nz_off + T.p0, int64_t(T.p1) - T.p0, int64_t(kWG) * items - 4,
                  budget, cs, table.data() + size_t(t) * RUN_WORDS);
        }
      },
      64);
  int64_t staged = 0;
  for (size_t i = 0; i < table.size(); i += RUN_WORDS) staged += table[i] > 0 ? 1 : 0;
  upload(h->b_runs, table.data(), table.size() * 4, "batch run table");
  h->b_runs_items = items;
  h->b_staged = staged;
}

}  // namespace

hipError_t batch_launch_direct(spmv_handle_s *h, const void *B, void *C, hipStream_t s) {
  if (h->main.plan.kernel == SPMV_KERNEL_STAGED)
    return launch_batch_staged(h->prec, h->main.row_ptr.as<int32_t>(), h->main.col.as<int32_t>(),
                               h->main.val.p, h->b_tiles.as<BatchTile>(),
                               h->b_runs.as<int32_t>(), h->b_ntiles, h->b_tiles_items,
                               h->main.plan.nontemporal, B, C, s);
  if (h->main.plan.kernel == SPMV_KERNEL_TILE_GRID)
    return launch_batch_flat(h->prec, h->main.row_ptr.as<int32_t>(), h->main.col.as<int32_t>(),
                             h->main.val.p, h->b_tiles.as<BatchTile>(),
                             h->b_ntiles, h->b_tiles_items, h->main.plan.nontemporal, B, C, s);
  hipError_t e = launch_batch_reset(h->b_counter.as<int32_t>(), s);
  if (e != hipSuccess) return e;
  return launch_batch_persistent(h->prec, h->main.row_ptr.as<int32_t>(), h->main.col.as<int32_t>(),
                                 h->main.val.p, h->b_tiles.as<BatchTile>(), h->b_ntiles, h->b_tiles_items,
                                 h->main.plan.nontemporal, h->b_counter.as<int32_t>(), h->b_grid,
                                 B, C, s);
}

void batch_run(spmv_handle_s *h, const void *B, void *C, hipStream_t s) {
  batch_prepare(h);
  if (h->b_ntiles == 0) return;
  if (h->schedule == SPMV_SCHEDULE_BATCH_DIRECT) {
    hip_ok(batch_launch_direct(h, B, C, s), "batch launch");
    return;
  }
  if (h->schedule == SPMV_SCHEDULE_BATCH_FLAT) {
    hip_ok(launch_batch_flat(h->prec, h->main.row_ptr.as<int32_t>(), h->main.col.as<int32_t>(),
                             h->main.val.p, h->b_tiles.as<BatchTile>(),
                             h->b_ntiles, h->b_tiles_items, h->main.plan.nontemporal, B, C, s),
           "batch flat launch");
    return;
  }
  // Graph: the counter reset and the persistent launch are captured once per
  // (B, C, plan) and replayed.
  if (!h->gexec || h->g_B != B || h->g_C != C || h->g_items != h->b_tiles_items ||
      h->g_nt != h->main.plan.nontemporal || h->g_kernel != h->main.plan.kernel) {
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
    hip_ok(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    const hipError_t le = batch_launch_direct(h, B, C, h->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(h->cap_stream, &g);
    hip_ok(le, "batch launch (capture)");
    hip_ok(ce, "end capture");
    h->graph = g;
    hip_ok(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0), "graph instantiate");
    h->g_B = B;
    h->g_C = C;
    h->g_items = h->b_tiles_items;
    h->g_nt = h->main.plan.nontemporal;
    h->g_kernel = h->main.plan.kernel;
  }
  hip_ok(hipGraphLaunch(h->gexec, s), "graph launch");
}

}  // namespace rt
}  // namespace spmv
