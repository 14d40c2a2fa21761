// libspmv runtime, core unit: errors, device memory, the handle registry,
// ingest of CRS arrays (validation of the Sect. 1.2 invariants and the
// single-rounding encodings of the precision modes), creation of plain and
// symmetric-storage handles (Sect. 1.3.1), destroy, introspection and the
// measurement probes.  No exception crosses the C boundary.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "runtime.h"

using namespace spmv;

namespace spmv {
namespace rt {

namespace {
constexpr uint64_t kMagic = 0x53504d5648444c45ull;
constexpr uint64_t kDead = 0xdeaddeaddeaddeadull;
}  // namespace

thread_local std::string g_last_error;

[[noreturn]] void fail(spmv_status_t st, const std::string &msg) { throw Failure{st, msg}; }

void hip_ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return;
  (void)hipGetLastError();
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    fail(SPMV_ERR_ALLOC, std::string(what) + ": " + hipGetErrorString(e));
  fail(SPMV_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---- device memory -------------------------------------------------------------

namespace {

std::atomic<int64_t> g_alloc_count{0};

int64_t fault_alloc_after() {
  static const int64_t v = [] {
    const char *s = std::getenv("SPMV_FAULT_ALLOC_AFTER");
    return s ? std::atoll(s) : int64_t(-1);
  }();
  return v;
}

}  // namespace

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

void DevBuf::alloc(size_t n, const char *what, hipStream_t s) {
  release();
  const int64_t lim = fault_alloc_after();
  if (lim >= 0 && g_alloc_count.fetch_add(1) >= lim)
    fail(SPMV_ERR_ALLOC, std::string(what) + ": allocation failure injected (SPMV_FAULT_ALLOC_AFTER)");
  // Never zero bytes, so every array has a valid address; 64 bytes of tail
  // padding let grouped loads read past the last entry.
  const size_t want = std::max<size_t>(n + 64, 256);
  hip_ok(hipMalloc(&p, want), what);
  bytes = n;
  // padding reads as 0
  if (s)
    hip_ok(hipMemsetAsync(static_cast<char *>(p) + n, 0, want - n, s), what);
  else
    hip_ok(hipMemset(static_cast<char *>(p) + n, 0, want - n), what);
}

void upload(DevBuf &d, const void *src, size_t bytes, const char *what, hipStream_t s) {
  d.alloc(bytes, what, s);
  if (!bytes) return;
  if (s)
    hip_ok(hipMemcpyAsync(d.p, src, bytes, hipMemcpyHostToDevice, s), what);
  else
    hip_ok(hipMemcpy(d.p, src, bytes, hipMemcpyHostToDevice), what);
}

SetupStream::SetupStream() { hip_ok(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "setup stream"); }
SetupStream::~SetupStream() {
  if (!s) return;
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
}
void SetupStream::sync() { hip_ok(hipStreamSynchronize(s), "setup stream"); }

DeviceGuard::DeviceGuard(int d) : want(d) {
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != want) hip_ok(hipSetDevice(want), "hipSetDevice");
}
DeviceGuard::~DeviceGuard() {
  if (prev >= 0 && prev != want) (void)hipSetDevice(prev);
}

int current_device() {
  int d = 0;
  hip_ok(hipGetDevice(&d), "hipGetDevice");
  return d;
}

// ---- encodings (each a single rounding of the binary64 input, ties to even) -------

// binary64 -> bfloat16 by integer arithmetic on the bit pattern: keep the top
// 8 significant bits (fewer for results below 2^-126, where bfloat16 is
// subnormal with spacing 2^-133), round the dropped bits to nearest-even.
namespace {

uint16_t f64_to_bf16(double d) {
  uint64_t u;
  std::memcpy(&u, &d, 8);
  const uint16_t sign = static_cast<uint16_t>((u >> 48) & 0x8000u);
  const int exp = static_cast<int>((u >> 52) & 0x7ff);
  const uint64_t frac = u & ((uint64_t(1) << 52) - 1);
  if (exp == 0x7ff) return frac ? static_cast<uint16_t>(sign | 0x7fc0u) : static_cast<uint16_t>(sign | 0x7f80u);
  if (exp == 0) return sign;  // binary64 subnormals are far below 2^-134
  int e = exp - 1023;
  const uint64_t m = frac | (uint64_t(1) << 52);  // 53-bit significand
  if (e > 127) return static_cast<uint16_t>(sign | 0x7f80u);
  if (e >= -126) {
    uint64_t r = m >> 45;  // 8 bits including the implicit one
    const uint64_t rem = m & ((uint64_t(1) << 45) - 1);
    const uint64_t half = uint64_t(1) << 44;
    if (rem > half || (rem == half && (r & 1))) ++r;
    if (r == 256) {
      r = 128;
      ++e;
    }
    if (e > 127) return static_cast<uint16_t>(sign | 0x7f80u);
    return static_cast<uint16_t>(sign | ((e + 127) << 7) | (r & 0x7f));
  }
  // value = m * 2^(e-52); in units of 2^-133 that is m >> (-81 - e)
  const int shift = -81 - e;  // >= 46 here
  if (shift >= 64) return sign;
  uint64_t r = m >> shift;
  const uint64_t rem = m & ((uint64_t(1) << shift) - 1);
  const uint64_t half = uint64_t(1) << (shift - 1);
  if (rem > half || (rem == half && (r & 1))) ++r;
  return static_cast<uint16_t>(sign | r);  // r == 128 encodes 2^-126 exactly
}

}  // namespace

// ---- handle registry ---------------------------------------------------------------

namespace {
std::mutex g_live_mu;
std::vector<spmv_handle_s *> g_live;
}  // namespace

void register_handle(spmv_handle_s *h) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  g_live.push_back(h);
}
bool unregister_handle(spmv_handle_s *h) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  auto it = std::find(g_live.begin(), g_live.end(), h);
  if (it == g_live.end()) return false;
  g_live.erase(it);
  return true;
}
spmv_handle_s *live(spmv_handle_t h) {
  if (!h) fail(SPMV_ERR_INVALID_ARG, "null handle");
  std::lock_guard<std::mutex> lk(g_live_mu);
  if (std::find(g_live.begin(), g_live.end(), h) == g_live.end() || h->magic != kMagic)
    fail(SPMV_ERR_STATE, "handle is not live (destroyed or foreign)");
  return h;
}


// ==== a1: ingest ===========================================================================

void validate_crs(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *rp,
                  const int32_t *col, const double *val, int32_t base, const std::string &who) {
  if (n_rows < 0 || n_cols < 0 || nnz < 0)
    fail(SPMV_ERR_INVALID_ARG, who + "negative size");
  if (n_rows >= int64_t(INT32_MAX) || n_cols > int64_t(INT32_MAX) || nnz > int64_t(INT32_MAX))
    fail(SPMV_ERR_INVALID_ARG, who + "size exceeds the int32 index range");
  if (base != 0 && base != 1) fail(SPMV_ERR_INVALID_ARG, who + "index_base must be 0 or 1");
  if (!rp) fail(SPMV_ERR_INVALID_ARG, who + "row_ptr is null");
  if (nnz > 0 && (!col || !val)) fail(SPMV_ERR_INVALID_ARG, who + "col_idx or val is null");
  if (rp[0] != base)
    fail(SPMV_ERR_INVALID_MATRIX, who + "row_ptr[0] = " + std::to_string(rp[0]) +
                                      " but index_base = " + std::to_string(base));
  if (int64_t(rp[n_rows]) != nnz + base)
    fail(SPMV_ERR_INVALID_MATRIX, who + "row_ptr[" + std::to_string(n_rows) + "] = " +
                                      std::to_string(rp[n_rows]) + " but nnz + index_base = " +
                                      std::to_string(nnz + base));
  for (int64_t i = 0; i < n_rows; ++i)
    if (rp[i + 1] < rp[i])
      fail(SPMV_ERR_INVALID_MATRIX, who + "row_ptr decreases at index " + std::to_string(i + 1));
  std::atomic<int64_t> first_bad{INT64_MAX};
  const int64_t lo = base, hi = n_cols + base;
  parallel_for(nnz, [&](int64_t b, int64_t e) {
    for (int64_t j = b; j < e; ++j)
      if (col[j] < lo || col[j] >= hi) {
        int64_t cur = first_bad.load();
        while (j < cur && !first_bad.compare_exchange_weak(cur, j)) {
        }
        return;
      }
  });
  if (first_bad.load() != INT64_MAX) {
    const int64_t j = first_bad.load();
    fail(SPMV_ERR_INVALID_MATRIX, who + "col_idx[" + std::to_string(j) + "] = " +
                                      std::to_string(col[j]) + " outside [" + std::to_string(lo) +
                                      ", " + std::to_string(hi) + ")");
  }
}

// The mode arrives as a plain int (an enum parameter would make an unknown
// value undefined behaviour before it could be checked).
int check_prec(int32_t p) {
  if (p != SPMV_PREC_F64 && p != SPMV_PREC_F32 && p != SPMV_PREC_BF16_F32ACC &&
      p != SPMV_PREC_F32_F64ACC)
    fail(SPMV_ERR_INVALID_ARG, "unknown precision mode");
  return int(p);
}

void encode(int64_t n_rows, int64_t nnz, const int32_t *rp, const int32_t *col, const double *val,
            int32_t base, int prec, Encoded &out) {
  out.rp.resize(size_t(n_rows + 1));
  for (int64_t i = 0; i <= n_rows; ++i) out.rp[size_t(i)] = rp[i] - base;
  if (base) {
    out.col.resize(size_t(nnz));
    int32_t *dst = out.col.data();
    parallel_for(nnz, [&](int64_t b, int64_t e) {
      for (int64_t j = b; j < e; ++j) dst[j] = col[j] - base;
    });
    out.col_ptr = out.col.data();
  } else {
    out.col_ptr = col;
  }
  switch (prec) {
    case P_F64:
      out.val_ptr = val;
      break;
    case P_F32:
    case P_F32_F64: {
      out.val.resize(size_t(nnz) * 4);
      float *dst = reinterpret_cast<float *>(out.val.data());
      parallel_for(nnz, [&](int64_t b, int64_t e) {
        for (int64_t j = b; j < e; ++j) dst[j] = static_cast<float>(val[j]);
      });
      out.val_ptr = out.val.data();
      break;
    }
    default: {
      out.val.resize(size_t(nnz) * 2);
      uint16_t *dst = reinterpret_cast<uint16_t *>(out.val.data());
      parallel_for(nnz, [&](int64_t b, int64_t e) {
        for (int64_t j = b; j < e; ++j) dst[j] = f64_to_bf16(val[j]);
      });
      out.val_ptr = out.val.data();
      break;
    }
  }
}

namespace {

// Plain or symmetric handle from host CRS arrays (validated by the caller).
spmv_handle_s *create_handle(int kind, int64_t n_rows, int64_t n_cols, int64_t nnz,
                             const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                             int32_t index_base, int p, uint32_t flags) {
  Encoded enc;
  encode(n_rows, nnz, row_ptr, col_idx, val, index_base, p, enc);
  std::unique_ptr<spmv_handle_s> h(new spmv_handle_s());
  h->device = current_device();
  h->prec = p;
  h->flags = flags;
  h->kind = kind;
  h->n_rows = n_rows;
  h->n_cols = n_cols;
  h->nnz = nnz;
  h->halo_begin = n_cols;
  Part &m = h->main;
  m.n_rows = n_rows;
  m.nnz = nnz;
  {
    // the three uploads are ordered on a stream of their own, synchronised
    // before the host arrays (the caller's, or the encoded copies) go away
    SetupStream up;
    upload(m.row_ptr, enc.rp.data(), enc.rp.size() * 4, "row_ptr", up.s);
    upload(m.col, enc.col_ptr, size_t(nnz) * 4, "col_idx", up.s);
    upload(m.val, enc.val_ptr, size_t(nnz) * val_bytes(p), "val", up.s);
    up.sync();
  }
  m.h_row_ptr = std::move(enc.rp);
  m.stats = row_stats(m.h_row_ptr.data(), n_rows);
  choose_plan(h.get(), m, kind == SPMV_KIND_SYMMETRIC ? "symmetric" : "main");
  register_handle(h.get());
  return h.release();
}

}  // namespace

}  // namespace rt
}  // namespace spmv

using namespace spmv::rt;

extern "C" spmv_status_t spmv_create_crs(int64_t n_rows, int64_t n_cols, int64_t nnz,
                                         const int32_t *row_ptr, const int32_t *col_idx,
                                         const double *val, int32_t index_base,
                                         int32_t prec, uint32_t flags,
                                         spmv_handle_t *out) {
  return guarded([&] {
    if (!out) fail(SPMV_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    const int p = check_prec(prec);
    validate_crs(n_rows, n_cols, nnz, row_ptr, col_idx, val, index_base, "");
    *out = create_handle(SPMV_KIND_PLAIN, n_rows, n_cols, nnz, row_ptr, col_idx, val, index_base,
                         p, flags);
  });
}

// ==== symmetric storage (Sect. 1.3.1) ==========================================================

extern "C" spmv_status_t spmv_create_sym_crs(int64_t n, int64_t nnz, const int32_t *row_ptr,
                                             const int32_t *col_idx, const double *val,
                                             int32_t index_base, int32_t prec, uint32_t flags,
                                             spmv_handle_t *out) {
  return guarded([&] {
    if (!out) fail(SPMV_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    const int p = check_prec(prec);
    if (p != P_F64) fail(SPMV_ERR_UNSUPPORTED, "symmetric storage is served in SPMV_PREC_F64 only");
    validate_crs(n, n, nnz, row_ptr, col_idx, val, index_base, "");
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = int64_t(row_ptr[i]) - index_base; j < int64_t(row_ptr[i + 1]) - index_base;
           ++j)
        if (int64_t(col_idx[j]) - index_base < i)
          fail(SPMV_ERR_INVALID_MATRIX, "col_idx[" + std::to_string(j) + "] = " +
                                            std::to_string(col_idx[j]) +
                                            " lies left of the diagonal of row " +
                                            std::to_string(i + index_base) +
                                            " (symmetric storage keeps the upper triangle)");
    *out = create_handle(SPMV_KIND_SYMMETRIC, n, n, nnz, row_ptr, col_idx, val, index_base, p,
                         flags);
  });
}

// ---- handle ------------------------------------------------------------------------------

spmv_handle_s::spmv_handle_s() : magic(spmv::rt::kMagic) {}

spmv_handle_s::~spmv_handle_s() {
  if (copy_stream) (void)hipStreamSynchronize(copy_stream);
  if (send_stream) (void)hipStreamSynchronize(send_stream);
  if (nl_stream) (void)hipStreamSynchronize(nl_stream);
  if (ev_nl_done) (void)hipEventDestroy(ev_nl_done);
  if (nl_stream) (void)hipStreamDestroy(nl_stream);
  if (ev_sent) (void)hipEventDestroy(ev_sent);
  for (hipEvent_t &e : tev)
    if (e) (void)hipEventDestroy(e);
  if (send_stream) (void)hipStreamDestroy(send_stream);
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);
  if (ev_start) (void)hipEventDestroy(ev_start);
  if (ev_copied) (void)hipEventDestroy(ev_copied);
  if (copy_stream) (void)hipStreamDestroy(copy_stream);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

// ==== destroy / errors ==================================================================================

extern "C" spmv_status_t spmv_destroy(spmv_handle_t h) {
  if (!h) {
    g_last_error.clear();
    return SPMV_OK;
  }
  return guarded([&] {
    if (!unregister_handle(h)) fail(SPMV_ERR_STATE, "handle is not live (destroyed or foreign)");
    DeviceGuard dg(h->device);
    h->magic = spmv::rt::kDead;
    delete h;
  });
}

extern "C" const char *spmv_last_error(void) { return g_last_error.c_str(); }

// ==== introspection ========================================================================================

extern "C" spmv_status_t spmv_get_info(spmv_handle_t h_, spmv_info_t *info) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    if (!info) fail(SPMV_ERR_INVALID_ARG, "info is null");
    std::memset(info, 0, sizeof(*info));
    info->kind = h->kind;
    info->precision = h->prec;
    info->n_rows = h->n_rows;
    info->n_cols = h->n_cols;
    info->nnz = h->nnz;
    info->halo_begin = h->halo_begin;
    info->nnz_local = h->main.nnz;
    info->nnz_nonlocal = h->kind == SPMV_KIND_SPLIT ? h->nl.nnz : 0;
    info->n_nonlocal_rows = h->kind == SPMV_KIND_SPLIT ? h->nl.n_rows : 0;
    info->batch_count = h->kind == SPMV_KIND_BATCH ? h->count : 1;
    if (h->kind == SPMV_KIND_BATCH) {
      DeviceGuard dg(h->device);
      batch_prepare(h);
      info->n_tiles = h->b_ntiles;
    } else if (h->main.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS) {
      auto it = h->main.sorted.find(std::make_pair(h->main.plan.tile_items, 1));
      info->n_tiles = it == h->main.sorted.end() ? 0 : it->second.n_chunks;
    } else {
      auto it = h->main.tiles.find(h->main.plan.tile_items);
      info->n_tiles = it == h->main.tiles.end() ? 0 : it->second.second;
    }
    info->row_len_mean = h->main.stats.mean;
    info->row_len_cv = h->main.stats.cv;
    info->row_len_max = h->main.stats.max;
    info->n_send = h->n_send;
    if (h->kind == SPMV_KIND_BATCH && h->main.plan.kernel == SPMV_KERNEL_STAGED)
      info->n_staged_tiles = h->b_staged;
    if (h->kind != SPMV_KIND_BATCH && h->main.plan.kernel == SPMV_KERNEL_STAGED) {
      const int items = h->main.plan.tile_items;
      auto count = [items](const Part &q) {
        auto r = q.runs.find(items);
        return r == q.runs.end() ? int64_t(0) : r->second.second;
      };
      if (h->main.plan.panels > 1) {
        auto ps = h->main.panel_sets.find(h->main.plan.panels);
        if (ps != h->main.panel_sets.end())
          for (auto &q : ps->second) info->n_staged_tiles += count(*q);
      } else {
        info->n_staged_tiles = count(h->main);
      }
    }
  });
}

extern "C" spmv_status_t spmv_export(spmv_handle_t h_, int32_t which, void *dst, int64_t bytes,
                                     int64_t *size_bytes) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    const int vb = val_bytes(h->prec);
    const DevBuf *src = nullptr;
    int64_t n = 0;
    const bool split = h->kind == SPMV_KIND_SPLIT;
    switch (which) {
      case SPMV_ARR_ROW_PTR: src = &h->main.row_ptr; n = int64_t(h->main.h_row_ptr.size()) * 4; break;
      case SPMV_ARR_COL: src = &h->main.col; n = h->main.nnz * 4; break;
      case SPMV_ARR_VAL: src = &h->main.val; n = h->main.nnz * vb; break;
      case SPMV_ARR_NL_ROWS: if (split) { src = &h->nl.row_ids; n = h->nl.n_rows * 4; } break;
      case SPMV_ARR_NL_PTR: if (split) { src = &h->nl.row_ptr; n = (h->nl.n_rows + 1) * 4; } break;
      case SPMV_ARR_NL_COL: if (split) { src = &h->nl.col; n = h->nl.nnz * 4; } break;
      case SPMV_ARR_NL_VAL: if (split) { src = &h->nl.val; n = h->nl.nnz * vb; } break;
      case SPMV_ARR_SEND_IDX: if (split) { src = &h->send_idx; n = h->n_send * 4; } break;
      case SPMV_ARR_TILES:
      case SPMV_ARR_RUNS: {
        if (h->kind == SPMV_KIND_BATCH) break;
        const int items = h->main.plan.tile_items;
        auto t = h->main.tiles.find(items);
        if (t == h->main.tiles.end()) break;
        const int64_t nt = t->second.second;
        if (which == SPMV_ARR_TILES) {
          src = &t->second.first;
          n = (nt + 1) * int64_t(sizeof(TileRP));
        } else {
          auto r = h->main.runs.find(items);
          if (r == h->main.runs.end()) break;
          src = &r->second.first;
          n = nt * RUN_WORDS * 4;
        }
        break;
      }
      default: break;
    }
    if (!src) fail(SPMV_ERR_INVALID_ARG, "no such array in this handle");
    if (size_bytes) *size_bytes = n;
    if (!dst) return;
    if (bytes < n) fail(SPMV_ERR_INVALID_ARG, "dst too small: need " + std::to_string(n) + " bytes");
    DeviceGuard dg(h->device);
    if (n) hip_ok(hipMemcpy(dst, src->p, size_t(n), hipMemcpyDeviceToHost), "export");
  });
}

extern "C" spmv_status_t spmv_set_schedule(spmv_handle_t h_, int32_t schedule) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    const bool ok_split = h->kind == SPMV_KIND_SPLIT &&
                          (schedule == SPMV_SCHEDULE_OVERLAP || schedule == SPMV_SCHEDULE_SERIAL ||
                           schedule == SPMV_SCHEDULE_OVERLAP_NONLOCAL ||
                           schedule == SPMV_SCHEDULE_OVERLAP_MERGED);
    const bool ok_batch = h->kind == SPMV_KIND_BATCH &&
                          (schedule == SPMV_SCHEDULE_BATCH_GRAPH ||
                           schedule == SPMV_SCHEDULE_BATCH_DIRECT ||
                           schedule == SPMV_SCHEDULE_BATCH_FLAT);
    if (!ok_split && !ok_batch) fail(SPMV_ERR_INVALID_ARG, "schedule not valid for this handle");
    if (schedule == SPMV_SCHEDULE_OVERLAP_MERGED &&
        h->main.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS && h->main.n_rows > 0 &&
        h->main.nnz > 0) {
      // built here, so that the products only enqueue work
      DeviceGuard dg(h->device);
      (void)merged_tail_for(h, h->main.plan.tile_items);
    }
    h->schedule = schedule;
    h->schedule_set = true;
  });
}

// ==== probes ================================================================================================

extern "C" spmv_status_t spmv_probe_copy(double *dst, const double *src, int64_t n, void *stream) {
  return guarded([&] {
    if (n < 0 || ((!dst || !src) && n > 0)) fail(SPMV_ERR_INVALID_ARG, "bad copy arguments");
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
      fail(SPMV_ERR_INVALID_ARG, "copy buffers must be 16-byte aligned");
    hip_ok(launch_copy(dst, src, n, static_cast<hipStream_t>(stream)), "copy launch");
  });
}

extern "C" spmv_status_t spmv_probe_triad(double *a, const double *b, const double *c, double s,
                                          int64_t n, void *stream) {
  return guarded([&] {
    if (n < 0 || ((!a || !b || !c) && n > 0)) fail(SPMV_ERR_INVALID_ARG, "bad triad arguments");
    if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
         reinterpret_cast<uintptr_t>(c)) % 16)
      fail(SPMV_ERR_INVALID_ARG, "triad buffers must be 16-byte aligned");
    hip_ok(launch_triad(a, b, c, s, n, static_cast<hipStream_t>(stream)), "triad launch");
  });
}

extern "C" spmv_status_t spmv_probe_read(const double *src, int64_t n, double *sums,
                                         int64_t sums_len, void *stream) {
  return guarded([&] {
    if (n < 0 || ((!src || !sums) && n > 1)) fail(SPMV_ERR_INVALID_ARG, "bad read arguments");
    if (sums_len < read_sums_needed(n))
      fail(SPMV_ERR_INVALID_ARG, "sums must hold " + std::to_string(read_sums_needed(n)) + " values");
    if (reinterpret_cast<uintptr_t>(src) % 16)
      fail(SPMV_ERR_INVALID_ARG, "read buffer must be 16-byte aligned");
    hip_ok(launch_read(src, n, sums, static_cast<hipStream_t>(stream)), "read launch");
  });
}

extern "C" spmv_status_t spmv_probe_gather(const double *src, int64_t n_rows, int32_t width,
                                           const int32_t *idx, int64_t n, int32_t xcd_remap,
                                           double *sums, int64_t sums_len, void *stream) {
  return guarded([&] {
    if (width != 1 && width != 2 && width != 4 && width != 8 && width != 16)
      fail(SPMV_ERR_INVALID_ARG, "width must be 1, 2, 4, 8 or 16");
    if (n < 0 || n_rows < 1 || n_rows > INT32_MAX) fail(SPMV_ERR_INVALID_ARG, "bad gather sizes");
    if (!src || !sums || (n > 0 && !idx)) fail(SPMV_ERR_INVALID_ARG, "null gather buffer");
    if (xcd_remap != 0 && xcd_remap != 1) fail(SPMV_ERR_INVALID_ARG, "xcd_remap must be 0 or 1");
    if (sums_len < gather_sums_needed(n, width))
      fail(SPMV_ERR_INVALID_ARG,
           "sums must hold " + std::to_string(gather_sums_needed(n, width)) + " values");
    if (width > 1 && reinterpret_cast<uintptr_t>(src) % 16)
      fail(SPMV_ERR_INVALID_ARG, "src must be 16-byte aligned for width > 1");
    hip_ok(launch_gather(src, n_rows, idx, n, width, xcd_remap, sums,
                         static_cast<hipStream_t>(stream)),
           "gather launch");
  });
}

extern "C" int64_t spmv_probe_gather_sums_needed(int64_t n, int32_t width) {
  if (n < 0 || (width != 1 && width != 2 && width != 4 && width != 8 && width != 16)) return -1;
  return gather_sums_needed(n, width);
}

extern "C" spmv_status_t spmv_probe_spin(int64_t nanoseconds, void *stream) {
  return guarded([&] {
    if (nanoseconds < 0 || nanoseconds > int64_t(10) * 1000 * 1000 * 1000)
      fail(SPMV_ERR_INVALID_ARG, "spin time must be in [0, 10 s]");
    hip_ok(launch_spin(nanoseconds, static_cast<hipStream_t>(stream)), "spin launch");
  });
}

extern "C" spmv_status_t spmv_probe_atomic(double *C, int64_t n, int32_t scattered, int32_t iters,
                                           void *stream) {
  return guarded([&] {
    if (!C) fail(SPMV_ERR_INVALID_ARG, "C is null");
    if (n < 64 || n > (int64_t(1) << 31) || (n & (n - 1)) != 0)
      fail(SPMV_ERR_INVALID_ARG, "n must be a power of two in [64, 2^31]");
    if (scattered != 0 && scattered != 1) fail(SPMV_ERR_INVALID_ARG, "scattered must be 0 or 1");
    if (iters < 1 || iters > 4096) fail(SPMV_ERR_INVALID_ARG, "iters must be in [1, 4096]");
    hip_ok(launch_atomic(C, n, scattered, iters, static_cast<hipStream_t>(stream)), "atomic launch");
  });
}
