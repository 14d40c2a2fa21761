// Internal declarations of the host runtime behind include/spmv.h, shared by
// its units:
//   rt_core.cpp      errors, device memory, handle registry, ingest (Sect. 1.2
//                    validation and encodings), destroy, introspection, probes
//   rt_plan.cpp      tiles, run tables, kernel plans, the autotuner and its cache
//   rt_split.cpp     the local / nonlocal split (Sect. 3.4) and diagonal panels
//   rt_batch.cpp     batch handles and their graph-replayed launch
//   rt_run.cpp       spmv_run (plain, split, symmetric, batch) and block products
//   rt_exchange.cpp  send side of the exchange and phase timing (Sect. 3.3 / 3.5)
//   rt_solvers.hip   the Chebyshev-moment and Lanczos loops
// Not part of the public interface.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <string>
#include <system_error>
#include <thread>
#include <utility>
#include <vector>

#include "spmv.h"
#include "spmv_internal.h"

namespace spmv {
namespace rt {

constexpr int kWG = 256;

// ---- errors ---------------------------------------------------------------------------

// Description of the last failure on this thread (spmv_last_error).
extern thread_local std::string g_last_error;

struct Failure {
  spmv_status_t status;
  std::string msg;
};

[[noreturn]] void fail(spmv_status_t st, const std::string &msg);
// Throws SPMV_ERR_ALLOC (out of memory) or SPMV_ERR_HIP for e != hipSuccess.
void hip_ok(hipError_t e, const char *what);

// Runs f(), turning every exception into a status and g_last_error, so no
// exception crosses the C boundary.
template <class F>
spmv_status_t guarded(F &&f) {
  try {
    f();
    g_last_error.clear();
    return SPMV_OK;
  } catch (const Failure &e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return SPMV_ERR_ALLOC;
  } catch (const std::exception &e) {
    g_last_error = std::string("internal error: ") + e.what();
    return SPMV_ERR_HIP;
  } catch (...) {
    g_last_error = "internal error";
    return SPMV_ERR_HIP;
  }
}

// ---- device memory ------------------------------------------------------------------------

// One device allocation owned by a handle.  Every array gets at least 256
// bytes and 64 zeroed bytes of tail padding (grouped loads may read past the
// last entry).  alloc / upload enqueue the zeroing and the copy on `s`; the
// caller synchronises `s` before the host source may go away.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release();
  void alloc(size_t n, const char *what, hipStream_t s = nullptr);
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// d = a new allocation holding `bytes` bytes copied from host `src`, both
// enqueued on `s` (see DevBuf).
void upload(DevBuf &d, const void *src, size_t bytes, const char *what, hipStream_t s = nullptr);

// A non-blocking stream for one setup call's uploads, synchronised (and
// destroyed) when the call leaves scope, so setup orders its copies on a
// stream of its own instead of the null stream.
struct SetupStream {
  hipStream_t s = nullptr;
  SetupStream();
  ~SetupStream();
  void sync();
  SetupStream(const SetupStream &) = delete;
  SetupStream &operator=(const SetupStream &) = delete;
};

struct DeviceGuard {
  int prev = -1;
  int want;
  explicit DeviceGuard(int d);
  ~DeviceGuard();
};

int current_device();

// ---- host parallel loops -------------------------------------------------------------------

// f(b, e) over chunks of [0, n) on up to 16 threads; one thread below
// `serial_below` items.
template <class F>
void parallel_for(int64_t n, F &&f, int64_t serial_below = int64_t(1) << 18) {
  unsigned T = std::thread::hardware_concurrency();
  T = T < 1u ? 1u : (T > 16u ? 16u : T);
  if (n < serial_below || T == 1) {
    f(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(T);
  const int64_t chunk = (n + T - 1) / T;
  for (unsigned t = 0; t < T; ++t) {
    const int64_t b = int64_t(t) * chunk, e = n < b + chunk ? n : b + chunk;
    if (b >= e) continue;
    try {
      th.emplace_back([&f, b, e] { f(b, e); });
    } catch (const std::system_error &) {
      f(b, e);  // no thread to be had: this chunk runs here, the started ones are joined below
    }
  }
  for (auto &x : th) x.join();
}

// ---- row statistics, tiles, run tables, plans (rt_plan.cpp) -------------------------------

struct RowStats {
  double mean = 0, cv = 0;
  int64_t max = 0;
};
RowStats row_stats(const int32_t *rp, int64_t n);

// Greedy tiles of consecutive rows holding at most `tile_items` - 4 entries
// and at most 512 rows; a longer row gets a tile of its own.  Returns the
// first row of every tile plus n.
std::vector<int32_t> make_tiles(const int32_t *rp, int64_t n, int64_t tile_items);

// One row of the staged kernel's run table (layout in spmv_internal.h) for
// the n columns of one tile; q (RUN_WORDS int32) zeroed by the caller.
void run_row(const int32_t *cols, int64_t n, int64_t max_entries, int64_t budget,
             std::vector<int32_t> &cs, int32_t *q);
std::vector<int32_t> make_runs(const int32_t *rp, const int32_t *col,
                               const std::vector<int32_t> &tiles, int64_t max_entries,
                               int64_t budget);

spmv_plan_t default_plan();
void check_plan(const spmv_plan_t &p);
PlanDev to_dev(const spmv_plan_t &p);
const char *prec_name(int p);

// ---- one CRS part on the device ------------------------------------------------------------

// Sorted-block layout of a part for one chunk size (see SortedDev).
struct SortedSet {
  DevBuf cs, col, val, row;
  int64_t n_blocks = 0, n_chunks = 0;
  int R = 0;           // rows per block
  int Q = 0;           // slots per chunk
  int64_t period = 0;  // the sweeps start at multiples of it
  int64_t b_first = 0; // blocks before it hold no chunk (a layout of the last blocks only)
  bool after_rounds = false;  // merged layout: b_first ends whole rounds of one block per CU
};

struct Part {
  int64_t n_rows = 0, nnz = 0;
  DevBuf row_ptr, col, val, row_ids;
  std::vector<int32_t> h_row_ptr;  // host copy (0-based), for tiling
  RowStats stats;
  spmv_plan_t plan = default_plan();
  // diagonal panels of this part, one set per panel count K > 1
  std::map<int, std::vector<std::unique_ptr<Part>>> panel_sets;
  int64_t d_min = 0, d_max = 0;
  std::map<int, std::pair<DevBuf, int64_t>> tiles;  // tile_items -> (tile starts, count)
  std::map<int, std::pair<DevBuf, int64_t>> runs;   // tile_items -> (run table, staged tiles)
  // (tile_items, kt) -> sorted-block layout; kt 1 for one right-hand side,
  // else the columns of B per pass of the block kernel
  std::map<std::pair<int, int>, SortedSet> sorted;
  // (panel count, entry capacity) -> rows per workgroup of the fused-panel kernels
  std::map<std::pair<int, int>, int> fused_rows;
  // Rows [0, cut_row) and [cut_row, n_rows) are tiled separately, so each
  // half can be launched on its own (the local part of a split handle, cut at
  // its first row with a nonlocal entry); -1: no cut.
  int64_t cut_row = -1;
  std::map<int, int64_t> cut_tile;  // tile_items -> first tile of the second half

  CsrDev dev() const {
    CsrDev d;
    d.row_ptr = row_ptr.as<const int32_t>();
    d.col = col.as<const int32_t>();
    d.val = val.p;
    d.row_ids = row_ids.p ? row_ids.as<const int32_t>() : nullptr;
    d.n_rows = n_rows;
    return d;
  }
  // Tile starts for `items` entries per lane (built and uploaded on first use).
  std::pair<const TileRP *, int64_t> tiles_for(int items);
  // The tiles of the part's own rows as make_tiles cuts them, honouring cut_row.
  std::vector<int32_t> host_tiles(int items) const;
  // Run table of the staged kernel for tiles of `items` (built on first use
  // from a copy of col_idx read back from the device; synchronous).
  const int32_t *runs_for(int items, int x_bytes);
};

}  // namespace rt
}  // namespace spmv

// ---- handle ---------------------------------------------------------------------------------

struct spmv_handle_s {
  uint64_t magic = 0;
  int kind = SPMV_KIND_PLAIN;
  int device = 0;
  int prec = spmv::P_F64;
  uint32_t flags = 0;
  int64_t n_rows = 0, n_cols = 0, nnz = 0;
  spmv::rt::Part main;  // plain: the matrix; split: local part
  spmv::rt::Part nl;    // split: nonlocal part
  int64_t halo_begin = 0;
  int schedule = SPMV_SCHEDULE_OVERLAP;
  bool schedule_set = false;  // set by spmv_set_schedule: spmv_tune then keeps it
  hipStream_t copy_stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_copied = nullptr;
  // split: timing events of the last call's phases (see spmv_set_phase_timing)
  bool timing = false;
  hipEvent_t tev[9] = {};
  bool tran[4] = {};  // phases that ran in the last timed call
  // split: send side of the exchange
  spmv::rt::DevBuf send_idx, send_buf;
  int64_t n_send = 0;
  hipStream_t send_stream = nullptr;
  hipEvent_t ev_sent = nullptr;
  // split: the nonlocal part's own stream (it runs beside the local part's
  // rows that have no nonlocal entry) and its completion event
  hipStream_t nl_stream = nullptr;
  hipEvent_t ev_nl_done = nullptr;
  // split, SPMV_SCHEDULE_OVERLAP_MERGED: chunk multiplier -> layout of the
  // local part's last blocks over local and nonlocal entries (see
  // merged_tail_for); a refused layout is kept as one with no blocks
  std::map<int, spmv::rt::SortedSet> merged;
  // batch
  int32_t count = 0;
  std::vector<int64_t> m_rows, m_cols;
  spmv::rt::DevBuf b_tiles, b_counter;
  int64_t b_ntiles = 0;
  int b_tiles_items = 0;
  int b_grid = 0;
  spmv::rt::DevBuf b_runs;  // run table of the batch tiles (staged kernel)
  int b_runs_items = 0;
  int64_t b_staged = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void *g_B = nullptr;
  void *g_C = nullptr;
  int g_items = -1, g_nt = -1, g_kernel = -1;
  std::vector<spmv::BatchTile> h_btiles;
  std::vector<spmv::BatchDesc> h_desc;
  std::map<int, spmv_plan_t> block_plans;  // k -> plan chosen by spmv_tune (or cached)
  std::map<int, bool> block_cache_read;     // k -> the cache was consulted for this k
  spmv::rt::DevBuf kpm_part;                // per-workgroup partial dot products

  spmv_handle_s();
  ~spmv_handle_s();
};

namespace spmv {
namespace rt {

// ---- ingest (rt_core.cpp) --------------------------------------------------------------------

// Sect. 1.2 invariants of one CRS matrix; `who` prefixes the messages.
void validate_crs(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *rp,
                  const int32_t *col, const double *val, int32_t base, const std::string &who);
// The precision mode, which arrives as a plain int (an enum parameter would
// make an unknown value undefined behaviour before it could be checked).
int check_prec(int32_t p);

// Host arrays shifted to 0-based, values encoded to the storage precision.
struct Encoded {
  std::vector<int32_t> rp;
  std::vector<int32_t> col;  // empty when no shift is needed (use caller's)
  std::vector<uint8_t> val;  // empty for f64 without shift (use caller's)
  const int32_t *col_ptr = nullptr;
  const void *val_ptr = nullptr;
};
void encode(int64_t n_rows, int64_t nnz, const int32_t *rp, const int32_t *col, const double *val,
            int32_t base, int prec, Encoded &out);

// ---- handle registry (rt_core.cpp) ------------------------------------------------------

void register_handle(spmv_handle_s *h);
bool unregister_handle(spmv_handle_s *h);
// h itself if it is a live handle; else throws SPMV_ERR_INVALID_ARG (null) or
// SPMV_ERR_STATE (destroyed or foreign).
spmv_handle_s *live(spmv_handle_t h);

// ---- autotuner cache and plans (rt_plan.cpp) ---------------------------------------------

std::string tune_key(int dev, int prec, int k, const char *part, int64_t n_rows,
                     const RowStats &s);
bool cache_lookup(const std::string &key, spmv_plan_t *p);
void cache_store(const std::string &key, const spmv_plan_t &p);

// The part's plan from the cache (else the default); builds its panels,
// tiles and run tables.
void choose_plan(spmv_handle_s *h, Part &p, const char *part_name);
// Tiles (and, for the staged kernel, run tables) of the part's plan and of
// its panels, so that running the part only enqueues work.
void prepare_part(spmv_handle_s *h, Part &p);
// True if running the part with its plan needs no allocation: its panels,
// tiles and run tables are already built.
bool part_prepared(const Part &p, int x_bytes);
// C = C + A*B over one part with its plan, on s.
void run_part(spmv_handle_s *h, Part &p, const void *B, void *C, hipStream_t s);
// Whether the part's plan can run the two halves of a cut part separately
// (tile-based kernels: stream and staged, with or without panels).
bool part_runs_halves(const Part &p);
// C = C + A*B over rows [0, cut_row) (half 0) or [cut_row, n_rows) (half 1)
// of a cut part whose plan part_runs_halves allows.
void run_part_half(spmv_handle_s *h, Part &p, int half, const void *B, void *C, hipStream_t s);
// The part's K diagonal panels (the part itself for K = 1) as the fused-panel
// kernels take them; builds the panels on first use.
PanelSetDev panel_set_dev(spmv_handle_s *h, Part &p, int K);
// Rows per workgroup of the fused-panel kernels: the largest R in
// {512, 256, ..., 16} such that no panel holds more than `cap` entries in any
// block of R rows (16 if none does); cached per (K, cap).  Needs the panels.
int fused_rows_for(spmv_handle_s *h, Part &p, int K, int cap);

// ---- split and panels (rt_split.cpp) -------------------------------------------------------

std::vector<std::unique_ptr<Part>> &build_panels(spmv_handle_s *h, Part &p, int K);
// Drops panel sets no chosen plan uses (each is a full copy of the part).
void prune_panels(Part &p, const std::vector<int> &keep);

// ---- sorted-block layout (rt_sorted.cpp) ------------------------------------------------------

// The layout of the part for chunks of SB_WG * items slots, built on first
// use (synchronous: col_idx and val are read back once).
// For block products (kt = 4, 8 or 16 columns per pass) the chunks hold
// (SB_WG / kt) * items slots and the blocks at most sorted_block_rows / kt
// rows.
const SortedSet &sorted_for(spmv_handle_s *h, Part &p, int items, int kt = 1);
SortedDev sorted_dev(spmv_handle_s *h, Part &p, int items, int kt = 1);
// Frees every layout but those listed as (items, kt).
void prune_sorted(Part &p, const std::vector<std::pair<int, int>> &keep);
// Split handle with a sorted-block local plan: the layout of the local
// part's last blocks over their rows' local and nonlocal entries together
// (same block size and sweep period as the local layout).  It starts at the
// last round boundary (a multiple of the CU count, one block per CU) at or
// above the block that holds the first nonlocal row (after_rounds), or at
// that block if fewer than one round precedes it.  Built on first use; null
// if the layout is refused (rows too long) or the handle has no nonlocal
// rows.
const SortedSet *merged_tail_for(spmv_handle_s *h, int items);
// Frees the merged layouts of every other chunk size (all with keep 0).
void prune_merged(spmv_handle_s *h, int keep_items);

// ---- batch (rt_batch.cpp) --------------------------------------------------------------------

void batch_prepare(spmv_handle_s *h);
hipError_t batch_launch_direct(spmv_handle_s *h, const void *B, void *C, hipStream_t s);
void batch_run(spmv_handle_s *h, const void *B, void *C, hipStream_t s);

// ---- products (rt_run.cpp) -----------------------------------------------------------------

void run_sym(spmv_handle_s *h, const void *B, void *C, hipStream_t s);
int default_kt(int k);
// Block product C = C + scale*A*B over a part, or over its diagonal panels
// in turn when `panels` > 1.  `scale` is 1 or a power of two (exact).
// sorted_items > 0: the sorted-block kernel for blocks, with that many
// slots per lane and load step (kt columns per pass; panels ignored).
void run_block_part(spmv_handle_s *h, Part &p, int kt, int nt, int remap, int panels, int k,
                    const void *B, int64_t ldb, void *C, int64_t ldc, hipStream_t s,
                    double scale = 1.0, bool fused = false, int sorted_items = 0);
// The plan block products with k columns use on this handle: chosen by
// spmv_tune, else read from the cache, else the defaults.
spmv_plan_t block_plan(spmv_handle_s *h, int k);
// C = C + scale*A*B for k columns of a plain handle (arguments checked).
void block_product(spmv_handle_s *h, int k, const void *B, int64_t ldb, void *C, int64_t ldc,
                   hipStream_t s, double scale = 1.0);

// ---- exchange and phase timing (rt_exchange.cpp) ------------------------------------------

// Phase events of split handles: tev[0] the call's start; then start and
// end of the halo copy (1, 2), the local part (3, 4), the nonlocal part
// (5, 6) and the send side (7, 8).
enum { T_START = 0, T_COPY = 1, T_LOCAL = 3, T_NONLOCAL = 5, T_SEND = 7 };
void mark(spmv_handle_s *h, int i, hipStream_t s);
void begin_timed_call(spmv_handle_s *h, hipStream_t s);
// Host memory of a copy that must overlap: pinned, unless the handle allows
// pageable memory (a pageable copy is staged by the runtime and does not
// proceed beside the kernels; nonblocking is not asynchronous, Sect. 3.1).
void require_pinned(const spmv_handle_s *h, const void *p, const char *what);
// The local and nonlocal parts of a split handle on stream s.  Under
// SPMV_SCHEDULE_OVERLAP_NONLOCAL with a local plan that can run its halves
// (part_runs_halves), the local rows above the first nonlocal row run on s
// while the nonlocal part runs on the handle's nonlocal stream after
// `nl_after` (the halo copy's event, or the call's start event), and the
// remaining local rows follow once the nonlocal part is done.  Under
// SPMV_SCHEDULE_OVERLAP_MERGED with a sorted-block local plan, the blocks
// above the first nonlocal row run on s and the blocks from there on run
// over their local and nonlocal entries together on the nonlocal stream
// after `nl_after`, with no separate nonlocal kernel.  Otherwise the local
// part, then (after `nl_after` unless it is null or the start event) the
// nonlocal part, in order on s.  Either way every row gets its local and
// nonlocal sums.
void split_compute(spmv_handle_s *h, const void *B, void *C, hipEvent_t nl_after, int schedule,
                   hipStream_t s);
// One product of a split handle under its schedule: the halo copy from
// B_halo_host (pinned; null: the halo is resident) and split_compute.
void split_run(spmv_handle_s *h, const void *B, void *C, const void *B_halo_host, hipStream_t s);

}  // namespace rt
}  // namespace spmv
