// libspmv runtime: the C interface of include/spmv.h.
//
// Host side of the CRS product of Schubert, Fehske, Hager, Wellein (2011):
// validation and encoding of the CRS arrays (Sect. 1.2), tiling, run tables
// of the staged kernel and kernel plans, the split handle and its overlap
// schedule (Sect. 3.4 / 3.5) with the send side of the exchange, batch
// handles with their launch captured in a HIP graph, symmetric-storage
// handles (Sect. 1.3.1), the Chebyshev-moment and Lanczos loops, and the
// autotuner with its persistent cache.  No exception crosses the C boundary.
#include <hip/hip_runtime_api.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "spmv.h"
#include "spmv_internal.h"

using namespace spmv;

namespace {

constexpr uint64_t kMagic = 0x53504d5648444c45ull;
constexpr uint64_t kDead = 0xdeaddeaddeaddeadull;
constexpr int kWG = 256;

thread_local std::string g_last_error;

struct Failure {
  spmv_status_t status;
  std::string msg;
};

[[noreturn]] void fail(spmv_status_t st, const std::string &msg) { throw Failure{st, msg}; }

void hip_ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return;
  (void)hipGetLastError();
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    fail(SPMV_ERR_ALLOC, std::string(what) + ": " + hipGetErrorString(e));
  fail(SPMV_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---- device memory -------------------------------------------------------------

std::atomic<int64_t> g_alloc_count{0};

int64_t fault_alloc_after() {
  static const int64_t v = [] {
    const char *s = std::getenv("SPMV_FAULT_ALLOC_AFTER");
    return s ? std::atoll(s) : int64_t(-1);
  }();
  return v;
}

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
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
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n, const char *what) {
    release();
    const int64_t lim = fault_alloc_after();
    if (lim >= 0 && g_alloc_count.fetch_add(1) >= lim)
      fail(SPMV_ERR_ALLOC, std::string(what) + ": allocation failure injected (SPMV_FAULT_ALLOC_AFTER)");
    // Never zero bytes, so every array has a valid address; 64 bytes of tail
    // padding let paired loads read one entry past the end.
    const size_t want = std::max<size_t>(n + 64, 256);
    hip_ok(hipMalloc(&p, want), what);
    bytes = n;
    hip_ok(hipMemset(static_cast<char *>(p) + n, 0, want - n), what);  // padding reads as 0
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

void upload(DevBuf &d, const void *src, size_t bytes, const char *what) {
  d.alloc(bytes, what);
  if (bytes) hip_ok(hipMemcpy(d.p, src, bytes, hipMemcpyHostToDevice), what);
}

struct DeviceGuard {
  int prev = -1;
  int want;
  explicit DeviceGuard(int d) : want(d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != want) hip_ok(hipSetDevice(want), "hipSetDevice");
  }
  ~DeviceGuard() {
    if (prev >= 0 && prev != want) (void)hipSetDevice(prev);
  }
};

// ---- host parallel loops -------------------------------------------------------

// f(b, e) over chunks of [0, n) on up to 16 threads; one thread below
// `serial_below` items.
template <class F>
void parallel_for(int64_t n, F &&f, int64_t serial_below = int64_t(1) << 18) {
  unsigned T = std::thread::hardware_concurrency();
  T = std::max(1u, std::min(T, 16u));
  if (n < serial_below || T == 1) {
    f(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(T);
  const int64_t chunk = (n + T - 1) / T;
  for (unsigned t = 0; t < T; ++t) {
    const int64_t b = int64_t(t) * chunk, e = std::min(n, b + chunk);
    if (b >= e) continue;
    try {
      th.emplace_back([&f, b, e] { f(b, e); });
    } catch (const std::system_error &) {
      f(b, e);  // no thread to be had: this chunk runs here, the started ones are joined below
    }
  }
  for (auto &x : th) x.join();
}

// ---- encodings (each a single rounding of the binary64 input, ties to even) -------

// binary64 -> bfloat16 by integer arithmetic on the bit pattern: keep the top
// 8 significant bits (fewer for results below 2^-126, where bfloat16 is
// subnormal with spacing 2^-133), round the dropped bits to nearest-even.
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

// ---- row statistics and tiles ----------------------------------------------------

struct RowStats {
  double mean = 0, cv = 0;
  int64_t max = 0;
};

RowStats row_stats(const int32_t *rp, int64_t n) {
  RowStats s;
  if (n <= 0) return s;
  double sum = 0, sq = 0;
  int64_t mx = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t l = int64_t(rp[i + 1]) - rp[i];
    sum += double(l);
    sq += double(l) * double(l);
    mx = std::max(mx, l);
  }
  s.mean = sum / double(n);
  const double var = std::max(0.0, sq / double(n) - s.mean * s.mean);
  s.cv = s.mean > 0 ? std::sqrt(var) / s.mean : 0.0;
  s.max = mx;
  return s;
}

// Greedy tiles of consecutive rows holding at most `tile` - 4 entries (room
// for the kernel's grouped loads to start up to three entries early) and at
// most 512 rows (two per lane of the workgroup, whose bounds the kernel
// prefetches); a row longer than that gets a tile of its own.
std::vector<int32_t> make_tiles(const int32_t *rp, int64_t n, int64_t tile_items) {
  constexpr int64_t kMaxRows = 2 * kWG;
  const int64_t tile = tile_items - 4;
  std::vector<int32_t> t;
  t.reserve(size_t(n / std::max<int64_t>(1, std::min(tile / 16, kMaxRows)) + 2));
  t.push_back(0);
  int64_t r = 0;
  while (r < n) {
    const int64_t start = rp[r];
    int64_t e = r + 1;
    if (int64_t(rp[e]) - start <= tile)
      while (e < n && int64_t(rp[e + 1]) - start <= tile && e - r < kMaxRows) ++e;
    t.push_back(int32_t(e));
    r = e;
  }
  return t;
}

// Run table of the staged kernel (layout in spmv_internal.h): each tile's
// distinct columns, ascending, merged into runs across gaps of at most
// kRunGap columns (the gap columns are loaded too).  A tile gets nr = 0, and
// is run as in the stream kernel, when it has no entries, more than
// `max_entries` (a single long row), more than RUN_MAX runs or more than
// `budget` columns to stage.
constexpr int64_t kRunGap = 16;

// One row of the run table for the n columns of one tile (q: RUN_WORDS
// int32, zeroed by the caller); `cs` is scratch.
void run_row(const int32_t *cols, int64_t n, int64_t max_entries, int64_t budget,
             std::vector<int32_t> &cs, int32_t *q) {
  if (n < 1 || n > max_entries) return;
  cs.assign(cols, cols + n);
  std::sort(cs.begin(), cs.end());
  int64_t start[RUN_MAX], end[RUN_MAX];  // [start, end)
  int nr = 0;
  for (const int32_t c : cs) {
    if (nr > 0 && c < end[nr - 1]) continue;  // repeated column
    if (nr > 0 && c - end[nr - 1] <= kRunGap) {
      end[nr - 1] = int64_t(c) + 1;
      continue;
    }
    if (nr == RUN_MAX) return;  // more runs than the kernel takes
    start[nr] = c;
    end[nr] = int64_t(c) + 1;
    ++nr;
  }
  int64_t L = 0;
  for (int r = 0; r < nr; ++r) L += end[r] - start[r];
  if (L > budget) return;
  q[0] = nr;
  q[1] = int32_t(L);
  int64_t o = 0;
  for (int r = 0; r < nr; ++r) {
    q[2 + r] = int32_t(start[r]);
    q[6 + r] = int32_t(o - start[r]);
    o += end[r] - start[r];
  }
}

std::vector<int32_t> make_runs(const int32_t *rp, const int32_t *col,
                               const std::vector<int32_t> &tiles, int64_t max_entries,
                               int64_t budget) {
  const int64_t n_tiles = int64_t(tiles.size()) - 1;
  std::vector<int32_t> out(size_t(std::max<int64_t>(n_tiles, 0)) * RUN_WORDS, 0);
  parallel_for(
      n_tiles,
      [&](int64_t b, int64_t e) {
        std::vector<int32_t> cs;
        for (int64_t t = b; t < e; ++t) {
          const int64_t p0 = rp[tiles[size_t(t)]], p1 = rp[tiles[size_t(t + 1)]];
          run_row(col + p0, p1 - p0, max_entries, budget, cs, out.data() + size_t(t) * RUN_WORDS);
        }
      },
      64);
  return out;
}

// ---- plans -------------------------------------------------------------------------

spmv_plan_t default_plan() {
  spmv_plan_t p;
  p.kernel = SPMV_KERNEL_STREAM;
  p.tile_items = 8;
  p.lanes = 32;
  p.nontemporal = 1;
  p.xcd_remap = 1;
  p.block_kt = 0;
  p.tiles_per_group = 1;
  p.panels = 1;
  return p;
}

void check_plan(const spmv_plan_t &p) {
  if (p.kernel != SPMV_KERNEL_STREAM && p.kernel != SPMV_KERNEL_VECTOR &&
      p.kernel != SPMV_KERNEL_TILE_GRID && p.kernel != SPMV_KERNEL_STAGED)
    fail(SPMV_ERR_INVALID_ARG,
         "plan.kernel must be SPMV_KERNEL_STREAM, _VECTOR, _TILE_GRID or _STAGED");
  if (p.tile_items != 4 && p.tile_items != 8 && p.tile_items != 16)
    fail(SPMV_ERR_INVALID_ARG, "plan.tile_items must be 4, 8 or 16");
  if (p.kernel == SPMV_KERNEL_STAGED && p.tile_items == 4)
    fail(SPMV_ERR_INVALID_ARG, "the staged kernel takes tile_items 8 or 16");
  if (p.lanes < 2 || p.lanes > 64 || (p.lanes & (p.lanes - 1)))
    fail(SPMV_ERR_INVALID_ARG, "plan.lanes must be a power of two in [2, 64]");
  if (p.block_kt != 0 && p.block_kt != 4 && p.block_kt != 8 && p.block_kt != 16)
    fail(SPMV_ERR_INVALID_ARG, "plan.block_kt must be 0, 4, 8 or 16");
  if (p.tiles_per_group < 1 || p.tiles_per_group > 64)
    fail(SPMV_ERR_INVALID_ARG, "plan.tiles_per_group must be in [1, 64]");
  if (p.panels != 1 && p.panels != 2 && p.panels != 4 && p.panels != 8)
    fail(SPMV_ERR_INVALID_ARG, "plan.panels must be 1, 2, 4 or 8");
}

PlanDev to_dev(const spmv_plan_t &p) {
  PlanDev d;
  d.kernel = p.kernel;
  d.tile_items = p.tile_items;
  d.lanes = p.lanes;
  d.nontemporal = p.nontemporal ? 1 : 0;
  d.xcd_remap = p.xcd_remap ? 1 : 0;
  d.tiles_per_group = p.tiles_per_group;
  return d;
}

const char *prec_name(int p) {
  switch (p) {
    case P_F64: return "f64";
    case P_F32: return "f32";
    case P_BF16: return "bf16";
    default: return "f32f64";
  }
}

// ---- one CRS part on the device -------------------------------------------------

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

  CsrDev dev() const {
    CsrDev d;
    d.row_ptr = row_ptr.as<const int32_t>();
    d.col = col.as<const int32_t>();
    d.val = val.p;
    d.row_ids = row_ids.p ? row_ids.as<const int32_t>() : nullptr;
    d.n_rows = n_rows;
    return d;
  }
  std::pair<const TileRP *, int64_t> tiles_for(int items) {
    auto it = tiles.find(items);
    if (it == tiles.end()) {
      const std::vector<int32_t> t = make_tiles(h_row_ptr.data(), n_rows, int64_t(kWG) * items);
      std::vector<TileRP> tr(t.size());
      for (size_t i = 0; i < t.size(); ++i) tr[i] = TileRP{t[i], h_row_ptr[size_t(t[i])]};
      DevBuf d;
      upload(d, tr.data(), tr.size() * sizeof(TileRP), "tiles");
      it = tiles.emplace(items, std::make_pair(std::move(d), int64_t(t.size()) - 1)).first;
    }
    return {it->second.first.as<const TileRP>(), it->second.second};
  }
  // Run table of the staged kernel for tiles of `items` (built on first use
  // from a copy of col_idx read back from the device; synchronous).
  const int32_t *runs_for(int items, int x_bytes) {
    auto it = runs.find(items);
    if (it == runs.end()) {
      const std::vector<int32_t> t = make_tiles(h_row_ptr.data(), n_rows, int64_t(kWG) * items);
      std::vector<int32_t> hc(static_cast<size_t>(nnz));
      if (nnz > 0)
        hip_ok(hipMemcpy(hc.data(), col.p, size_t(nnz) * 4, hipMemcpyDeviceToHost), "col readback");
      const std::vector<int32_t> table = make_runs(h_row_ptr.data(), hc.data(), t,
                                                   int64_t(kWG) * items - 4,
                                                   RUN_STAGE_BYTES / x_bytes);
      int64_t staged = 0;
      for (size_t i = 0; i < table.size(); i += RUN_WORDS) staged += table[i] > 0 ? 1 : 0;
      DevBuf d;
      upload(d, table.data(), table.size() * 4, "run table");
      it = runs.emplace(items, std::make_pair(std::move(d), staged)).first;
    }
    return it->second.first.as<const int32_t>();
  }
};

}  // namespace

// ---- handle ----------------------------------------------------------------------------

struct spmv_handle_s {
  uint64_t magic = kMagic;
  int kind = SPMV_KIND_PLAIN;
  int device = 0;
  int prec = P_F64;
  uint32_t flags = 0;
  int64_t n_rows = 0, n_cols = 0, nnz = 0;
  Part main;  // plain: the matrix; split: local part
  Part nl;    // split: nonlocal part
  int64_t halo_begin = 0;
  int schedule = SPMV_SCHEDULE_OVERLAP;
  hipStream_t copy_stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_copied = nullptr;
  // split: timing events of the last call's phases (see spmv_set_phase_timing)
  bool timing = false;
  hipEvent_t tev[9] = {};
  bool tran[4] = {};  // phases that ran in the last timed call
  // split: send side of the exchange
  DevBuf send_idx, send_buf;
  int64_t n_send = 0;
  hipStream_t send_stream = nullptr;
  hipEvent_t ev_sent = nullptr;
  // batch
  int32_t count = 0;
  std::vector<int64_t> m_rows, m_cols;
  DevBuf b_desc, b_tiles, b_counter;
  int64_t b_ntiles = 0;
  int b_tiles_items = 0;
  int b_grid = 0;
  DevBuf b_runs;           // run table of the batch tiles (staged kernel)
  int b_runs_items = 0;
  int64_t b_staged = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void *g_B = nullptr;
  void *g_C = nullptr;
  int g_items = -1, g_nt = -1, g_kernel = -1;
  std::vector<BatchTile> h_btiles;
  std::vector<BatchDesc> h_desc;
  std::map<int, spmv_plan_t> block_plans;  // k -> plan chosen by spmv_tune
  DevBuf kpm_part;                          // per-workgroup partial dot products

  ~spmv_handle_s() {
    if (copy_stream) (void)hipStreamSynchronize(copy_stream);
    if (send_stream) (void)hipStreamSynchronize(send_stream);
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
};

namespace {

std::mutex g_live_mu;
std::vector<spmv_handle_s *> g_live;

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

// ---- autotuner cache -----------------------------------------------------------------

std::mutex g_cache_mu;

std::string cache_path() {
  if (const char *p = std::getenv("SPMV_TUNE_CACHE")) return p;
  const char *home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/libspmv_tune.json";
}

std::string device_tag(int dev) {
  hipDeviceProp_t pr;
  if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
  std::string arch = pr.gcnArchName;
  const size_t c = arch.find(':');
  if (c != std::string::npos) arch = arch.substr(0, c);
  return arch + "-cu" + std::to_string(pr.multiProcessorCount);
}

std::string tune_key(int dev, int prec, int k, const char *part, int64_t n_rows,
                     const RowStats &s) {
  int nb = 0;
  while ((int64_t(1) << (nb + 1)) <= std::max<int64_t>(1, n_rows)) ++nb;
  int mb = 0;
  while ((int64_t(1) << (mb + 1)) <= std::max<int64_t>(1, s.max)) ++mb;
  std::ostringstream o;
  o << device_tag(dev) << "|" << prec_name(prec) << "|k" << k << "|" << part << "|n" << nb << "|m"
    << int(std::lround(s.mean)) << "|x" << mb << "|cv" << int(std::lround(s.cv * 4));
  return o.str();
}

// The cache file is a flat JSON object: "key": {"kernel": 1, ...}.
std::map<std::string, spmv_plan_t> cache_read() {
  std::map<std::string, spmv_plan_t> out;
  std::ifstream f(cache_path());
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t pos = 0;
  while (true) {
    const size_t k0 = s.find('"', pos);
    if (k0 == std::string::npos) break;
    const size_t k1 = s.find('"', k0 + 1);
    const size_t b0 = s.find('{', k1);
    const size_t b1 = s.find('}', b0);
    if (k1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) break;
    const std::string key = s.substr(k0 + 1, k1 - k0 - 1);
    const std::string body = s.substr(b0 + 1, b1 - b0 - 1);
    spmv_plan_t p = default_plan();
    auto field = [&](const char *name, int32_t &dst) {
      const std::string pat = std::string("\"") + name + "\"";
      const size_t q = body.find(pat);
      if (q == std::string::npos) return;
      const size_t colon = body.find(':', q);
      if (colon != std::string::npos) dst = int32_t(std::atoi(body.c_str() + colon + 1));
    };
    field("kernel", p.kernel);
    field("tile_items", p.tile_items);
    field("lanes", p.lanes);
    field("nontemporal", p.nontemporal);
    field("xcd_remap", p.xcd_remap);
    field("block_kt", p.block_kt);
    field("tiles_per_group", p.tiles_per_group);
    field("panels", p.panels);
    out[key] = p;
    pos = b1 + 1;
  }
  return out;
}

bool cache_lookup(const std::string &key, spmv_plan_t *p) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto m = cache_read();
  auto it = m.find(key);
  if (it == m.end()) return false;
  try {
    check_plan(it->second);
  } catch (const Failure &) {
    return false;
  }
  *p = it->second;
  return true;
}

void cache_store(const std::string &key, const spmv_plan_t &p) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto m = cache_read();
  m[key] = p;
  const std::string path = cache_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    const std::string dir = path.substr(0, slash);
    for (size_t i = 1; i <= dir.size(); ++i)
      if (i == dir.size() || dir[i] == '/') (void)::mkdir(dir.substr(0, i).c_str(), 0755);
  }
  const std::string tmp = path + ".tmp" + std::to_string(::getpid());
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t i = 0;
    for (auto &kv : m) {
      const spmv_plan_t &q = kv.second;
      f << "  \"" << kv.first << "\": {\"kernel\": " << q.kernel << ", \"tile_items\": "
        << q.tile_items << ", \"lanes\": " << q.lanes << ", \"nontemporal\": " << q.nontemporal
        << ", \"xcd_remap\": " << q.xcd_remap << ", \"block_kt\": " << q.block_kt
        << ", \"tiles_per_group\": " << q.tiles_per_group << ", \"panels\": " << q.panels
        << "}"
        << (++i < m.size() ? ",\n" : "\n");
    }
    f << "}\n";
  }
  std::rename(tmp.c_str(), path.c_str());
}

}  // namespace

// ==== a1: ingest ===========================================================================

namespace {

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

// Host arrays shifted to 0-based, values encoded to the storage precision.
struct Encoded {
  std::vector<int32_t> rp;
  std::vector<int32_t> col;  // empty when no shift is needed (use caller's)
  std::vector<uint8_t> val;  // empty for f64 without shift (use caller's)
  const int32_t *col_ptr = nullptr;
  const void *val_ptr = nullptr;
};

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

std::vector<std::unique_ptr<Part>> &build_panels(spmv_handle_s *h, Part &p, int K);
void prepare_part(spmv_handle_s *h, Part &p);

void choose_plan(spmv_handle_s *h, Part &p, const char *part_name) {
  p.plan = default_plan();
  if (h->kind == SPMV_KIND_SYMMETRIC) {  // the symmetric kernel: lanes per row only
    p.plan.kernel = SPMV_KERNEL_VECTOR;
    p.plan.lanes = 16;
    if (!(h->flags & SPMV_FLAG_NO_TUNE_CACHE)) {
      spmv_plan_t c;
      if (cache_lookup(tune_key(h->device, h->prec, 1, "symmetric", p.n_rows, p.stats), &c) &&
          c.kernel == SPMV_KERNEL_VECTOR && c.panels == 1)
        p.plan = c;
    }
    return;
  }
  if (!(h->flags & SPMV_FLAG_NO_TUNE_CACHE)) {
    spmv_plan_t c;
    if (cache_lookup(tune_key(h->device, h->prec, 1, part_name, p.n_rows, p.stats), &c)) p.plan = c;
  }
  if (p.plan.panels > 1 && (p.row_ids.p || h->kind == SPMV_KIND_BATCH)) p.plan.panels = 1;
  if (p.plan.panels > 1) build_panels(h, p, p.plan.panels);
  if (h->kind != SPMV_KIND_BATCH) prepare_part(h, p);
  if (std::getenv("SPMV_LOG"))
    std::fprintf(stderr, "libspmv: %s part n=%lld nnz=%lld mean=%.2f max=%lld cv=%.2f -> kernel=%d "
                         "tile_items=%d lanes=%d nt=%d remap=%d\n",
                 part_name, (long long)p.n_rows, (long long)p.nnz, p.stats.mean,
                 (long long)p.stats.max, p.stats.cv, p.plan.kernel, p.plan.tile_items,
                 p.plan.lanes, p.plan.nontemporal, p.plan.xcd_remap);
}

int current_device() {
  int d = 0;
  hip_ok(hipGetDevice(&d), "hipGetDevice");
  return d;
}

}  // namespace

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
  upload(m.row_ptr, enc.rp.data(), enc.rp.size() * 4, "row_ptr");
  upload(m.col, enc.col_ptr, size_t(nnz) * 4, "col_idx");
  upload(m.val, enc.val_ptr, size_t(nnz) * val_bytes(p), "val");
  m.h_row_ptr = std::move(enc.rp);
  m.stats = row_stats(m.h_row_ptr.data(), n_rows);
  choose_plan(h.get(), m, kind == SPMV_KIND_SYMMETRIC ? "symmetric" : "main");
  register_handle(h.get());
  return h.release();
}

}  // namespace

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
    choose_plan(h.get(), L, "local");
    choose_plan(h.get(), N, "nonlocal");
    hip_ok(hipStreamCreateWithFlags(&h->copy_stream, hipStreamNonBlocking), "copy stream");
    hip_ok(hipEventCreateWithFlags(&h->ev_start, hipEventDisableTiming), "event");
    hip_ok(hipEventCreateWithFlags(&h->ev_copied, hipEventDisableTiming), "event");
    hip_ok(hipStreamCreateWithFlags(&h->send_stream, hipStreamNonBlocking), "send stream");
    hip_ok(hipEventCreateWithFlags(&h->ev_sent, hipEventDisableTiming), "event");
    register_handle(h.get());
    *out_split = h.release();
  });
}

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
    upload(M.row_ptr, M.h_row_ptr.data(), M.h_row_ptr.size() * 4, "batch row_ptr");
    upload(M.col, col_all.data(), col_all.size() * 4, "batch col_idx");
    upload(M.val, val_all.data(), val_all.size(), "batch val");
    upload(h->b_desc, h->h_desc.data(), h->h_desc.size() * sizeof(BatchDesc), "batch descriptors");
    h->b_counter.alloc(8 * sizeof(int32_t), "batch queue counters");
    choose_plan(h.get(), M, "batch");
    hip_ok(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking), "capture stream");
    register_handle(h.get());
    *out = h.release();
  });
}

namespace {

// Tile queue of a batch for the current tile size.
void batch_runs(spmv_handle_s *h);

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
    for (size_t i = 0; i + 1 < t.size(); ++i) tl.push_back(BatchTile{m, t[i], t[i + 1], 0});
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
          const BatchDesc &D = h->h_desc[size_t(T.member)];
          const int64_t p0 = M.h_row_ptr[size_t(D.rp_off + T.r0)];
          const int64_t p1 = M.h_row_ptr[size_t(D.rp_off + T.r1)];
          run_row(hc.data() + D.nz_off + p0, p1 - p0, int64_t(kWG) * items - 4, budget, cs,
                  table.data() + size_t(t) * RUN_WORDS);
        }
      },
      64);
  int64_t staged = 0;
  for (size_t i = 0; i < table.size(); i += RUN_WORDS) staged += table[i] > 0 ? 1 : 0;
  upload(h->b_runs, table.data(), table.size() * 4, "batch run table");
  h->b_runs_items = items;
  h->b_staged = staged;
}

hipError_t batch_launch_direct(spmv_handle_s *h, const void *B, void *C, hipStream_t s) {
  if (h->main.plan.kernel == SPMV_KERNEL_STAGED)
    return launch_batch_staged(h->prec, h->main.row_ptr.as<int32_t>(), h->main.col.as<int32_t>(),
                               h->main.val.p, h->b_desc.as<BatchDesc>(), h->b_tiles.as<BatchTile>(),
                               h->b_runs.as<int32_t>(), h->b_ntiles, h->b_tiles_items,
                               h->main.plan.nontemporal, B, C, s);
  if (h->main.plan.kernel == SPMV_KERNEL_TILE_GRID)
    return launch_batch_flat(h->prec, h->main.row_ptr.as<int32_t>(), h->main.col.as<int32_t>(),
                             h->main.val.p, h->b_desc.as<BatchDesc>(), h->b_tiles.as<BatchTile>(),
                             h->b_ntiles, h->b_tiles_items, h->main.plan.nontemporal, B, C, s);
  hipError_t e = launch_batch_reset(h->b_counter.as<int32_t>(), s);
  if (e != hipSuccess) return e;
  return launch_batch_persistent(h->prec, h->main.row_ptr.as<int32_t>(), h->main.col.as<int32_t>(),
                                 h->main.val.p, h->b_desc.as<BatchDesc>(),
                                 h->b_tiles.as<BatchTile>(), h->b_ntiles, h->b_tiles_items,
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
                             h->main.val.p, h->b_desc.as<BatchDesc>(), h->b_tiles.as<BatchTile>(),
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

// Host memory of a copy that must overlap: pinned, unless the handle allows
// pageable memory (a pageable copy is staged by the runtime and does not
// proceed beside the kernels; nonblocking is not asynchronous, Sect. 3.1).
// Phase events of split handles: tev[0] the call's start; then start and
// end of the halo copy (1, 2), the local part (3, 4), the nonlocal part
// (5, 6) and the send side (7, 8).
enum { T_START = 0, T_COPY = 1, T_LOCAL = 3, T_NONLOCAL = 5, T_SEND = 7 };

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

// Drops panel sets no chosen plan uses (each is a full copy of the part).
void prune_panels(Part &p, const std::vector<int> &keep) {
  for (auto it = p.panel_sets.begin(); it != p.panel_sets.end();) {
    if (std::find(keep.begin(), keep.end(), it->first) == keep.end())
      it = p.panel_sets.erase(it);
    else
      ++it;
  }
}

// Tiles (and, for the staged kernel, run tables) of the part's plan, and of
// its panels when the plan uses them: built here so that spmv_run only
// enqueues work.
void prepare_part(spmv_handle_s *h, Part &p) {
  const int items = p.plan.tile_items;
  const bool staged = p.plan.kernel == SPMV_KERNEL_STAGED;
  const int xb = vec_bytes(h->prec);
  if (p.plan.panels > 1) {
    for (auto &q : build_panels(h, p, p.plan.panels)) {
      (void)q->tiles_for(items);
      if (staged) (void)q->runs_for(items, xb);
    }
    return;
  }
  (void)p.tiles_for(items);
  if (staged) (void)p.runs_for(items, xb);
}

void run_part(spmv_handle_s *h, Part &p, const void *B, void *C, hipStream_t s) {
  if (p.n_rows == 0 || p.nnz == 0) return;
  const bool staged = p.plan.kernel == SPMV_KERNEL_STAGED;
  const int xb = vec_bytes(h->prec);
  if (p.plan.panels > 1) {
    auto &set = build_panels(h, p, p.plan.panels);
    spmv_plan_t sub = p.plan;
    sub.panels = 1;
    const PlanDev pl = to_dev(sub);
    for (auto &q : set) {
      if (q->nnz == 0) continue;
      auto t = q->tiles_for(sub.tile_items);
      const int32_t *r = staged ? q->runs_for(sub.tile_items, xb) : nullptr;
      hip_ok(launch_spmv(h->prec, q->dev(), pl, t.first, r, t.second, B, C, s), "kernel launch");
    }
    return;
  }
  const PlanDev pl = to_dev(p.plan);
  auto t = p.tiles_for(p.plan.tile_items);
  const int32_t *r = staged ? p.runs_for(p.plan.tile_items, xb) : nullptr;
  hip_ok(launch_spmv(h->prec, p.dev(), pl, t.first, r, t.second, B, C, s), "kernel launch");
}

}  // namespace

namespace {

void run_sym(spmv_handle_s *h, const void *B, void *C, hipStream_t s) {
  const Part &p = h->main;
  if (p.n_rows == 0 || p.nnz == 0) return;
  hip_ok(launch_spmv_sym(p.dev(), p.plan.lanes, p.plan.nontemporal, p.plan.xcd_remap,
                         static_cast<const double *>(B), static_cast<double *>(C), s),
         "symmetric kernel launch");
}

}  // namespace

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
    const int64_t n_halo = h->n_cols - h->halo_begin;
    const size_t vb = size_t(vec_bytes(h->prec));
    void *recv = static_cast<char *>(const_cast<void *>(B)) + size_t(h->halo_begin) * vb;
    const bool copy = B_halo_host && n_halo > 0;
    if (copy) require_pinned(h, B_halo_host, "B_halo_host");
    begin_timed_call(h, s);
    if (copy && h->schedule == SPMV_SCHEDULE_OVERLAP) {
      hip_ok(hipEventRecord(h->ev_start, s), "event record");
      hip_ok(hipStreamWaitEvent(h->copy_stream, h->ev_start, 0), "stream wait");
      mark(h, T_COPY, h->copy_stream);
      hip_ok(hipMemcpyAsync(recv, B_halo_host, size_t(n_halo) * vb, hipMemcpyHostToDevice,
                            h->copy_stream),
             "halo copy");
      mark(h, T_COPY + 1, h->copy_stream);
      hip_ok(hipEventRecord(h->ev_copied, h->copy_stream), "event record");
      mark(h, T_LOCAL, s);
      run_part(h, h->main, B, C, s);
      mark(h, T_LOCAL + 1, s);
      hip_ok(hipStreamWaitEvent(s, h->ev_copied, 0), "stream wait");
      mark(h, T_NONLOCAL, s);
      run_part(h, h->nl, B, C, s);
      mark(h, T_NONLOCAL + 1, s);
    } else {
      if (copy) {
        mark(h, T_COPY, s);
        hip_ok(hipMemcpyAsync(recv, B_halo_host, size_t(n_halo) * vb, hipMemcpyHostToDevice, s),
               "halo copy");
        mark(h, T_COPY + 1, s);
      }
      mark(h, T_LOCAL, s);
      run_part(h, h->main, B, C, s);
      mark(h, T_LOCAL + 1, s);
      mark(h, T_NONLOCAL, s);
      run_part(h, h->nl, B, C, s);
      mark(h, T_NONLOCAL + 1, s);
    }
    h->tran[0] = copy;
    h->tran[1] = h->tran[2] = true;
    h->tran[3] = false;
  });
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
      mark(h, T_LOCAL, s);
      run_part(h, h->main, B, C, s);
      mark(h, T_LOCAL + 1, s);
      mark(h, T_NONLOCAL, s);
      run_part(h, h->nl, B, C, s);
      mark(h, T_NONLOCAL + 1, s);
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
    mark(h, T_LOCAL, s);
    run_part(h, h->main, B, C, s);
    mark(h, T_LOCAL + 1, s);
    if (copy) hip_ok(hipStreamWaitEvent(s, h->ev_copied, 0), "stream wait");
    mark(h, T_NONLOCAL, s);
    run_part(h, h->nl, B, C, s);
    mark(h, T_NONLOCAL + 1, s);
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

// ==== a8: block of right-hand sides ===================================================================

namespace {

int default_kt(int k) {
  if (k <= 4) return 4;
  if (k <= 8) return 8;
  return 16;
}

// Block product C = C + scale*A*B over a part, or over its diagonal panels
// in turn when `panels` > 1 (the panels are shared with the single-vector
// plan).  `scale` is 1 or a power of two, applied exactly to every value.
void run_block_part(spmv_handle_s *h, Part &p, int kt, int nt, int remap, int panels, int k,
                    const void *B, int64_t ldb, void *C, int64_t ldc, hipStream_t s,
                    double scale = 1.0) {
  if (p.n_rows == 0 || p.nnz == 0) return;
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

// C = C + scale*A*B for k columns of a plain handle (arguments already
// checked; scale as in run_block_part).
void block_product(spmv_handle_s *h, int k, const void *B, int64_t ldb, void *C, int64_t ldc,
                   hipStream_t s, double scale = 1.0) {
    Part &p = h->main;
    // per-k choices made by spmv_tune for this handle, else the cache, else defaults
    int kt = p.plan.block_kt, nt = p.plan.nontemporal, panels = p.plan.panels;
    auto it = h->block_plans.find(k);
    if (it != h->block_plans.end()) {
      kt = it->second.block_kt;
      nt = it->second.nontemporal;
      panels = it->second.panels;
    } else if (kt == 0) {
      spmv_plan_t c;
      kt = default_kt(k);
      if (!(h->flags & SPMV_FLAG_NO_TUNE_CACHE) &&
          cache_lookup(tune_key(h->device, h->prec, k, "block", p.n_rows, p.stats), &c) &&
          c.block_kt) {
        kt = c.block_kt;
        nt = c.nontemporal;
        panels = c.panels;
        h->block_plans[k] = c;
      }
    }
    run_block_part(h, p, kt, nt, p.plan.xcd_remap, panels, k, B, ldb, C, ldc, s, scale);
}

}  // namespace

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

// ==== destroy / errors ==================================================================================

extern "C" spmv_status_t spmv_destroy(spmv_handle_t h) {
  if (!h) {
    g_last_error.clear();
    return SPMV_OK;
  }
  return guarded([&] {
    if (!unregister_handle(h)) fail(SPMV_ERR_STATE, "handle is not live (destroyed or foreign)");
    DeviceGuard dg(h->device);
    h->magic = kDead;
    delete h;
  });
}

extern "C" const char *spmv_last_error(void) { return g_last_error.c_str(); }

// ==== a10: plans and autotuner ===========================================================================

namespace {

Part &part_of(spmv_handle_s *h, int32_t part) {
  if (part == SPMV_PART_MAIN) return h->main;
  if (part == SPMV_PART_NONLOCAL && h->kind == SPMV_KIND_SPLIT) return h->nl;
  fail(SPMV_ERR_INVALID_ARG, "no such part in this handle");
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  Timer() {
    hip_ok(hipEventCreate(&a), "event");
    hip_ok(hipEventCreate(&b), "event");
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  template <class F>
  float median_ms(F &&launch, hipStream_t s, int warm = 2, int reps = 7) {
    for (int i = 0; i < warm; ++i) launch();
    std::vector<float> t;
    for (int i = 0; i < reps; ++i) {
      hip_ok(hipEventRecord(a, s), "event record");
      launch();
      hip_ok(hipEventRecord(b, s), "event record");
      hip_ok(hipEventSynchronize(b), "event sync");
      float ms = 0;
      hip_ok(hipEventElapsedTime(&ms, a, b), "elapsed");
      t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
  }
};

std::vector<spmv_plan_t> candidates() {
  std::vector<spmv_plan_t> c;
  for (int e : {4, 8, 16})
    for (int tpw : {1, 2, 4, 8, 16, 32}) {
      spmv_plan_t p = default_plan();
      p.tile_items = e;
      p.tiles_per_group = tpw;
      c.push_back(p);
    }
  for (int e : {4, 8}) {
    spmv_plan_t p = default_plan();
    p.tile_items = e;
    p.tiles_per_group = 8;
    p.nontemporal = 0;
    c.push_back(p);
    p.nontemporal = 1;
    p.xcd_remap = 0;
    c.push_back(p);
  }
  for (int l : {4, 8, 16, 32, 64}) {
    spmv_plan_t p = default_plan();
    p.kernel = SPMV_KERNEL_VECTOR;
    p.lanes = l;
    c.push_back(p);
  }
  for (int e : {8, 16})
    for (int rm : {1, 0}) {
      spmv_plan_t p = default_plan();
      p.kernel = SPMV_KERNEL_STAGED;
      p.tile_items = e;
      p.xcd_remap = rm;
      c.push_back(p);
    }
  return c;
}

// Diagonal-panel candidates (parts that cover all rows only).
std::vector<spmv_plan_t> panel_candidates() {
  std::vector<spmv_plan_t> c;
  for (int k : {2, 4, 8})
    for (int e : {4, 8, 16})
      for (int rm : {0, 1}) {
        spmv_plan_t p = default_plan();
        p.panels = k;
        p.tile_items = e;
        p.xcd_remap = rm;
        c.push_back(p);
      }
  for (int k : {4, 8}) {
    spmv_plan_t p = default_plan();
    p.panels = k;
    p.tile_items = 8;
    p.tiles_per_group = 4;
    c.push_back(p);
  }
  return c;
}

// Whether the staged kernel can stage most tiles of `items` entries per
// lane: the run rule applied to up to 64 tiles spread over the part, whose
// columns alone are read back.  Saves building whole run tables (a copy of
// col_idx and a sort per tile) for matrices whose tiles would all gather.
bool staged_promising(const spmv_handle_s *h, const Part &p, int items) {
  const std::vector<int32_t> t = make_tiles(p.h_row_ptr.data(), p.n_rows, int64_t(kWG) * items);
  const int64_t n_tiles = int64_t(t.size()) - 1;
  if (n_tiles <= 0) return false;
  const int64_t n_sample = std::min<int64_t>(64, n_tiles);
  std::vector<int32_t> rp_s{0}, tiles_s{0}, col_s;
  for (int64_t i = 0; i < n_sample; ++i) {
    const int64_t k = i * n_tiles / n_sample;
    const int64_t p0 = p.h_row_ptr[size_t(t[size_t(k)])], p1 = p.h_row_ptr[size_t(t[size_t(k + 1)])];
    const size_t at = col_s.size();
    col_s.resize(at + size_t(p1 - p0));
    if (p1 > p0)
      hip_ok(hipMemcpy(col_s.data() + at, p.col.as<int32_t>() + p0, size_t(p1 - p0) * 4,
                       hipMemcpyDeviceToHost),
             "col readback");
    rp_s.push_back(int32_t(col_s.size()));  // one pseudo-row per sampled tile
    tiles_s.push_back(int32_t(i + 1));
  }
  const std::vector<int32_t> table =
      make_runs(rp_s.data(), col_s.data(), tiles_s, int64_t(kWG) * items - 4,
                RUN_STAGE_BYTES / vec_bytes(h->prec));
  int64_t fit = 0;
  for (size_t i = 0; i < table.size(); i += RUN_WORDS) fit += table[i] > 0 ? 1 : 0;
  return 2 * fit > n_sample;
}

void tune_part(spmv_handle_s *h, Part &p, const char *name, void *x, void *y, hipStream_t s,
               Timer &tm) {
  if (p.n_rows == 0 || p.nnz == 0) return;
  float best = 1e30f;
  spmv_plan_t best_p = p.plan;
  std::vector<spmv_plan_t> cands;
  {
    const bool promising[2] = {staged_promising(h, p, 8), staged_promising(h, p, 16)};
    for (const spmv_plan_t &c : candidates())
      if (c.kernel != SPMV_KERNEL_STAGED || promising[c.tile_items == 16 ? 1 : 0])
        cands.push_back(c);
  }
  if (!p.row_ids.p) {
    const std::vector<spmv_plan_t> pc = panel_candidates();
    cands.insert(cands.end(), pc.begin(), pc.end());
  }
  std::vector<float> times;
  for (const spmv_plan_t &c : cands) {
    p.plan = c;
    prepare_part(h, p);
    times.push_back(tm.median_ms([&] { run_part(h, p, x, y, s); }, s));
    best = std::min(best, times.back());
  }
  // the earliest candidate within 1% of the fastest: near-ties resolve the
  // same way from run to run
  for (size_t i = 0; i < cands.size(); ++i)
    if (times[i] <= best * 1.01f) {
      best_p = cands[i];
      best = times[i];
      break;
    }
  best_p.block_kt = 0;
  p.plan = best_p;
  prepare_part(h, p);
  // free the device copies of panel sets no chosen plan uses
  std::vector<int> keep{p.plan.panels};
  for (auto &bp : h->block_plans) keep.push_back(bp.second.panels);
  prune_panels(p, keep);
  if (std::getenv("SPMV_LOG"))
    std::fprintf(stderr, "libspmv: tuned %s part: kernel=%d tile_items=%d lanes=%d nt=%d remap=%d "
                         "(%.1f us)\n",
                 name, p.plan.kernel, p.plan.tile_items, p.plan.lanes, p.plan.nontemporal,
                 p.plan.xcd_remap, best * 1000.0f);
  if (!(h->flags & SPMV_FLAG_NO_TUNE_CACHE))
    cache_store(tune_key(h->device, h->prec, 1, name, p.n_rows, p.stats), p.plan);
}

}  // namespace

extern "C" spmv_status_t spmv_get_plan(spmv_handle_t h_, int32_t part, spmv_plan_t *plan) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    if (!plan) fail(SPMV_ERR_INVALID_ARG, "plan is null");
    *plan = part_of(h, part).plan;
  });
}

extern "C" spmv_status_t spmv_set_plan(spmv_handle_t h_, int32_t part, const spmv_plan_t *plan) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    if (!plan) fail(SPMV_ERR_INVALID_ARG, "plan is null");
    check_plan(*plan);
    if (h->kind == SPMV_KIND_BATCH && plan->kernel == SPMV_KERNEL_VECTOR)
      fail(SPMV_ERR_UNSUPPORTED, "batch handles run the stream, tile-grid or staged kernel");
    if (h->kind == SPMV_KIND_SYMMETRIC && (plan->kernel != SPMV_KERNEL_VECTOR || plan->panels != 1))
      fail(SPMV_ERR_UNSUPPORTED, "symmetric handles take SPMV_KERNEL_VECTOR plans (lanes per row)");
    if (h->kind != SPMV_KIND_BATCH && plan->kernel == SPMV_KERNEL_TILE_GRID)
      fail(SPMV_ERR_UNSUPPORTED, "the tile-grid kernel serves batch handles only");
    if (h->kind == SPMV_KIND_BATCH && plan->panels != 1)
      fail(SPMV_ERR_UNSUPPORTED, "batch handles do not use diagonal panels");
    Part &p = part_of(h, part);
    if (plan->panels > 1 && p.row_ids.p)
      fail(SPMV_ERR_UNSUPPORTED, "diagonal panels need a part that covers all rows");
    DeviceGuard dg(h->device);
    p.plan = *plan;
    if (h->kind == SPMV_KIND_BATCH)
      batch_prepare(h);
    else if (h->kind != SPMV_KIND_SYMMETRIC)
      prepare_part(h, p);
  });
}

extern "C" spmv_status_t spmv_tune(spmv_handle_t h_, int32_t k, void *stream) {
  return guarded([&] {
    spmv_handle_s *h = live(h_);
    if (k < 1 || k > 64) fail(SPMV_ERR_INVALID_ARG, "k must be in [1, 64]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard dg(h->device);
    Timer tm;
    const int64_t xb = std::max<int64_t>(1, h->n_cols) * k * vec_bytes(h->prec);
    const int64_t yb = std::max<int64_t>(1, h->n_rows) * k * vec_bytes(h->prec);
    DevBuf x, y;
    x.alloc(size_t(xb), "tune B");
    y.alloc(size_t(yb), "tune C");
    hip_ok(hipMemsetAsync(x.p, 0, size_t(xb), s), "memset");
    hip_ok(hipMemsetAsync(y.p, 0, size_t(yb), s), "memset");
    if (h->kind == SPMV_KIND_BATCH) {
      Part &p = h->main;
      const spmv_plan_t keep = p.plan;
      float best = 1e30f;
      spmv_plan_t best_p = keep;
      const int saved_sched = h->schedule;
      h->schedule = SPMV_SCHEDULE_BATCH_DIRECT;
      for (int kern : {SPMV_KERNEL_STREAM, SPMV_KERNEL_TILE_GRID, SPMV_KERNEL_STAGED})
      for (int e : {4, 8, 16})
        for (int nt : {1, 0}) {
          if (kern == SPMV_KERNEL_STAGED && e == 4) continue;
          p.plan = keep;
          p.plan.kernel = kern;
          p.plan.tile_items = e;
          p.plan.nontemporal = nt;
          batch_prepare(h);  // tiles and run tables before the timing
          const float ms = tm.median_ms([&] { batch_run(h, x.p, y.p, s); }, s);
          if (ms < best) {
            best = ms;
            best_p = p.plan;
          }
        }
      h->schedule = saved_sched;
      p.plan = best_p;
      if (!(h->flags & SPMV_FLAG_NO_TUNE_CACHE))
        cache_store(tune_key(h->device, h->prec, 1, "batch", p.n_rows, p.stats), p.plan);
      return;
    }
    if (h->kind == SPMV_KIND_SYMMETRIC) {
      if (k != 1) fail(SPMV_ERR_UNSUPPORTED, "symmetric handles serve one right-hand side");
      Part &p = h->main;
      float best = 1e30f;
      spmv_plan_t best_p = p.plan;
      for (int l : {4, 8, 16, 32, 64})
        for (int nt : {1, 0}) {
          p.plan = default_plan();
          p.plan.kernel = SPMV_KERNEL_VECTOR;
          p.plan.lanes = l;
          p.plan.nontemporal = nt;
          const float ms = tm.median_ms([&] { run_sym(h, x.p, y.p, s); }, s);
          if (ms < best * 0.99f) {
            best = ms;
            best_p = p.plan;
          }
        }
      p.plan = best_p;
      if (!(h->flags & SPMV_FLAG_NO_TUNE_CACHE))
        cache_store(tune_key(h->device, h->prec, 1, "symmetric", p.n_rows, p.stats), p.plan);
      return;
    }
    if (k == 1) {
      tune_part(h, h->main, h->kind == SPMV_KIND_SPLIT ? "local" : "main", x.p, y.p, s, tm);
      if (h->kind == SPMV_KIND_SPLIT) tune_part(h, h->nl, "nonlocal", x.p, y.p, s, tm);
      return;
    }
    if (h->kind != SPMV_KIND_PLAIN) fail(SPMV_ERR_UNSUPPORTED, "block tuning needs a plain handle");
    Part &p = h->main;
    float best = 1e30f;
    int best_kt = default_kt(k), best_nt = p.plan.nontemporal, best_pn = 1;
    for (int pn : {1, 2, 4, 8})
      for (int kt : {4, 8, 16}) {
        if (kt > 2 * k && kt != 4) continue;
        for (int nt : {1, 0}) {
          const float ms = tm.median_ms(
              [&] { run_block_part(h, p, kt, nt, p.plan.xcd_remap, pn, k, x.p, k, y.p, k, s); }, s);
          if (ms < best * 0.99f) {
            best = ms;
            best_kt = kt;
            best_nt = nt;
            best_pn = pn;
          }
        }
      }
    spmv_plan_t c = p.plan;
    c.block_kt = best_kt;
    c.nontemporal = best_nt;
    c.panels = best_pn;
    h->block_plans[k] = c;
    std::vector<int> keep{p.plan.panels};
    for (auto &bp : h->block_plans) keep.push_back(bp.second.panels);
    prune_panels(p, keep);
    if (std::getenv("SPMV_LOG"))
      std::fprintf(stderr, "libspmv: tuned block k=%d: kt=%d nt=%d panels=%d (%.1f us)\n", k,
                   best_kt, best_nt, best_pn, best * 1000.0f);
    if (!(h->flags & SPMV_FLAG_NO_TUNE_CACHE))
      cache_store(tune_key(h->device, h->prec, k, "block", p.n_rows, p.stats), c);
  });
}

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
                          (schedule == SPMV_SCHEDULE_OVERLAP || schedule == SPMV_SCHEDULE_SERIAL);
    const bool ok_batch = h->kind == SPMV_KIND_BATCH &&
                          (schedule == SPMV_SCHEDULE_BATCH_GRAPH ||
                           schedule == SPMV_SCHEDULE_BATCH_DIRECT ||
                           schedule == SPMV_SCHEDULE_BATCH_FLAT);
    if (!ok_split && !ok_batch) fail(SPMV_ERR_INVALID_ARG, "schedule not valid for this handle");
    h->schedule = schedule;
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
