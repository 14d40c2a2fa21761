// libspmv runtime, plan unit: row statistics, the stream kernel's tiles, the
// staged kernel's run tables, kernel plans (the row -> lane mapping, the
// GPU's analogue of the loop schedule of Sect. 2), running one part with its
// plan, and the autotuner with its persistent cache.
#include <hip/hip_runtime_api.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.h"

using namespace spmv;

namespace spmv {
namespace rt {

// ---- row statistics and tiles ----------------------------------------------------

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

// Greedy tiles: at most `tile` - 4 entries (room for the kernel's grouped
// loads to start up to three entries early) and at most 512 rows (two per
// lane of the workgroup, whose bounds the kernel prefetches).
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
namespace {
constexpr int64_t kRunGap = 16;
}  // namespace

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
      p.kernel != SPMV_KERNEL_TILE_GRID && p.kernel != SPMV_KERNEL_STAGED &&
      p.kernel != SPMV_KERNEL_FUSED_PANELS && p.kernel != SPMV_KERNEL_SORTED_BLOCKS)
    fail(SPMV_ERR_INVALID_ARG, "plan.kernel must be SPMV_KERNEL_STREAM, _VECTOR, _TILE_GRID, "
                               "_STAGED, _FUSED_PANELS or _SORTED_BLOCKS");
  if (p.kernel == SPMV_KERNEL_SORTED_BLOCKS) {
    if (p.tile_items != 1 && p.tile_items != 2 && p.tile_items != 4)
      fail(SPMV_ERR_INVALID_ARG, "the sorted-block kernel takes tile_items 1, 2 or 4");
    if (p.panels != 1) fail(SPMV_ERR_INVALID_ARG, "the sorted-block kernel takes panels 1");
  } else if (p.tile_items != 4 && p.tile_items != 8 && p.tile_items != 16) {
    fail(SPMV_ERR_INVALID_ARG, "plan.tile_items must be 4, 8 or 16");
  }
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

std::vector<int32_t> Part::host_tiles(int items) const {
  const int64_t cap = int64_t(kWG) * items;
  if (cut_row <= 0 || cut_row >= n_rows) return make_tiles(h_row_ptr.data(), n_rows, cap);
  std::vector<int32_t> t = make_tiles(h_row_ptr.data(), cut_row, cap);
  const std::vector<int32_t> t2 = make_tiles(h_row_ptr.data() + cut_row, n_rows - cut_row, cap);
  for (size_t i = 1; i < t2.size(); ++i) t.push_back(int32_t(t2[i] + cut_row));
  return t;
}

std::pair<const TileRP *, int64_t> Part::tiles_for(int items) {
  auto it = tiles.find(items);
  if (it == tiles.end()) {
    const std::vector<int32_t> t = host_tiles(items);
    if (cut_row > 0 && cut_row < n_rows)
      cut_tile[items] = int64_t(std::lower_bound(t.begin(), t.end(), int32_t(cut_row)) - t.begin());
    std::vector<TileRP> tr(t.size());
    for (size_t i = 0; i < t.size(); ++i) tr[i] = TileRP{t[i], h_row_ptr[size_t(t[i])]};
    DevBuf d;
    upload(d, tr.data(), tr.size() * sizeof(TileRP), "tiles");
    it = tiles.emplace(items, std::make_pair(std::move(d), int64_t(t.size()) - 1)).first;
  }
  return {it->second.first.as<const TileRP>(), it->second.second};
}
const int32_t *Part::runs_for(int items, int x_bytes) {
  auto it = runs.find(items);
  if (it == runs.end()) {
    const std::vector<int32_t> t = host_tiles(items);
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

// ---- autotuner cache -----------------------------------------------------------------

namespace {

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

}  // namespace

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

namespace {

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

}  // namespace

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
  if (p.plan.kernel == SPMV_KERNEL_FUSED_PANELS && (p.row_ids.p || h->kind == SPMV_KIND_BATCH))
    p.plan.kernel = SPMV_KERNEL_STREAM;
  if (p.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS && (p.row_ids.p || h->kind == SPMV_KIND_BATCH))
    p.plan = default_plan();
  if (p.plan.panels > 1) build_panels(h, p, p.plan.panels);
  if (h->kind != SPMV_KIND_BATCH) prepare_part(h, p);
  if (std::getenv("SPMV_LOG"))
    std::fprintf(stderr, "libspmv: %s part n=%lld nnz=%lld mean=%.2f max=%lld cv=%.2f -> kernel=%d "
                         "tile_items=%d lanes=%d nt=%d remap=%d\n",
                 part_name, (long long)p.n_rows, (long long)p.nnz, p.stats.mean,
                 (long long)p.stats.max, p.stats.cv, p.plan.kernel, p.plan.tile_items,
                 p.plan.lanes, p.plan.nontemporal, p.plan.xcd_remap);
}

// Tiles (and, for the staged kernel, run tables) of the part's plan, and of
// its panels when the plan uses them: built here so that spmv_run only
// enqueues work.
void prepare_part(spmv_handle_s *h, Part &p) {
  const int items = p.plan.tile_items;
  const bool staged = p.plan.kernel == SPMV_KERNEL_STAGED;
  const int xb = vec_bytes(h->prec);
  if (p.plan.kernel == SPMV_KERNEL_FUSED_PANELS) {
    (void)fused_rows_for(h, p, p.plan.panels, kWG * items - 4);
    return;
  }
  if (p.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS) {
    if (p.n_rows > 0 && p.nnz > 0) {
      (void)sorted_for(h, p, items);
      // block products of this plan use the block form of the kernel
      if (p.plan.block_kt != 0) (void)sorted_for(h, p, items, p.plan.block_kt);
    }
    return;
  }
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


bool part_prepared(const Part &p, int x_bytes) {
  (void)x_bytes;
  const int items = p.plan.tile_items;
  if (p.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS)
    return p.n_rows == 0 || p.nnz == 0 || p.sorted.find(std::make_pair(items, 1)) != p.sorted.end();
  if (p.plan.kernel == SPMV_KERNEL_FUSED_PANELS) {
    if (p.plan.panels > 1 && p.panel_sets.find(p.plan.panels) == p.panel_sets.end()) return false;
    return p.fused_rows.find(std::make_pair(p.plan.panels, kWG * items - 4)) != p.fused_rows.end();
  }
  const bool staged = p.plan.kernel == SPMV_KERNEL_STAGED;
  auto ready = [&](const Part &q) {
    if (q.n_rows == 0 || q.nnz == 0) return true;
    if (p.plan.kernel == SPMV_KERNEL_VECTOR) return true;
    if (q.tiles.find(items) == q.tiles.end()) return false;
    return !staged || q.runs.find(items) != q.runs.end();
  };
  if (p.plan.panels > 1) {
    auto it = p.panel_sets.find(p.plan.panels);
    if (it == p.panel_sets.end()) return p.n_rows == 0 || p.nnz == 0;
    for (auto &q : it->second)
      if (!ready(*q)) return false;
    return true;
  }
  return ready(p);
}

PanelSetDev panel_set_dev(spmv_handle_s *h, Part &p, int K) {
  PanelSetDev S{};
  S.n_rows = p.n_rows;
  if (K <= 1) {
    S.K = 1;
    S.rp[0] = p.row_ptr.as<const int32_t>();
    S.col[0] = p.col.as<const int32_t>();
    S.val[0] = p.val.p;
    return S;
  }
  auto &set = build_panels(h, p, K);
  S.K = int(set.size());
  for (int k = 0; k < S.K; ++k) {
    S.rp[k] = set[size_t(k)]->row_ptr.as<const int32_t>();
    S.col[k] = set[size_t(k)]->col.as<const int32_t>();
    S.val[k] = set[size_t(k)]->val.p;
  }
  return S;
}

int fused_rows_for(spmv_handle_s *h, Part &p, int K, int cap) {
  const auto key = std::make_pair(K, cap);
  auto it = p.fused_rows.find(key);
  if (it != p.fused_rows.end()) return it->second;
  std::vector<const std::vector<int32_t> *> rps;
  if (K > 1) {
    for (auto &q : build_panels(h, p, K)) rps.push_back(&q->h_row_ptr);
  } else {
    rps.push_back(&p.h_row_ptr);
  }
  const int64_t n = p.n_rows;
  int R = 512;
  for (; R > 16; R /= 2) {
    bool ok = true;
    for (const std::vector<int32_t> *rp : rps) {
      for (int64_t b = 0; b < n && ok; b += R) {
        const int64_t e = std::min<int64_t>(b + R, n);
        if (int64_t((*rp)[size_t(e)]) - (*rp)[size_t(b)] > cap) ok = false;
      }
      if (!ok) break;
    }
    if (ok) break;
  }
  p.fused_rows.emplace(key, R);
  return R;
}

bool part_runs_halves(const Part &p) {
  return p.cut_row > 0 && p.cut_row < p.n_rows &&
         (p.plan.kernel == SPMV_KERNEL_STREAM || p.plan.kernel == SPMV_KERNEL_STAGED ||
          p.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS);
}

void run_part_half(spmv_handle_s *h, Part &p, int half, const void *B, void *C, hipStream_t s) {
  if (p.n_rows == 0 || p.nnz == 0) return;
  if (p.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS) {
    // halves at block granularity: the blocks wholly above the cut row, and
    // the rest (the block that holds the cut row goes with the second half)
    SortedDev S = sorted_dev(h, p, p.plan.tile_items);
    const int64_t cb = std::min<int64_t>(S.n_blocks, p.cut_row / S.R);
    if (half == 0)
      S.b1 = cb;
    else
      S.b0 = cb;
    hip_ok(launch_spmv_sorted(h->prec, S, p.plan.tile_items, p.plan.nontemporal, p.plan.xcd_remap,
                              B, C, s),
           "kernel launch");
    return;
  }
  const bool staged = p.plan.kernel == SPMV_KERNEL_STAGED;
  const int xb = vec_bytes(h->prec);
  const int items = p.plan.tile_items;
  spmv_plan_t sub = p.plan;
  sub.panels = 1;
  const PlanDev pl = to_dev(sub);
  auto one = [&](Part &q) {
    if (q.nnz == 0) return;
    auto t = q.tiles_for(items);
    const int32_t *r = staged ? q.runs_for(items, xb) : nullptr;
    const int64_t tc = q.cut_tile.at(items);
    const int64_t t0 = half == 0 ? 0 : tc, t1 = half == 0 ? tc : t.second;
    if (t1 <= t0) return;
    hip_ok(launch_spmv(h->prec, q.dev(), pl, t.first + t0, r ? r + t0 * RUN_WORDS : nullptr,
                       t1 - t0, B, C, s),
           "kernel launch");
  };
  if (p.plan.panels > 1) {
    for (auto &q : build_panels(h, p, p.plan.panels)) one(*q);
  } else {
    one(p);
  }
}

void run_part(spmv_handle_s *h, Part &p, const void *B, void *C, hipStream_t s) {
  if (p.n_rows == 0 || p.nnz == 0) return;
  if (p.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS) {
    const SortedDev S = sorted_dev(h, p, p.plan.tile_items);
    hip_ok(launch_spmv_sorted(h->prec, S, p.plan.tile_items, p.plan.nontemporal, p.plan.xcd_remap,
                              B, C, s),
           "kernel launch");
    return;
  }
  if (p.plan.kernel == SPMV_KERNEL_FUSED_PANELS) {
    const PanelSetDev S = panel_set_dev(h, p, p.plan.panels);
    const int R = fused_rows_for(h, p, p.plan.panels, kWG * p.plan.tile_items - 4);
    hip_ok(launch_spmv_fused(h->prec, S, R, p.plan.tile_items, p.plan.nontemporal,
                             p.plan.xcd_remap, B, C, s),
           "kernel launch");
    return;
  }
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

// Diagonal-panel candidates (parts that cover all rows only): the panels
// applied one launch each, and walked by the fused-panel kernel.
std::vector<spmv_plan_t> panel_candidates() {
  std::vector<spmv_plan_t> c;
  for (int k : {1, 2, 4, 8})
    for (int e : {8, 16})
      for (int rm : {1, 0}) {
        spmv_plan_t p = default_plan();
        p.kernel = SPMV_KERNEL_FUSED_PANELS;
        p.panels = k;
        p.tile_items = e;
        p.xcd_remap = rm;
        c.push_back(p);
      }
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

// The sorted-block layouts the part's plans use: (tile_items, 1) for the
// one-vector plan, (tile_items, block_kt) for block plans of that kernel.
std::vector<std::pair<int, int>> sorted_keys(spmv_handle_s *h, const Part &p) {
  std::vector<std::pair<int, int>> keep;
  if (p.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS) {
    keep.emplace_back(p.plan.tile_items, 1);
    if (p.plan.block_kt != 0) keep.emplace_back(p.plan.tile_items, p.plan.block_kt);
  }
  if (&p == &h->main)
    for (auto &bp : h->block_plans)
      if (bp.second.kernel == SPMV_KERNEL_SORTED_BLOCKS)
        keep.emplace_back(bp.second.tile_items, bp.second.block_kt);
  return keep;
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
    // sorted blocks: one 1024-thread workgroup per block, so only for parts
    // of at least one block per two CUs
    const int R = sorted_block_rows(h->prec);
    int n_cu = 256;
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device);
    if (R > 0 && 2 * p.n_rows >= int64_t(R) * std::max(n_cu, 1))
      for (int e : {1, 2, 4}) {
        spmv_plan_t c = default_plan();
        c.kernel = SPMV_KERNEL_SORTED_BLOCKS;
        c.tile_items = e;
        cands.push_back(c);
      }
  }
  std::vector<spmv_plan_t> ran;
  std::vector<float> times;
  for (const spmv_plan_t &c : cands) {
    p.plan = c;
    try {
      prepare_part(h, p);
    } catch (const Failure &f) {
      // a part whose rows are too long for the sorted-block layout
      if (c.kernel == SPMV_KERNEL_SORTED_BLOCKS && f.status == SPMV_ERR_UNSUPPORTED) continue;
      throw;
    }
    ran.push_back(c);
    times.push_back(tm.median_ms([&] { run_part(h, p, x, y, s); }, s));
    best = std::min(best, times.back());
  }
  // the earliest candidate within 1% of the fastest: near-ties resolve the
  // same way from run to run
  for (size_t i = 0; i < ran.size(); ++i)
    if (times[i] <= best * 1.01f) {
      best_p = ran[i];
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
  prune_sorted(p, sorted_keys(h, p));
  if (std::getenv("SPMV_LOG"))
    std::fprintf(stderr, "libspmv: tuned %s part: kernel=%d tile_items=%d lanes=%d nt=%d remap=%d "
                         "(%.1f us)\n",
                 name, p.plan.kernel, p.plan.tile_items, p.plan.lanes, p.plan.nontemporal,
                 p.plan.xcd_remap, best * 1000.0f);
  if (!(h->flags & SPMV_FLAG_NO_TUNE_CACHE))
    cache_store(tune_key(h->device, h->prec, 1, name, p.n_rows, p.stats), p.plan);
}

}  // namespace

}  // namespace rt
}  // namespace spmv

using namespace spmv::rt;

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
    if (plan->kernel == SPMV_KERNEL_FUSED_PANELS && (p.row_ids.p || h->kind == SPMV_KIND_BATCH ||
                                                     h->kind == SPMV_KIND_SYMMETRIC))
      fail(SPMV_ERR_UNSUPPORTED, "the fused-panel kernel needs a part that covers all rows");
    if (plan->kernel == SPMV_KERNEL_SORTED_BLOCKS && (p.row_ids.p || h->kind == SPMV_KIND_BATCH ||
                                                      h->kind == SPMV_KIND_SYMMETRIC))
      fail(SPMV_ERR_UNSUPPORTED, "the sorted-block kernel needs a part that covers all rows");
    DeviceGuard dg(h->device);
    const spmv_plan_t before = p.plan;
    p.plan = *plan;
    try {
      if (h->kind == SPMV_KIND_BATCH)
        batch_prepare(h);
      else if (h->kind != SPMV_KIND_SYMMETRIC)
        prepare_part(h, p);
    } catch (...) {
      p.plan = before;  // a plan that cannot be prepared (a refused layout) is not kept
      throw;
    }
    if (h->kind == SPMV_KIND_SPLIT && &p == &h->main) {
      // the merged layout of SPMV_SCHEDULE_OVERLAP_MERGED follows the local plan
      const bool sorted = plan->kernel == SPMV_KERNEL_SORTED_BLOCKS;
      prune_merged(h, sorted ? plan->tile_items : 0);
      if (sorted && h->schedule == SPMV_SCHEDULE_OVERLAP_MERGED && p.n_rows > 0 && p.nnz > 0)
        (void)merged_tail_for(h, plan->tile_items);
    }
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
      if (h->kind == SPMV_KIND_SPLIT) {
        tune_part(h, h->nl, "nonlocal", x.p, y.p, s, tm);
        const bool sorted = h->main.plan.kernel == SPMV_KERNEL_SORTED_BLOCKS;
        if (!sorted) prune_merged(h, 0);
        if (!h->schedule_set && part_runs_halves(h->main) && h->nl.nnz > 0) {
          // the ordered schedule, the nonlocal part beside the local part,
          // or (sorted-block local plans) the last blocks over local and
          // nonlocal entries together, whichever runs fastest with the
          // plans just chosen, the halo copied in from a pinned buffer of
          // the tuner's own (a schedule that waits for the halo longer
          // shows it); another than the ordered one must win by 1%
          const int64_t n_halo = h->n_cols - h->halo_begin;
          const size_t hb = size_t(std::max<int64_t>(n_halo, 1)) * size_t(vec_bytes(h->prec));
          void *pin = nullptr;
          hip_ok(hipHostMalloc(&pin, hb, hipHostMallocDefault), "pinned tune halo");
          struct PinFree {
            void *p;
            ~PinFree() { (void)hipHostFree(p); }
          } pin_free{pin};
          std::memset(pin, 0, hb);
          struct Restore {  // the caller's schedule again if a trial fails
            spmv_handle_s *h;
            int saved;
            bool done;
            ~Restore() {
              if (!done) h->schedule = saved;
            }
          } restore{h, h->schedule, false};
          auto timed = [&](int schedule) {
            h->schedule = schedule;
            return tm.median_ms([&] { split_run(h, x.p, y.p, n_halo > 0 ? pin : nullptr, s); }, s);
          };
          const float ordered = timed(SPMV_SCHEDULE_OVERLAP);
          float best = 0.99f * ordered;
          int chosen = SPMV_SCHEDULE_OVERLAP;
          std::vector<int> others{SPMV_SCHEDULE_OVERLAP_NONLOCAL};
          if (sorted && merged_tail_for(h, h->main.plan.tile_items))
            others.push_back(SPMV_SCHEDULE_OVERLAP_MERGED);
          for (int sc : others) {
            const float t = timed(sc);
            if (t < best) {
              best = t;
              chosen = sc;
            }
          }
          h->schedule = chosen;
          restore.done = true;
          if (chosen != SPMV_SCHEDULE_OVERLAP_MERGED) prune_merged(h, 0);
        }
        if (sorted) prune_merged(h, h->main.plan.tile_items);
      }
      return;
    }
    if (h->kind != SPMV_KIND_PLAIN) fail(SPMV_ERR_UNSUPPORTED, "block tuning needs a plain handle");
    Part &p = h->main;
    float best = 1e30f;
    int best_kt = default_kt(k), best_nt = p.plan.nontemporal, best_pn = 1;
    int best_rm = p.plan.xcd_remap;
    // remap 0 spreads every row range over all eight XCDs, so the XCDs
    // gather from one shared window of B, which the MALL can hold where a
    // window per XCD would not (wide blocks)
    bool best_fused = false;
    for (int fused : {0, 1})
      for (int rm : {p.plan.xcd_remap, 1 - p.plan.xcd_remap})
        for (int pn : {1, 2, 4, 8})
          for (int kt : {4, 8, 16}) {
            if (kt > 2 * k && kt != 4) continue;
            for (int nt : {1, 0}) {
              const float ms = tm.median_ms(
                  [&] {
                    run_block_part(h, p, kt, nt, rm, pn, k, x.p, k, y.p, k, s, 1.0, fused != 0);
                  },
                  s);
              if (ms < best * 0.99f) {
                best = ms;
                best_kt = kt;
                best_nt = nt;
                best_pn = pn;
                best_rm = rm;
                best_fused = fused != 0;
              }
            }
          }
    // the sorted-block kernel for blocks, for parts of at least half a round
    // of its blocks (R * kt sums per block), its layout built when tried;
    // 4 or 8 columns per pass: with 16 its chunks of distinct rows shrink
    // and it has not been competitive
    int best_sorted = 0;
    {
      int n_cu = 256;
      (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device);
      for (int kt : {4, 8}) {
        if (kt > 2 * k && kt != 4) continue;
        const int R = sorted_block_rows(h->prec) / kt;
        if (R <= 0 || 2 * p.n_rows < int64_t(R) * std::max(n_cu, 1)) continue;
        for (int e : {2, 4}) {
          try {
            (void)sorted_for(h, p, e, kt);
          } catch (const Failure &f) {
            if (f.status == SPMV_ERR_UNSUPPORTED) continue;  // rows too long
            throw;
          }
          // remap 0 lets the XCDs share one window of B in the MALL, as
          // for the fused walk; the layout is the same either way
          for (int rm : {1, 0}) {
            const float ms = tm.median_ms(
                [&] { run_block_part(h, p, kt, 1, rm, 1, k, x.p, k, y.p, k, s, 1.0, false, e); },
                s);
            if (ms < best * 0.99f) {
              best = ms;
              best_kt = kt;
              best_nt = 1;
              best_pn = 1;
              best_rm = rm;
              best_fused = false;
              best_sorted = e;
            }
          }
        }
      }
    }
    spmv_plan_t c = p.plan;
    c.block_kt = best_kt;
    c.nontemporal = best_nt;
    c.panels = best_pn;
    c.xcd_remap = best_rm;
    c.kernel = best_sorted    ? SPMV_KERNEL_SORTED_BLOCKS
               : best_fused ? SPMV_KERNEL_FUSED_PANELS
                            : SPMV_KERNEL_STREAM;
    if (best_sorted) c.tile_items = best_sorted;
    h->block_plans[k] = c;
    std::vector<int> keep{p.plan.panels};
    for (auto &bp : h->block_plans) keep.push_back(bp.second.panels);
    prune_panels(p, keep);
    prune_sorted(p, sorted_keys(h, p));
    if (std::getenv("SPMV_LOG"))
      std::fprintf(stderr,
                   "libspmv: tuned block k=%d: kt=%d nt=%d panels=%d remap=%d fused=%d sorted=%d "
                   "(%.1f us)\n",
                   k, best_kt, best_nt, best_pn, best_rm, int(best_fused), best_sorted,
                   best * 1000.0f);
    if (!(h->flags & SPMV_FLAG_NO_TUNE_CACHE))
      cache_store(tune_key(h->device, h->prec, k, "block", p.n_rows, p.stats), c);
  });
}
