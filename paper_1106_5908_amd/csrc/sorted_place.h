// Chunk placement of the sorted-block layout, and the rows its merged tail
// is built from (host code, no HIP): plain C++ so that it can be built and
// checked on its own.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

namespace spmv {
namespace rt {

// Bits of the per-block (chunk, row) membership table above which a block
// is dealt round-robin instead (rows of very many entries).
constexpr int64_t kMaxMembershipBits = int64_t(1) << 26;
// Chunks searched for a slot to free before a block gets one more chunk.
constexpr int64_t kSwapSearch = 64;

// Chunk assignment of one block of m entries (block-local indices 0..m-1,
// CRS order), `lrow[i]` the row of entry i within the block, `len[r]` the
// entries of row r.  Returns the slots of the block's chunks, chunk after
// chunk, Q per chunk: a block-local entry index, or -1 for an empty slot.
//
// N = max(ceil(m / Q), longest row) chunks.  The entries, in column order
// (rotated to start at a multiple of `period`, see below),
// go to the first chunk, searching cyclically from the chunk proportional to
// their rank, that has room and does not yet hold their row.  If every chunk
// with room holds the row, an entry of a full chunk without it moves to a
// chunk with room that lacks the moved entry's row; failing that the block
// gets one more chunk.  Each chunk's entries are then laid out in column
// order, so neighbouring lanes gather neighbouring columns.
inline std::vector<int32_t> sorted_place_block(const int32_t *col, const int32_t *lrow,
                                               const int32_t *len, int64_t m, int R, int Q,
                                               int64_t period = 0) {
  std::vector<int32_t> slots;
  if (m == 0) return slots;
  // entries by column, ties by position (a total order: the layout is the
  // same on every build)
  std::vector<int32_t> by_col(static_cast<size_t>(m));
  std::iota(by_col.begin(), by_col.end(), 0);
  std::sort(by_col.begin(), by_col.end(), [&](int32_t a, int32_t b) {
    return col[a] != col[b] ? col[a] < col[b] : a < b;
  });
  // With period > 0 the sweep starts at the first multiple of `period` above
  // the block's lowest column (when the block reaches that far) and wraps
  // round: blocks that run at the same time and cover that column then read
  // the same columns of B at the same time, and share them in L2.
  if (period > 0) {
    const int64_t lo = col[by_col[0]], hi = col[by_col[size_t(m - 1)]];
    const int64_t s0 = (lo + period - 1) / period * period;
    if (s0 > lo && s0 <= hi) {
      const auto it = std::lower_bound(by_col.begin(), by_col.end(), s0,
                                       [&](int32_t a, int64_t v) { return col[a] < v; });
      std::rotate(by_col.begin(), it, by_col.end());
    }
  }
  int64_t maxl = 0;
  for (int r = 0; r < R; ++r) maxl = std::max<int64_t>(maxl, len[r]);
  int64_t N = std::max<int64_t>((m + Q - 1) / Q, maxl);
  std::vector<std::vector<int32_t>> chunk;  // ranks (positions in by_col) per chunk
  if (N * int64_t(R) > kMaxMembershipBits) {
    // round-robin over the entries grouped by row: a row's entries are
    // consecutive and at most N, so they land in distinct chunks
    chunk.assign(size_t(N), {});
    std::vector<int32_t> rank(static_cast<size_t>(m)), by_row(static_cast<size_t>(m));
    for (int64_t k = 0; k < m; ++k) rank[size_t(by_col[size_t(k)])] = int32_t(k);
    std::iota(by_row.begin(), by_row.end(), 0);
    std::stable_sort(by_row.begin(), by_row.end(),
                     [&](int32_t a, int32_t b) { return lrow[a] < lrow[b]; });
    for (int64_t i = 0; i < m; ++i) chunk[size_t(i % N)].push_back(rank[size_t(by_row[size_t(i)])]);
  } else {
    chunk.assign(size_t(N), {});
    std::vector<uint64_t> bits(size_t((N * R + 63) / 64), 0);
    auto has = [&](int64_t c, int r) {
      const int64_t b = c * R + r;
      return (bits[size_t(b >> 6)] >> (b & 63)) & 1;
    };
    auto set = [&](int64_t c, int r, bool on) {
      const int64_t b = c * R + r;
      if (on)
        bits[size_t(b >> 6)] |= uint64_t(1) << (b & 63);
      else
        bits[size_t(b >> 6)] &= ~(uint64_t(1) << (b & 63));
    };
    for (int64_t k = 0; k < m; ++k) {
      const int r = lrow[by_col[size_t(k)]];
      const int64_t t = k * N / m;
      int64_t c = -1;
      for (int64_t i = 0; i < N && c < 0; ++i) {
        const int64_t cc = (t + i) % N;
        if (int64_t(chunk[size_t(cc)].size()) < Q && !has(cc, r)) c = cc;
      }
      for (int64_t i = 0; i < N && i < kSwapSearch && c < 0; ++i) {
        const int64_t c1 = (t + i) % N;
        if (has(c1, r)) continue;  // full (else it was taken above), lacks r
        auto &v1 = chunk[size_t(c1)];
        for (size_t j = 0; j < v1.size() && c < 0; ++j) {
          const int s = lrow[by_col[size_t(v1[j])]];
          for (int64_t c2 = 0; c2 < N; ++c2) {
            if (int64_t(chunk[size_t(c2)].size()) >= Q || has(c2, s)) continue;
            chunk[size_t(c2)].push_back(v1[j]);
            set(c2, s, true);
            set(c1, s, false);
            v1[j] = v1.back();
            v1.pop_back();
            c = c1;
            break;
          }
        }
      }
      if (c < 0) {
        c = N++;
        chunk.emplace_back();
        bits.resize(size_t((N * R + 63) / 64), 0);
      }
      chunk[size_t(c)].push_back(int32_t(k));
      set(c, r, true);
    }
  }
  int64_t used = 0;
  for (int64_t c = 0; c < N; ++c)
    if (!chunk[size_t(c)].empty()) used = c + 1;
  slots.assign(size_t(used * Q), -1);
  int64_t out = 0;
  for (int64_t c = 0; c < used; ++c) {
    auto &v = chunk[size_t(c)];
    std::sort(v.begin(), v.end());
    for (size_t j = 0; j < v.size(); ++j) slots[size_t(out + int64_t(j))] = by_col[size_t(v[j])];
    out += Q;
  }
  return slots;
}

// Rows [base, n) of a split part with each row's local and nonlocal entries
// (Sect. 3.4: a row's product is its local part's plus its nonlocal part's).
// lrp: the local part's n + 1 row pointers; nl_rows (ascending) and nrp
// (n_nl + 1 pointers): the nonlocal part's rows.  Fills rp with the merged
// rows' n - base + 1 pointers, relative to row base; false if a nonlocal row
// lies outside [base, n).
inline bool merged_row_ptr(const int32_t *lrp, int64_t base, int64_t n, const int32_t *nl_rows,
                           const int32_t *nrp, int64_t n_nl, std::vector<int32_t> &rp) {
  rp.assign(static_cast<size_t>(n - base + 1), 0);
  for (int64_t r = base; r < n; ++r) rp[size_t(r - base + 1)] = lrp[r + 1] - lrp[r];
  for (int64_t i = 0; i < n_nl; ++i) {
    const int64_t r = nl_rows[i];
    if (r < base || r >= n) return false;
    rp[size_t(r - base + 1)] += nrp[i + 1] - nrp[i];
  }
  for (size_t i = 1; i < rp.size(); ++i) rp[i] += rp[i - 1];
  return true;
}

// The merged rows' entries in the layout rp describes: each row's local
// entries (lc / lv: those of rows base.., lrp[base] first) in their order,
// then its nonlocal ones (nc / nv, in nrp order); vb bytes per value.
inline void merged_entries(const int32_t *lrp, int64_t base, int64_t n, const int32_t *lc,
                           const unsigned char *lv, const int32_t *nl_rows, const int32_t *nrp,
                           int64_t n_nl, const int32_t *nc, const unsigned char *nv, int vb,
                           const std::vector<int32_t> &rp, int32_t *hc, unsigned char *hv) {
  std::vector<int32_t> fill(rp.begin(), rp.end() - 1);
  for (int64_t r = base; r < n; ++r) {
    const size_t at = size_t(fill[size_t(r - base)]), k = size_t(lrp[r + 1] - lrp[r]);
    const size_t from = size_t(lrp[r] - lrp[base]);
    if (k) {
      std::memcpy(&hc[at], &lc[from], k * 4);
      std::memcpy(&hv[at * size_t(vb)], &lv[from * size_t(vb)], k * size_t(vb));
    }
    fill[size_t(r - base)] += int32_t(k);
  }
  for (int64_t i = 0; i < n_nl; ++i) {
    const int64_t r = nl_rows[i];
    const size_t at = size_t(fill[size_t(r - base)]), k = size_t(nrp[i + 1] - nrp[i]);
    if (k) {
      std::memcpy(&hc[at], &nc[size_t(nrp[i])], k * 4);
      std::memcpy(&hv[at * size_t(vb)], &nv[size_t(nrp[i]) * size_t(vb)], k * size_t(vb));
    }
    fill[size_t(r - base)] += int32_t(k);
  }
}

}  // namespace rt
}  // namespace spmv
