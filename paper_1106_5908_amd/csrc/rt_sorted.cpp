// libspmv runtime, sorted-block layout (SPMV_KERNEL_SORTED_BLOCKS): the
// part's rows are cut into blocks whose entries are re-ordered by column and
// dealt into chunks in which no row appears twice (see k_sorted).  Built on
// the host from one copy of col_idx and val read back from the device; the
// product is the one of Listing 1, summed per row in chunk order.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "runtime.h"
#include "sorted_place.h"

namespace spmv {
namespace rt {

namespace {

// Rows per block for a part of n rows.  One workgroup per CU at a time.  A
// part of at least three quarters of a round (rmax rows on every CU) gets
// blocks sized to come in whole rounds of one per CU, the fewest rounds
// blocks of at most rmax rows allow, so that no CU idles in the last round;
// a smaller part gets blocks of rmax rows.
int cu_count(spmv_handle_s *h) {
  int n_cu = 256;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess ||
      n_cu < 1)
    n_cu = 256;
  return n_cu;
}

int block_rows(spmv_handle_s *h, int64_t n, int rmax) {
  const int n_cu = cu_count(h);
  const int64_t full = int64_t(rmax) * n_cu;
  if (4 * n < 3 * full) return rmax;
  const int64_t rounds = (n + full - 1) / full;
  return int(std::min<int64_t>(rmax, (n + rounds * n_cu - 1) / (rounds * n_cu)));
}

// A block needs at least max(ceil(m / Q), longest row) chunks: a row of many
// entries makes the layout mostly empty slots.  Such layouts are refused:
// the slots may not exceed four per entry, plus one chunk per block, plus
// 2^20.  rp: row pointers of rows [b_first * R, n), relative to that row.
void check_slots(const int32_t *rp, int64_t n, int R, int Q, int64_t b_first) {
  const int64_t nb = (n + R - 1) / R, base = b_first * R;
  int64_t bound = 0;
  for (int64_t b = b_first; b < nb; ++b) {
    const int64_t r0 = b * R - base, r1 = std::min<int64_t>(n, b * R + R) - base;
    int64_t longest = 0;
    for (int64_t r = r0; r < r1; ++r) longest = std::max<int64_t>(longest, rp[r + 1] - rp[r]);
    bound += std::max<int64_t>((int64_t(rp[r1]) - rp[r0] + Q - 1) / Q, longest) * Q;
  }
  const int64_t m = rp[n - base];
  if (bound > 4 * m + (nb - b_first) * int64_t(Q) + (int64_t(1) << 20))
    fail(SPMV_ERR_UNSUPPORTED, "rows too long for the sorted-block kernel: " + std::to_string(bound) +
                                   " slots for " + std::to_string(m) + " entries");
}

// The layout of blocks [b_first, nb) of a part of n rows in blocks of R
// rows, from host arrays of rows [b_first * R, n): rp (relative to that
// row), col and val (vb bytes an entry).  period 0: the widest block span.
SortedSet build_layout(const int32_t *rp, const int32_t *hc, const unsigned char *hv, int vb,
                       int64_t n, int R, int Q, int64_t b_first, int64_t period) {
  const int64_t nb = (n + R - 1) / R, base = b_first * R, nbl = nb - b_first;
  // block b's rows, relative to the first row of the arrays
  auto rows = [&](int64_t b, int64_t &r0, int64_t &r1) {
    r0 = b * R - base;
    r1 = std::min<int64_t>(n, b * R + R) - base;
  };
  if (period == 0) {
    // the sweeps' common period: the widest column range of a block
    std::vector<int64_t> span(static_cast<size_t>(nbl), 0);
    parallel_for(
        nbl,
        [&](int64_t b0, int64_t b1) {
          for (int64_t i = b0; i < b1; ++i) {
            int64_t r0, r1;
            rows(b_first + i, r0, r1);
            int32_t lo = INT32_MAX, hi = -1;
            for (int64_t j = rp[r0]; j < rp[r1]; ++j) {
              lo = std::min(lo, hc[size_t(j)]);
              hi = std::max(hi, hc[size_t(j)]);
            }
            span[size_t(i)] = rp[r1] > rp[r0] ? int64_t(hi) - lo + 1 : 0;
          }
        },
        2);
    period = span.empty() ? 0 : *std::max_element(span.begin(), span.end());
  }
  auto local_rows = [&](int64_t r0, int64_t r1, std::vector<int32_t> &lrow) {
    lrow.resize(size_t(rp[r1] - rp[r0]));
    for (int64_t r = r0; r < r1; ++r)
      for (int64_t j = rp[r]; j < rp[r + 1]; ++j) lrow[size_t(j - rp[r0])] = int32_t(r - r0);
  };
  std::vector<std::vector<int32_t>> placed(static_cast<size_t>(nbl));
  parallel_for(
      nbl,
      [&](int64_t b0, int64_t b1) {
        std::vector<int32_t> lrow, len(static_cast<size_t>(R));
        for (int64_t i = b0; i < b1; ++i) {
          int64_t r0, r1;
          rows(b_first + i, r0, r1);
          local_rows(r0, r1, lrow);
          std::fill(len.begin(), len.end(), 0);
          for (int64_t r = r0; r < r1; ++r) len[size_t(r - r0)] = rp[r + 1] - rp[r];
          placed[size_t(i)] = sorted_place_block(hc + rp[r0], lrow.data(), len.data(),
                                                 rp[r1] - rp[r0], R, Q, period);
        }
      },
      2);
  std::vector<int64_t> cs(static_cast<size_t>(nb + 1), 0);
  for (int64_t b = b_first; b < nb; ++b)
    cs[size_t(b + 1)] = cs[size_t(b)] + int64_t(placed[size_t(b - b_first)].size()) / Q;
  const int64_t n_slots = cs[size_t(nb)] * Q;
  if (n_slots > (int64_t(1) << 40)) fail(SPMV_ERR_UNSUPPORTED, "sorted-block layout too large");
  std::vector<int32_t> oc(size_t(std::max<int64_t>(n_slots, 1)));
  std::vector<unsigned char> ov(size_t(std::max<int64_t>(n_slots, 1)) * size_t(vb), 0);
  std::vector<uint16_t> orow(size_t(std::max<int64_t>(n_slots, 1)));
  parallel_for(
      nbl,
      [&](int64_t b0, int64_t b1) {
        std::vector<int32_t> lrow;
        for (int64_t i = b0; i < b1; ++i) {
          int64_t r0, r1;
          rows(b_first + i, r0, r1);
          local_rows(r0, r1, lrow);
          const int64_t p0 = rp[r0];
          const std::vector<int32_t> &sl = placed[size_t(i)];
          const size_t at = size_t(cs[size_t(b_first + i)] * Q);
          for (size_t c = 0; c * size_t(Q) < sl.size(); ++c) {
            // an empty slot gathers a column its chunk already reads
            const int32_t first = sl[c * size_t(Q)];
            const int32_t pad_col = first >= 0 ? hc[size_t(p0 + first)] : 0;
            for (size_t q = c * size_t(Q); q < (c + 1) * size_t(Q); ++q) {
              const int32_t e = sl[q];
              if (e >= 0) {
                const size_t j = size_t(p0 + e);
                oc[at + q] = hc[j];
                std::memcpy(&ov[(at + q) * size_t(vb)], &hv[j * size_t(vb)], size_t(vb));
                orow[at + q] = uint16_t(lrow[size_t(e)]);
              } else {
                oc[at + q] = pad_col;
                orow[at + q] = SB_PAD_ROW;  // val stays zero
              }
            }
          }
        }
      },
      2);
  SortedSet S;
  S.R = R;
  S.Q = Q;
  S.n_blocks = nb;
  S.n_chunks = cs[size_t(nb)];
  S.period = period;
  S.b_first = b_first;
  upload(S.cs, cs.data(), cs.size() * 8, "sorted-block chunk starts");
  if (n_slots > 0) {
    upload(S.col, oc.data(), size_t(n_slots) * 4, "sorted-block col_idx");
    upload(S.val, ov.data(), size_t(n_slots) * size_t(vb), "sorted-block val");
    upload(S.row, orow.data(), size_t(n_slots) * 2, "sorted-block rows");
  }
  return S;
}

int checked_rmax(spmv_handle_s *h) {
  const int rmax = sorted_block_rows(h->prec);
  if (rmax <= 0 || rmax > int(SB_PAD_ROW)) fail(SPMV_ERR_UNSUPPORTED, "no sorted-block layout for this precision");
  return rmax;
}

}  // namespace

const SortedSet &sorted_for(spmv_handle_s *h, Part &p, int items, int kt) {
  const std::pair<int, int> key(items, kt);
  auto it = p.sorted.find(key);
  if (it != p.sorted.end()) return it->second;
  if (p.row_ids.p) fail(SPMV_ERR_UNSUPPORTED, "the sorted-block kernel needs a part that covers all rows");
  if (kt != 1 && kt != 4 && kt != 8 && kt != 16)
    fail(SPMV_ERR_INVALID_ARG, "sorted-block layouts take 1, 4, 8 or 16 columns per pass");
  const int R = block_rows(h, p.n_rows, checked_rmax(h) / kt);
  const int Q = sorted_chunk_slots(h->prec, kt, items);
  const int vb = val_bytes(h->prec);
  const int64_t n = p.n_rows, nnz = p.nnz;
  check_slots(p.h_row_ptr.data(), n, R, Q, 0);
  std::vector<int32_t> hc(size_t(std::max<int64_t>(nnz, 1)));
  std::vector<unsigned char> hv(size_t(std::max<int64_t>(nnz, 1)) * size_t(vb));
  if (nnz > 0) {
    hip_ok(hipMemcpy(hc.data(), p.col.p, size_t(nnz) * 4, hipMemcpyDeviceToHost), "col readback");
    hip_ok(hipMemcpy(hv.data(), p.val.p, size_t(nnz) * size_t(vb), hipMemcpyDeviceToHost),
           "val readback");
  }
  SortedSet S = build_layout(p.h_row_ptr.data(), hc.data(), hv.data(), vb, n, R, Q, 0, 0);
  return p.sorted.emplace(key, std::move(S)).first->second;
}

const SortedSet *merged_tail_for(spmv_handle_s *h, int items) {
  auto it = h->merged.find(items);
  if (it == h->merged.end()) {
    Part &L = h->main, &N = h->nl;
    if (h->kind != SPMV_KIND_SPLIT || L.cut_row < 0 || N.n_rows == 0 || N.nnz == 0) return nullptr;
    const SortedSet &S = sorted_for(h, L, items);
    const int R = S.R, Q = S.Q, vb = val_bytes(h->prec);
    const int64_t n_cu = cu_count(h), first = L.cut_row / R;
    // from the last whole round of blocks above the first nonlocal row
    const int64_t n = L.n_rows;
    const int64_t cb = first >= n_cu ? first / n_cu * n_cu : first, base = cb * R;
    const int32_t *lrp = L.h_row_ptr.data();
    // rows [base, n): their local entries, then their nonlocal ones
    std::vector<int32_t> nl_rows(size_t(N.n_rows));
    hip_ok(hipMemcpy(nl_rows.data(), N.row_ids.p, size_t(N.n_rows) * 4, hipMemcpyDeviceToHost),
           "nonlocal rows readback");
    const int64_t m_loc = int64_t(lrp[n]) - lrp[base], m = m_loc + N.nnz;
    const int32_t *nrp = N.h_row_ptr.data();
    std::vector<int32_t> rp;
    if (!merged_row_ptr(lrp, base, n, nl_rows.data(), nrp, N.n_rows, rp))
      fail(SPMV_ERR_STATE, "nonlocal row outside the local part's tail");
    SortedSet T;
    bool refused = false;
    try {
      check_slots(rp.data(), n, R, Q, cb);
    } catch (const Failure &e) {
      if (e.status != SPMV_ERR_UNSUPPORTED) throw;
      refused = true;
    }
    if (!refused) {
      std::vector<int32_t> lc(size_t(std::max<int64_t>(m_loc, 1))), nc(size_t(std::max<int64_t>(N.nnz, 1)));
      std::vector<unsigned char> lv(lc.size() * size_t(vb)), nv(nc.size() * size_t(vb));
      if (m_loc > 0) {
        hip_ok(hipMemcpy(lc.data(), L.col.as<int32_t>() + lrp[base], size_t(m_loc) * 4,
                         hipMemcpyDeviceToHost),
               "col readback");
        hip_ok(hipMemcpy(lv.data(), static_cast<const char *>(L.val.p) + size_t(lrp[base]) * vb,
                         size_t(m_loc) * size_t(vb), hipMemcpyDeviceToHost),
               "val readback");
      }
      hip_ok(hipMemcpy(nc.data(), N.col.p, size_t(N.nnz) * 4, hipMemcpyDeviceToHost),
             "nonlocal col readback");
      hip_ok(hipMemcpy(nv.data(), N.val.p, size_t(N.nnz) * size_t(vb), hipMemcpyDeviceToHost),
             "nonlocal val readback");
      std::vector<int32_t> hc(size_t(std::max<int64_t>(m, 1)));
      std::vector<unsigned char> hv(hc.size() * size_t(vb));
      merged_entries(lrp, base, n, lc.data(), lv.data(), nl_rows.data(), nrp, N.n_rows, nc.data(),
                     nv.data(), vb, rp, hc.data(), hv.data());
      T = build_layout(rp.data(), hc.data(), hv.data(), vb, n, R, Q, cb, S.period);
      T.after_rounds = first >= n_cu;
    }
    it = h->merged.emplace(items, std::move(T)).first;
  }
  return it->second.n_blocks > 0 ? &it->second : nullptr;
}

void prune_merged(spmv_handle_s *h, int keep_items) {
  for (auto it = h->merged.begin(); it != h->merged.end();) {
    if (it->first != keep_items)
      it = h->merged.erase(it);
    else
      ++it;
  }
}

SortedDev sorted_dev(spmv_handle_s *h, Part &p, int items, int kt) {
  const SortedSet &S = sorted_for(h, p, items, kt);
  SortedDev d;
  d.cs = S.cs.as<const int64_t>();
  d.col = S.col.as<const int32_t>();
  d.val = S.val.p;
  d.row = S.row.as<const uint16_t>();
  d.n_rows = p.n_rows;
  d.n_blocks = S.n_blocks;
  d.R = S.R;
  d.q = S.Q;
  d.b0 = 0;
  d.b1 = S.n_blocks;
  return d;
}

void prune_sorted(Part &p, const std::vector<std::pair<int, int>> &keep) {
  for (auto it = p.sorted.begin(); it != p.sorted.end();) {
    if (std::find(keep.begin(), keep.end(), it->first) == keep.end())
      it = p.sorted.erase(it);
    else
      ++it;
  }
}

}  // namespace rt
}  // namespace spmv
