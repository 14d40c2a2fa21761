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

const SortedSet &sorted_for(spmv_handle_s *h, Part &p, int items) {
  auto it = p.sorted.find(items);
  if (it != p.sorted.end()) return it->second;
  if (p.row_ids.p) fail(SPMV_ERR_UNSUPPORTED, "the sorted-block kernel needs a part that covers all rows");
  const int rmax = sorted_block_rows(h->prec);
  const int Q = SB_WG * items;
  if (rmax <= 0 || rmax > int(SB_PAD_ROW)) fail(SPMV_ERR_UNSUPPORTED, "no sorted-block layout for this precision");
  const int vb = val_bytes(h->prec);
  const int64_t n = p.n_rows, nnz = p.nnz;
  // One workgroup per CU at a time.  A part of at least three quarters of
  // a round (rmax rows on every CU) gets blocks sized to come in whole
  // rounds of one per CU, the fewest rounds blocks of at most rmax rows
  // allow, so that no CU idles in the last round; a smaller part gets
  // blocks of rmax rows.
  int n_cu = 256;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess ||
      n_cu < 1)
    n_cu = 256;
  const int64_t full = int64_t(rmax) * n_cu;
  int R = rmax;
  if (4 * n >= 3 * full) {
    const int64_t rounds = (n + full - 1) / full;
    R = int(std::min<int64_t>(rmax, (n + rounds * n_cu - 1) / (rounds * n_cu)));
  }
  const int64_t nb = (n + R - 1) / R;
  const int32_t *rp = p.h_row_ptr.data();
  // A block needs at least max(ceil(m / Q), longest row) chunks: a row of
  // many entries makes the layout mostly empty slots.  Such parts are
  // refused: the slots may not exceed four per entry, plus one chunk per
  // block, plus 2^20.
  {
    int64_t bound = 0;
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t r0 = b * R, r1 = std::min<int64_t>(n, r0 + R);
      int64_t longest = 0;
      for (int64_t r = r0; r < r1; ++r) longest = std::max<int64_t>(longest, rp[r + 1] - rp[r]);
      bound += std::max<int64_t>((int64_t(rp[r1]) - rp[r0] + Q - 1) / Q, longest) * Q;
    }
    if (bound > 4 * nnz + nb * int64_t(Q) + (int64_t(1) << 20))
      fail(SPMV_ERR_UNSUPPORTED, "rows too long for the sorted-block kernel: " + std::to_string(bound) +
                                     " slots for " + std::to_string(nnz) + " entries");
  }
  std::vector<int32_t> hc(size_t(std::max<int64_t>(nnz, 1)));
  std::vector<unsigned char> hv(size_t(std::max<int64_t>(nnz, 1)) * size_t(vb));
  if (nnz > 0) {
    hip_ok(hipMemcpy(hc.data(), p.col.p, size_t(nnz) * 4, hipMemcpyDeviceToHost), "col readback");
    hip_ok(hipMemcpy(hv.data(), p.val.p, size_t(nnz) * size_t(vb), hipMemcpyDeviceToHost),
           "val readback");
  }
  // The sweeps' common period: the widest column range of a block.
  std::vector<int64_t> span(static_cast<size_t>(nb), 0);
  parallel_for(
      nb,
      [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
          const int64_t p0 = rp[b * R], p1 = rp[std::min<int64_t>(n, b * R + R)];
          int32_t lo = INT32_MAX, hi = -1;
          for (int64_t j = p0; j < p1; ++j) {
            lo = std::min(lo, hc[size_t(j)]);
            hi = std::max(hi, hc[size_t(j)]);
          }
          span[size_t(b)] = p1 > p0 ? int64_t(hi) - lo + 1 : 0;
        }
      },
      2);
  const int64_t period = span.empty() ? 0 : *std::max_element(span.begin(), span.end());
  std::vector<std::vector<int32_t>> placed(static_cast<size_t>(nb));
  parallel_for(
      nb,
      [&](int64_t b0, int64_t b1) {
        std::vector<int32_t> lrow, len(static_cast<size_t>(R));
        for (int64_t b = b0; b < b1; ++b) {
          const int64_t r0 = b * R, r1 = std::min<int64_t>(n, r0 + R);
          const int64_t p0 = rp[r0], p1 = rp[r1];
          lrow.resize(size_t(p1 - p0));
          std::fill(len.begin(), len.end(), 0);
          for (int64_t r = r0; r < r1; ++r) {
            len[size_t(r - r0)] = rp[r + 1] - rp[r];
            for (int64_t j = rp[r]; j < rp[r + 1]; ++j) lrow[size_t(j - p0)] = int32_t(r - r0);
          }
          placed[size_t(b)] =
              sorted_place_block(hc.data() + p0, lrow.data(), len.data(), p1 - p0, R, Q, period);
        }
      },
      2);
  std::vector<int64_t> cs(static_cast<size_t>(nb + 1), 0);
  for (int64_t b = 0; b < nb; ++b) cs[size_t(b + 1)] = cs[size_t(b)] + int64_t(placed[size_t(b)].size()) / Q;
  const int64_t n_slots = cs[size_t(nb)] * Q;
  if (n_slots > (int64_t(1) << 40)) fail(SPMV_ERR_UNSUPPORTED, "sorted-block layout too large");
  std::vector<int32_t> oc(size_t(std::max<int64_t>(n_slots, 1)));
  std::vector<unsigned char> ov(size_t(std::max<int64_t>(n_slots, 1)) * size_t(vb), 0);
  std::vector<uint16_t> orow(size_t(std::max<int64_t>(n_slots, 1)));
  parallel_for(
      nb,
      [&](int64_t b0, int64_t b1) {
        std::vector<int32_t> lrow;
        for (int64_t b = b0; b < b1; ++b) {
          const int64_t r0 = b * R, r1 = std::min<int64_t>(n, r0 + R);
          const int64_t p0 = rp[r0];
          lrow.resize(size_t(rp[r1] - p0));
          for (int64_t r = r0; r < r1; ++r)
            for (int64_t j = rp[r]; j < rp[r + 1]; ++j) lrow[size_t(j - p0)] = int32_t(r - r0);
          const std::vector<int32_t> &sl = placed[size_t(b)];
          const size_t base = size_t(cs[size_t(b)] * Q);
          for (size_t c = 0; c * size_t(Q) < sl.size(); ++c) {
            // an empty slot gathers a column its chunk already reads
            const int32_t first = sl[c * size_t(Q)];
            const int32_t pad_col = first >= 0 ? hc[size_t(p0 + first)] : 0;
            for (size_t q = c * size_t(Q); q < (c + 1) * size_t(Q); ++q) {
              const int32_t e = sl[q];
              if (e >= 0) {
                const size_t j = size_t(p0 + e);
                oc[base + q] = hc[j];
                std::memcpy(&ov[(base + q) * size_t(vb)], &hv[j * size_t(vb)], size_t(vb));
                orow[base + q] = uint16_t(lrow[size_t(e)]);
              } else {
                oc[base + q] = pad_col;
                orow[base + q] = SB_PAD_ROW;  // val stays zero
              }
            }
          }
        }
      },
      2);
  SortedSet S;
  S.R = R;
  S.n_blocks = nb;
  S.n_chunks = cs[size_t(nb)];
  upload(S.cs, cs.data(), cs.size() * 8, "sorted-block chunk starts");
  if (n_slots > 0) {
    upload(S.col, oc.data(), size_t(n_slots) * 4, "sorted-block col_idx");
    upload(S.val, ov.data(), size_t(n_slots) * size_t(vb), "sorted-block val");
    upload(S.row, orow.data(), size_t(n_slots) * 2, "sorted-block rows");
  }
  return p.sorted.emplace(items, std::move(S)).first->second;
}

SortedDev sorted_dev(spmv_handle_s *h, Part &p, int items) {
  const SortedSet &S = sorted_for(h, p, items);
  SortedDev d;
  d.cs = S.cs.as<const int64_t>();
  d.col = S.col.as<const int32_t>();
  d.val = S.val.p;
  d.row = S.row.as<const uint16_t>();
  d.n_rows = p.n_rows;
  d.n_blocks = S.n_blocks;
  d.R = S.R;
  d.b0 = 0;
  d.b1 = S.n_blocks;
  return d;
}

void prune_sorted(Part &p, int keep_items) {
  for (auto it = p.sorted.begin(); it != p.sorted.end();) {
    if (it->first != keep_items)
      it = p.sorted.erase(it);
    else
      ++it;
  }
}

}  // namespace rt
}  // namespace spmv
