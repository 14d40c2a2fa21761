"""Rows of a split part merged for the merged-tail schedule
(csrc/sorted_place.h: merged_row_ptr, merged_entries), built on their own
with g++ and checked on the host: the local and nonlocal parts of a random
CRS, split by the oracle at a halo column (Sect. 3.4), merged from a base
row on give back every row's entries of the unsplit matrix, its local ones
first in their order, then its nonlocal ones; a nonlocal row above the base
row is reported.  Runs without a GPU."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from workloads import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1106_5908_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <vector>
#include "sorted_place.h"
template <class T> static bool rd(FILE *f, std::vector<T> &v, size_t n) {
  v.resize(n + 1);
  return n == 0 || std::fread(v.data(), sizeof(T), n, f) == n;
}
int main(int argc, char **argv) {
  FILE *f = std::fopen(argv[1], "rb");
  int64_t hdr[4];
  if (std::fread(hdr, 8, 4, f) != 4) return 2;
  const int64_t n = hdr[0], base = hdr[1], n_nl = hdr[2], m_nl = hdr[3];
  std::vector<int32_t> lrp, lc, nl_rows, nrp, nc;
  std::vector<double> lv, nv;
  if (!rd(f, lrp, size_t(n + 1))) return 3;
  const size_t m_loc = size_t(lrp[size_t(n)] - lrp[size_t(base)]);
  if (!rd(f, lc, m_loc) || !rd(f, lv, m_loc) || !rd(f, nl_rows, size_t(n_nl)) ||
      !rd(f, nrp, size_t(n_nl + 1)) || !rd(f, nc, size_t(m_nl)) || !rd(f, nv, size_t(m_nl)))
    return 4;
  std::fclose(f);
  std::vector<int32_t> rp;
  FILE *o = std::fopen(argv[2], "wb");
  const bool ok = spmv::rt::merged_row_ptr(lrp.data(), base, n, nl_rows.data(), nrp.data(), n_nl, rp);
  int64_t flag = ok ? 1 : 0;
  std::fwrite(&flag, 8, 1, o);
  if (ok) {
    const size_t m = size_t(rp.back());
    std::vector<int32_t> hc(m + 1);
    std::vector<double> hv(m + 1);
    spmv::rt::merged_entries(lrp.data(), base, n, lc.data(),
                             reinterpret_cast<const unsigned char *>(lv.data()), nl_rows.data(),
                             nrp.data(), n_nl, nc.data(),
                             reinterpret_cast<const unsigned char *>(nv.data()), 8, rp, hc.data(),
                             reinterpret_cast<unsigned char *>(hv.data()));
    std::fwrite(rp.data(), 4, rp.size(), o);
    if (m) {
      std::fwrite(hc.data(), 4, m, o);
      std::fwrite(hv.data(), 8, m, o);
    }
  }
  std::fclose(o);
  return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ missing")
    d = tmp_path_factory.mktemp("merge")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    exe = d / "h"
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-I", CSRC, str(src), "-o", str(exe)])
    return d, exe


def _merge(harness, parts, n, base):
    d, exe = harness
    lrp = parts["loc_row_ptr"].astype(np.int32)
    p0 = int(lrp[base])
    inp, out = d / "in.bin", d / "out.bin"
    with open(inp, "wb") as f:
        np.array([n, base, parts["nl_rows"].size, parts["nl_col"].size], dtype=np.int64).tofile(f)
        lrp.tofile(f)
        parts["loc_col"][p0:].astype(np.int32).tofile(f)
        parts["loc_val"][p0:].astype(np.float64).tofile(f)
        parts["nl_rows"].astype(np.int32).tofile(f)
        parts["nl_ptr"].astype(np.int32).tofile(f)
        parts["nl_col"].astype(np.int32).tofile(f)
        parts["nl_val"].astype(np.float64).tofile(f)
    subprocess.check_call([str(exe), str(inp), str(out)])
    with open(out, "rb") as f:
        if int(np.fromfile(f, dtype=np.int64, count=1)[0]) == 0:
            return None
        rp = np.fromfile(f, dtype=np.int32, count=n - base + 1)
        m = int(rp[-1])
        return rp, np.fromfile(f, dtype=np.int32, count=m), np.fromfile(f, dtype=np.float64, count=m)


@pytest.mark.parametrize("halo", [0.5, 0.94, 0.999])
def test_merged_rows_match_the_unsplit_rows(harness, halo):
    rng = gen.rng_for(31, int(halo * 1000))
    n = 3000
    A = gen.random_crs(n, n, rng, max_len=25)
    hb = int(halo * n)
    parts = oracle.split(A.row_ptr, A.col_idx, A.val, hb)
    first = int(parts["nl_rows"][0]) if parts["nl_rows"].size else n
    for base in sorted({0, min(first, n - 1), max(first - 37, 0)}):
        got = _merge(harness, parts, n, base)
        assert got is not None
        rp, hc, hv = got
        for r in range(base, n):
            a, b = int(A.row_ptr[r]), int(A.row_ptr[r + 1])
            cols, vals = A.col_idx[a:b], A.val[a:b]
            loc = cols < hb
            want = np.concatenate([cols[loc], cols[~loc]]), np.concatenate([vals[loc], vals[~loc]])
            s, e = int(rp[r - base]), int(rp[r - base + 1])
            assert np.array_equal(hc[s:e], want[0]), r
            assert np.array_equal(hv[s:e], want[1]), r


def test_nonlocal_row_above_the_base_is_reported(harness):
    A, _ = gen.workload_c3(N=4000)  # banded: the first rows have no halo entry
    n = A.n_rows
    parts = oracle.split(A.row_ptr, A.col_idx, A.val, gen.halo_begin(A.n_cols))
    first = int(parts["nl_rows"][0])
    assert first > 0
    assert _merge(harness, parts, n, first + 1) is None
    assert _merge(harness, parts, n, first) is not None
