"""Chunk placement of the sorted-block layout (csrc/sorted_place.h), built
on its own with g++ and checked on the host: every entry of a block lands in
exactly one slot, no row appears twice in a chunk, each chunk's entries come
first and in column order (rotated to the sweep's start when a period is
given), and the chunk count stays at its lower bound max(ceil(m / Q),
longest row) up to a small slack.  Runs without a GPU."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1106_5908_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <vector>
#include "sorted_place.h"
int main(int argc, char **argv) {
  FILE *f = std::fopen(argv[1], "rb");
  int64_t hdr[4];
  if (std::fread(hdr, 8, 4, f) != 4) return 2;
  const int R = int(hdr[0]), Q = int(hdr[1]);
  const int64_t m = hdr[2], period = hdr[3];
  std::vector<int32_t> col(size_t(m) + 1), lrow(size_t(m) + 1), len(size_t(R), 0);
  if (m > 0 && (std::fread(col.data(), 4, size_t(m), f) != size_t(m) ||
                std::fread(lrow.data(), 4, size_t(m), f) != size_t(m))) return 3;
  std::fclose(f);
  for (int64_t i = 0; i < m; ++i) len[size_t(lrow[size_t(i)])]++;
  const std::vector<int32_t> s =
      spmv::rt::sorted_place_block(col.data(), lrow.data(), len.data(), m, R, Q, period);
  FILE *o = std::fopen(argv[2], "wb");
  const int64_t n = int64_t(s.size());
  std::fwrite(&n, 8, 1, o);
  if (n) std::fwrite(s.data(), 4, size_t(n), o);
  std::fclose(o);
  return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ missing")
    d = tmp_path_factory.mktemp("place")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    exe = d / "h"
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-I", CSRC, str(src), "-o", str(exe)])
    return d, exe


def _place(harness, R, Q, col, lrow, period=0):
    d, exe = harness
    inp, out = d / "in.bin", d / "out.bin"
    with open(inp, "wb") as f:
        np.array([R, Q, col.size, period], dtype=np.int64).tofile(f)
        col.astype(np.int32).tofile(f)
        lrow.astype(np.int32).tofile(f)
    subprocess.check_call([str(exe), str(inp), str(out)])
    with open(out, "rb") as f:
        n = int(np.fromfile(f, dtype=np.int64, count=1)[0])
        return np.fromfile(f, dtype=np.int32, count=n)


def _check(slots, R, Q, col, lrow, slack, start=None):
    """start: the column the sweep begins at (columns below it come last)."""
    m = col.size
    assert slots.size % Q == 0
    used = slots[slots >= 0]
    assert np.array_equal(np.sort(used), np.arange(m)), "every entry exactly once"
    longest = int(np.bincount(lrow, minlength=R).max()) if m else 0
    bound = max(-(-m // Q), longest)
    chunks = slots.reshape(-1, Q) if slots.size else np.zeros((0, Q), np.int32)
    assert len(chunks) <= bound + slack, (len(chunks), bound)
    for c in chunks:
        k = int((c >= 0).sum())
        assert k >= 1, "a chunk's first slot holds an entry"
        assert (c[:k] >= 0).all() and (c[k:] < 0).all(), "entries first, then empty slots"
        e = c[:k]
        assert np.unique(lrow[e]).size == k, "no row twice in a chunk"
        c = col[e].astype(np.int64)
        if start is not None:
            c = np.where(c >= start, c, c + (1 << 40))
        key = c * (m + 1) + e
        assert (np.diff(key) > 0).all(), "column order inside a chunk"
    return len(chunks), bound


def _band_block(rng, R, mean_len, width):
    lens = np.minimum(rng.geometric(1.0 / mean_len, size=R), 4 * mean_len)
    lrow = np.repeat(np.arange(R), lens)
    col = np.clip(lrow + rng.integers(-width, width + 1, size=lrow.size), 0, None)
    return col, lrow


@pytest.mark.parametrize("Q", [1024, 2048, 4096])
def test_band_blocks_at_the_bound(harness, Q):
    rng = np.random.default_rng(1106 + Q)
    R = 4096
    col, lrow = _band_block(rng, R, 13, 200000)
    slots = _place(harness, R, Q, col, lrow)
    n, bound = _check(slots, R, Q, col, lrow, slack=1)
    # the empty slots stay under one chunk's worth plus what the bound adds
    assert slots.size - col.size <= (bound - col.size / Q + 1) * Q


def test_one_long_row_sets_the_chunk_count(harness):
    rng = np.random.default_rng(7)
    R, Q = 64, 1024
    col, lrow = _band_block(rng, R, 8, 1000)
    lrow = np.concatenate([lrow, np.full(5000, 17)])
    col = np.concatenate([col, rng.integers(0, 3000, size=5000)])
    n, bound = _check(_place(harness, R, Q, col, lrow), R, Q, col, lrow, slack=0)
    assert n == bound == 5000 + int((lrow[:-5000] == 17).sum())


def test_round_robin_fallback(harness):
    # N * R above the membership-table limit: dealt round-robin by row
    rng = np.random.default_rng(8)
    R, Q = 16384, 1024
    lrow = np.concatenate([np.repeat(np.arange(R), 2), np.full(4500, 3)])
    col = rng.integers(0, 100000, size=lrow.size)
    n, bound = _check(_place(harness, R, Q, col, lrow), R, Q, col, lrow, slack=0)
    assert bound == 4502 and n == bound


def test_degenerate_blocks(harness):
    R, Q = 256, 1024
    empty = np.zeros(0, dtype=np.int64)
    assert _place(harness, R, Q, empty, empty).size == 0
    # one column for every entry, duplicates inside rows
    lrow = np.repeat(np.arange(R), 3)
    col = np.full(lrow.size, 42)
    _check(_place(harness, R, Q, col, lrow), R, Q, col, lrow, slack=0)
    # a single entry
    one = np.array([5]), np.array([0])
    s = _place(harness, R, Q, *one)
    assert s.size == Q and s[0] == 0 and (s[1:] < 0).all()


def test_sweep_rotated_to_the_period(harness):
    """With a period, a block's sweep starts at the first multiple of it
    above the block's lowest column and wraps round; the placement stays
    valid and at its bound, and the first chunk begins at that column."""
    rng = np.random.default_rng(11)
    R, Q = 4096, 2048
    col, lrow = _band_block(rng, R, 13, 200000)
    col = col + 1000
    lo, hi = int(col.min()), int(col.max())
    for period in (150000, 300000, 10 ** 9):
        s0 = -(-lo // period) * period
        rotated = lo < s0 <= hi
        slots = _place(harness, R, Q, col, lrow, period)
        _check(slots, R, Q, col, lrow, slack=1, start=s0 if rotated else None)
        first = slots[0]
        if rotated:
            assert col[first] == col[col >= s0].min()
        else:
            assert col[first] == lo
