"""Host model of the stream kernel's grouped loads (no GPU).

A workgroup reads its tile's col_idx / val in aligned groups of G entries
(G = 2 for 8-byte values, 4 for 4- and 2-byte values).  The first group
starts up to G - 1 entries before the tile and the last may run past it; in
a batch the members' arrays are packed back to back, so the early slots of a
member's first tile hold the previous member's columns, which index another
member's vector.  The kernel replaces the column of every slot outside the
tile by the column of the group's first in-tile entry before gathering.

This test applies that rule, and the greedy tiling of the runtime, to every
tile of the 512-stencil batch in all three tile sizes and both group sizes,
and checks that every gathered index comes from a slot inside the tile (so
it is one of the tile's own columns, below the member's column count).
Groups strictly between the first and the last lie inside the tile by
construction (their slots start at G or later and end before nnz + off), so
only the first and last groups are modelled.  It also checks that the rule
the kernel used before, which kept the early slots' columns, does gather
other members' columns on this workload, so the model tells the two apart."""
from __future__ import annotations

import numpy as np
import pytest

from workloads import gen

WG = 256
MAX_ROWS = 2 * WG
ITEMS = (4, 8, 16)


def tiles_of(rp: np.ndarray, tile_items: int) -> np.ndarray:
    """Greedy tiles of consecutive rows holding at most 256 * E - 4 entries
    and at most 512 rows; a longer row gets a tile of its own."""
    n = rp.size - 1
    cap = WG * tile_items - 4
    out = [0]
    r = 0
    while r < n:
        e = int(np.searchsorted(rp, rp[r] + cap, side="right")) - 1
        e = max(r + 1, min(e, r + MAX_ROWS, n))
        out.append(e)
        r = e
    return np.asarray(out, dtype=np.int64)


def gather_sources(p0, p1, nz_off, G, keep_early):
    """For the tiles [p0, p1) of a member at nz_off (arrays), the slot (within
    the group window starting at base = p0 - off) whose column each position
    of the first and of the last load group gathers, under the kernel's rule
    (keep_early=False) or the earlier one (keep_early=True).  Returns
    (source slots [T, 2G], off [T], nnz [T], base [T])."""
    nnz = p1 - p0
    off = (p0 + nz_off) % G
    base = p0 - off
    lastg = (nnz + off - 1) // G
    src = []
    for g in (np.zeros_like(lastg), lastg):
        slots = G * g[:, None] + np.arange(G)[None, :]
        inside = (slots >= off[:, None]) & (slots < (nnz + off)[:, None])
        if keep_early:
            keep = (np.arange(G)[None, :] == 0) | (slots < (nnz + off)[:, None])
            src.append(np.where(keep, slots, (G * g)[:, None]))
        else:
            first = np.where(g == 0, off, G * g)
            src.append(np.where(inside, slots, first[:, None]))
    return np.concatenate(src, axis=1), off, nnz, base


@pytest.fixture(scope="module")
def batch_pool():
    sizes, kinds = gen.batch_sizes()
    members = []
    cols = []
    at = 0
    for n, three_d in zip(sizes, kinds):
        A = gen.truncated_stencil(int(n), bool(three_d))
        rp = A.row_ptr.astype(np.int64)
        tiles = {e: tiles_of(rp, e) for e in ITEMS}
        members.append((rp, at, A.n_cols, tiles))
        cols.append(A.col_idx)
        at += A.nnz
    # the pooled col_idx as the runtime packs it, plus the 64-byte tail padding
    pool = np.concatenate(cols + [np.zeros(16, dtype=np.int32)]).astype(np.int64)
    return members, pool


@pytest.mark.parametrize("G", [2, 4])
def test_every_gather_index_is_a_tile_column(batch_pool, G):
    members, pool = batch_pool
    members_old = set()
    checked = 0
    for m, (rp, nz_off, nc, tiles) in enumerate(members):
        for items in ITEMS:
            t = tiles[items]
            p0, p1 = rp[t[:-1]], rp[t[1:]]
            use = (p1 > p0) & (p1 - p0 <= WG * items - (G - 1))  # else: early return / long row
            p0, p1 = p0[use], p1[use]
            src, off, nnz, base = gather_sources(p0, p1, nz_off, G, keep_early=False)
            inside = (src >= off[:, None]) & (src < (nnz + off)[:, None])
            assert inside.all(), f"member {m}, {items} entries per lane: a gather slot outside its tile"
            vals = pool[nz_off + base[:, None] + src]
            assert (vals >= 0).all() and (vals < nc).all()
            checked += p0.size
            src, off, nnz, base = gather_sources(p0, p1, nz_off, G, keep_early=True)
            vals = pool[nz_off + base[:, None] + src]
            if (vals >= nc).any() or not ((src >= off[:, None]) & (src < (nnz + off)[:, None])).all():
                members_old.add(m)
    assert checked > 100_000
    # the earlier rule gathered columns outside the tile for many members
    assert len(members_old) > 100, len(members_old)
