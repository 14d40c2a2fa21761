// gfx950 kernels of the CRS product C = C + A*B (the kernel of Listing 1 of
// Schubert, Fehske, Hager, Wellein 2011, with the storage of Sect. 1.2).
//
// The loop is bound by memory bandwidth (code balance of Eq. (1): at least
// 6 bytes per flop in FP64), so nothing here uses the matrix cores; the
// kernels are organised around moving val / col_idx at full HBM rate:
//   * stream kernel: the planner cuts the rows into tiles of at most
//     256 * E stored entries; a 256-thread workgroup reads its tile's val and
//     col_idx with fully coalesced loads (E per lane, all issued before the
//     gathers of B), writes the products to LDS and reduces each row there
//     with L lanes per row (L chosen per tile from its row count).
//   * staged stream kernel: the stream kernel's tiles, with the few column
//     ranges a tile of a stencil-like matrix reads loaded into LDS first, so
//     the entries read B from LDS instead of gathering it.
//   * vector kernel: L lanes of a wavefront share a row, stride through it
//     and combine their partial sums with cross-lane shuffles.
//   * symmetric kernel: the upper triangle of a symmetric matrix, the
//     transposed half scattered into C with atomic adds (Sect. 1.3.1).
//   * block kernel: k right-hand sides; a tile's col_idx / val are staged in
//     LDS once and each row is handled by KT/VW lanes holding VW columns.
//   * batch kernels: many matrices; the tiles of all members are cut into
//     eight per-XCD work queues that a persistent grid drains through atomic
//     counters (with stealing once a workgroup's own queue is empty), or
//     one workgroup per tile (plain or staged).
// val and col_idx are read with the nontemporal hint so the single-use
// matrix stream does not evict B from L2 / MALL.  Tile numbers can be
// remapped so that each of the eight XCDs (each with a private L2) gets a
// contiguous range of rows and therefore a compact window of B.
//
// Accumulators start at -0.0, the additive identity of IEEE arithmetic, so a
// row whose products are all -0.0 keeps the sign the sequential loop gives;
// rows without entries leave C untouched.
#include <hip/hip_runtime.h>

#include <climits>

#include "spmv_internal.h"

namespace spmv {
namespace {

constexpr int WG = 256;
constexpr int NXCD = 8;
static_assert(NXCD == NXCD_QUEUES, "one queue counter per XCD");

template <int P> struct Ty;
template <> struct Ty<P_F64> { using V = double;   using X = double; };
template <> struct Ty<P_F32> { using V = float;    using X = float;  };
template <> struct Ty<P_BF16> { using V = uint16_t; using X = float;  };
template <> struct Ty<P_F32_F64> { using V = float; using X = double; };
// In every mode the accumulator has the type of B and C.

template <class T, bool NT>
__device__ __forceinline__ T ld(const T *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <class X, class V>
__device__ __forceinline__ X widen(V v) { return static_cast<X>(v); }
template <>
__device__ __forceinline__ float widen<float, uint16_t>(uint16_t v) {
  return __uint_as_float(static_cast<uint32_t>(v) << 16);
}

template <class X> __device__ __forceinline__ X neg_zero() { return static_cast<X>(-0.0); }

// Tile `bid` of `n` -> the tile it processes.  Workgroups are handed to the
// XCDs round-robin (bid % 8); XCD x receives the contiguous range of tiles
// starting at x*q + min(x, r).  A bijection of [0, n).
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t n, int remap) {
  if (!remap) return bid;
  const int64_t x = bid % NXCD, i = bid / NXCD;
  const int64_t q = n / NXCD, r = n % NXCD;
  return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ int floor_pow2(int v) { return 1 << (31 - __builtin_clz(v)); }

// Barrier for LDS hand-over only.  The fence is restricted to the local
// address space, so loads of global memory still in flight (the next tile's
// prefetch) are not drained at the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Stream kernel building blocks.  A tile is rows [r0, r1) holding entries
// [p0, p1); p1 - p0 <= 256 * E unless the tile is a single long row.
// ---------------------------------------------------------------------------

// Coalesced loads of a tile's col_idx and val: lane tid takes entries
// tid, tid + 256, ...; indices past the tile are clamped to its last entry
// (nnz >= 1), so every lane issues all E loads with no branch.
template <int E, bool NT, class V>
__device__ __forceinline__ void load_cv(const int32_t *__restrict__ col,
                                        const V *__restrict__ val, int p0, int nnz, int (&c)[E],
                                        V (&v)[E]) {
  const int last = nnz - 1;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = min(e * WG + (int)threadIdx.x, last);
    c[e] = ld<int32_t, NT>(col + p0 + k);
    v[e] = ld<V, NT>(val + p0 + k);
  }
}

// Grouped form of load_cv: lane tid takes groups of G adjacent entries
// (G = 2 for 8-byte values, 4 for 4- and 2-byte values), group g covering
// entries base + G*g .. base + G*g + G - 1 with g = tid, tid + 256, ...;
// base = p0 - off is the entry at or below the tile start whose index in the
// allocation is a multiple of G, so each group is one aligned vector load of
// indices (8 or 16 bytes) and one of values (16 or 8 bytes).  Groups past the
// tile are clamped to its last group.  A group's slots may lie outside the
// tile: the first group starts `off` entries early, inside the previous tile
// (or, in a batch, inside the previous member, whose columns index another
// vector), and the last one may run past it -- for the part's last tile, into
// the arrays' tail padding.  Such slots take the column of the group's first
// in-tile entry (slot `off` of group 0, slot 0 of every later group), so
// every gather index is one of the tile's own columns; their products land
// in LDS slots phase 2 never reads.  Needs nnz + off <= 256 * E.
template <class V> constexpr int group_of() { return sizeof(V) == 8 ? 2 : 4; }
template <class V, int G> struct VecOf;
template <> struct VecOf<double, 2> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float, 4> { typedef float T __attribute__((ext_vector_type(4))); };
template <> struct VecOf<uint16_t, 4> { typedef uint16_t T __attribute__((ext_vector_type(4))); };
template <int G> struct IdxOf;
template <> struct IdxOf<2> { typedef int32_t T __attribute__((ext_vector_type(2))); };
template <> struct IdxOf<4> { typedef int32_t T __attribute__((ext_vector_type(4))); };

template <int E, bool NT, class V>
__device__ __forceinline__ void load_cv_groups(const int32_t *__restrict__ col,
                                               const V *__restrict__ val, int base, int nnz, int off,
                                               int (&c)[E], V (&v)[E]) {
  constexpr int G = group_of<V>();
  using VV = typename VecOf<V, G>::T;
  using IV = typename IdxOf<G>::T;
  const int lastg = (nnz + off - 1) / G;
#pragma unroll
  for (int e = 0; e < E / G; ++e) {
    const int g = min(e * WG + (int)threadIdx.x, lastg);
    const IV ci = ld<IV, NT>(reinterpret_cast<const IV *>(col + base + G * g));
    const VV vi = ld<VV, NT>(reinterpret_cast<const VV *>(val + base + G * g));
    int first = ci[0];
#pragma unroll
    for (int j = 1; j < G; ++j) first = (g == 0 && off == j) ? ci[j] : first;
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int slot = G * g + j;
      c[G * e + j] = (slot >= off && slot < nnz + off) ? ci[j] : first;
      v[G * e + j] = vi[j];
    }
  }
}

// A row longer than a tile (the planner gives it a tile of its own): the
// workgroup strides through it and reduces in LDS.  Ends with a barrier.
template <int P, bool NT>
__device__ void long_row(const int32_t *__restrict__ col, const typename Ty<P>::V *__restrict__ val,
                         int p0, int p1, int64_t out, const typename Ty<P>::X *__restrict__ x,
                         typename Ty<P>::X *__restrict__ y, typename Ty<P>::X *s_red) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  const int tid = threadIdx.x;
  X acc = neg_zero<X>();
  for (int j = p0 + tid; j < p1; j += WG)
    acc += widen<X>(ld<V, NT>(val + j)) * x[ld<int32_t, NT>(col + j)];
  s_red[tid] = acc;
  lds_barrier();
  for (int off = WG / 2; off > 0; off >>= 1) {
    if (tid < off) s_red[tid] += s_red[tid + off];
    lds_barrier();
  }
  if (tid == 0) y[out] = y[out] + s_red[0];
  lds_barrier();
}

// Where a lane's row sums go in phase 2 (see tile_reduce).  A tile of at
// most 256 rows gives each row L lanes (a power of two, at most 64); a tile
// of 257..512 rows gives each lane the rows tid and tid + 256 (L = 1).  More
// rows per tile are handled by a loop (the planner does not produce them).
template <class X>
struct RowSlot {
  int L, lane;
  int a0, b0, a1, b1;
  int64_t o0, o1;
  X c0, c1;
};

// Row bounds and old C values are loaded here, early and without branches
// (lanes past the last row take the last row with an empty range), so their
// latency hides under phase 1.  C rows of a tile are written by this
// workgroup only.
template <class X, bool IND>
__device__ __forceinline__ RowSlot<X> row_slot(const int32_t *__restrict__ rp,
                                               const int32_t *__restrict__ row_ids, int r0,
                                               int nrows, int p0, const X *__restrict__ y) {
  RowSlot<X> s;
  const int nr = max(nrows, 1);
  const int tid = (int)threadIdx.x;
  int row0, row1;
  if (nr <= WG) {
    s.L = min(floor_pow2(WG / nr), 64);
    const int lg = __builtin_ctz(s.L);
    row0 = tid >> lg;
    s.lane = tid & (s.L - 1);
    row1 = nr;  // none
  } else {
    s.L = 1;
    s.lane = 0;
    row0 = tid;
    row1 = tid + WG;
  }
  const int rc0 = min(row0, nr - 1), rc1 = min(row1, nr - 1);
  s.a0 = rp[r0 + rc0] - p0;
  s.b0 = rp[r0 + rc0 + (row0 < nrows ? 1 : 0)] - p0;
  s.a1 = rp[r0 + rc1] - p0;
  s.b1 = rp[r0 + rc1 + (row1 < nrows ? 1 : 0)] - p0;
  if constexpr (IND) {
    s.o0 = row_ids[r0 + rc0];
    s.o1 = row_ids[r0 + rc1];
  } else {
    s.o0 = (int64_t)(r0 + rc0);
    s.o1 = (int64_t)(r0 + rc1);
  }
  s.c0 = y[s.o0];
  s.c1 = y[s.o1];
  return s;
}

// s[a] + s[a + L] + ... (indices below b) with four independent partial
// sums, so that four LDS reads are in flight at a time instead of one.
// Every partial sum starts at -0.0 (see above).
template <class X>
__device__ __forceinline__ X lds_row_sum(const X *s, int a, int b, int L) {
  X p0 = neg_zero<X>(), p1 = neg_zero<X>(), p2 = neg_zero<X>(), p3 = neg_zero<X>();
  int j = a;
  for (; j + 3 * L < b; j += 4 * L) {
    p0 += s[j];
    p1 += s[j + L];
    p2 += s[j + 2 * L];
    p3 += s[j + 3 * L];
  }
  for (; j < b; j += L) p0 += s[j];
  return (p0 + p1) + (p2 + p3);
}

// Phase 2: every row of the tile summed out of LDS and added to C.
template <class X, bool IND>
__device__ __forceinline__ void tile_reduce(const int32_t *__restrict__ rp,
                                            const int32_t *__restrict__ row_ids, int r0, int nrows,
                                            int p0, const RowSlot<X> &s, X *__restrict__ y,
                                            const X *s_prod) {
  if (nrows <= 2 * WG) {
    X acc = lds_row_sum(s_prod, s.a0 + s.lane, s.b0, s.L);
    for (int off = s.L >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (s.lane == 0 && s.b0 > s.a0) y[s.o0] = s.c0 + acc;
    if (nrows > WG) {
      const X acc1 = lds_row_sum(s_prod, s.a1, s.b1, 1);
      if (s.b1 > s.a1) y[s.o1] = s.c1 + acc1;
    }
  } else {
    for (int rr = (int)threadIdx.x; rr < nrows; rr += WG) {
      const int ra = rp[r0 + rr] - p0;
      const int rb = rp[r0 + rr + 1] - p0;
      if (rb > ra) {
        const X acc = lds_row_sum(s_prod, ra, rb, 1);
        int64_t oo;
        if constexpr (IND) oo = row_ids[r0 + rr];
        else oo = (int64_t)(r0 + rr);
        y[oo] = y[oo] + acc;
      }
    }
  }
}

// Stream kernel: workgroup g takes tiles [g*tpw, min((g+1)*tpw, n_tiles)) in
// order.  While a tile's products are reduced, the next tile's col_idx and
// val are already in flight (issued before the current tile's barrier).
// Phase 1 per tile: E coalesced col_idx / val loads per lane, then E gathers
// of B, then products into LDS; indices past the tile are clamped to its
// last entry and their products land in LDS slots phase 2 never reads.
// Every load of the loop is issued unconditionally (a tile without entries,
// or a missing next tile, reads entry 0 of the part instead), so the
// compiler's wait counts never have to drain the prefetch early.  The kernel
// is only launched for parts with at least one entry.
// One tile with grouped loads (see load_cv_groups).  `bias` is the index of
// element 0 of `col` / `val` within their allocation modulo the group size,
// so every grouped load is aligned; products go to LDS slot (entry - base)
// and phase 2 reads relative to base.  Ends without a trailing barrier.
template <int P, int E, bool NT, bool IND>
__device__ __forceinline__ void tile_grouped(const int32_t *__restrict__ rp,
                                            const int32_t *__restrict__ col,
                                            const typename Ty<P>::V *__restrict__ val,
                                            const int32_t *__restrict__ row_ids, TileRP m0,
                                            TileRP m1, int bias,
                                            const typename Ty<P>::X *__restrict__ x,
                                            typename Ty<P>::X *__restrict__ y,
                                            typename Ty<P>::X *s_prod) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  constexpr int TILE = WG * E;
  const int nnz = m1.p - m0.p;
  const int nrows = m1.r - m0.r;
  constexpr int G = group_of<V>();
  if (nnz > TILE - (G - 1)) {
    long_row<P, NT>(col, val, m0.p, m1.p, IND ? (int64_t)row_ids[m0.r] : (int64_t)m0.r, x, y,
                    s_prod);
    return;
  }
  if (nnz == 0) return;  // only empty rows: C stays as it is
  const int off = (m0.p + bias) % G;
  const int base = m0.p - off;
  int c[E];
  V v[E];
  load_cv_groups<E, NT>(col, val, base, nnz, off, c, v);
  const RowSlot<X> slot = row_slot<X, IND>(rp, row_ids, m0.r, nrows, base, y);
  X xg[E];
#pragma unroll
  for (int e = 0; e < E; ++e) xg[e] = x[c[e]];
#pragma unroll
  for (int e = 0; e < E / G; ++e) {
    const int g = e * WG + (int)threadIdx.x;
#pragma unroll
    for (int j = 0; j < G; ++j) s_prod[G * g + j] = widen<X>(v[G * e + j]) * xg[G * e + j];
  }
  lds_barrier();
  tile_reduce<X, IND>(rp, row_ids, m0.r, nrows, base, slot, y, s_prod);
}

// One tile per workgroup (tiles_per_group == 1): the plain form of the
// stream kernel, with no prefetch state.
template <int P, int E, bool NT, bool IND>
__global__ __launch_bounds__(WG) void k_stream1(CsrDev A, const TileRP *__restrict__ tiles,
                                                int64_t n_tiles, int remap, const void *xv,
                                                void *yv) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  __shared__ X s_prod[WG * E];
  const int64_t t = xcd_tile(blockIdx.x, n_tiles, remap);
  tile_grouped<P, E, NT, IND>(A.row_ptr, A.col, static_cast<const V *>(A.val), A.row_ids, tiles[t],
                             tiles[t + 1], 0, static_cast<const X *>(xv), static_cast<X *>(yv),
                             s_prod);
}

template <int P, int E, bool NT, bool IND>
__global__ __launch_bounds__(WG) void k_stream(CsrDev A, const TileRP *__restrict__ tiles,
                                               int64_t n_tiles, int tpw, int64_t n_groups,
                                               int remap, const void *xv, void *yv) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  constexpr int TILE = WG * E;
  __shared__ X s_prod[TILE];
  const V *__restrict__ val = static_cast<const V *>(A.val);
  const X *__restrict__ x = static_cast<const X *>(xv);
  X *__restrict__ y = static_cast<X *>(yv);
  const int64_t g = xcd_tile(blockIdx.x, n_groups, remap);
  int64_t t = g * tpw;
  const int64_t t_end = min(t + (int64_t)tpw, n_tiles);
  if (t >= t_end) return;
  TileRP m0 = tiles[t], m1 = tiles[t + 1];
  int c[E];
  V v[E];
  RowSlot<X> slot;
  {
    const int nnz = m1.p - m0.p;
    const bool ok = nnz > 0 && nnz <= TILE;
    load_cv<E, NT>(A.col, val, ok ? m0.p : 0, ok ? nnz : 1, c, v);
    slot = row_slot<X, IND>(A.row_ptr, A.row_ids, m0.r, m1.r - m0.r, m0.p, y);
  }
  for (;;) {
    const int nnz = m1.p - m0.p;
    const int nrows = m1.r - m0.r;
    const bool more = t + 1 < t_end;
    const TileRP m2 = tiles[min(t + 2, n_tiles)];
    if (nnz > TILE) {
      long_row<P, NT>(A.col, val, m0.p, m1.p, IND ? (int64_t)A.row_ids[m0.r] : (int64_t)m0.r, x, y,
                      s_prod);
      if (!more) break;
      ++t;
      m0 = m1;
      m1 = m2;
      const int nn = m1.p - m0.p;
      const bool ok = nn > 0 && nn <= TILE;
      load_cv<E, NT>(A.col, val, ok ? m0.p : 0, ok ? nn : 1, c, v);
      slot = row_slot<X, IND>(A.row_ptr, A.row_ids, m0.r, m1.r - m0.r, m0.p, y);
      continue;
    }
    X xg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) xg[e] = x[c[e]];
    // prefetch the next tile: its entries and its row assignment (the
    // current tile's again when there is no next tile)
    int cn[E];
    V vn[E];
    RowSlot<X> slot_n;
    {
      const int nn = m2.p - m1.p;
      const bool ok = more && nn > 0 && nn <= TILE;
      load_cv<E, NT>(A.col, val, ok ? m1.p : 0, ok ? nn : 1, cn, vn);
      const TileRP q0 = more ? m1 : m0, q1 = more ? m2 : m1;
      slot_n = row_slot<X, IND>(A.row_ptr, A.row_ids, q0.r, q1.r - q0.r, q0.p, y);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) s_prod[e * WG + threadIdx.x] = widen<X>(v[e]) * xg[e];
    lds_barrier();
    tile_reduce<X, IND>(A.row_ptr, A.row_ids, m0.r, nrows, m0.p, slot, y, s_prod);
    lds_barrier();
    if (!more) break;
    ++t;
    m0 = m1;
    m1 = m2;
    slot = slot_n;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      c[e] = cn[e];
      v[e] = vn[e];
    }
  }
}

// ---------------------------------------------------------------------------
// Staged stream kernel.  A tile of a stencil-like matrix reads B from a few
// contiguous column ranges (one per plane of neighbours).  The planner
// merges each tile's columns into at most RUN_MAX ascending runs and records
// them in a run table (see spmv_internal.h); the workgroup loads the runs
// into LDS with coalesced loads issued before the tile's col_idx / val, and
// each entry then reads its B value from LDS at col + d_r (r: the last run
// starting at or below col).  The gathers thus leave the chain that follows
// the col_idx loads.  A tile whose table row says nr = 0 is run as in the
// stream kernel.  The arithmetic is the stream kernel's: the same products
// summed in the same order.
// ---------------------------------------------------------------------------
// LDS elements of B a staged tile may hold.
template <class X> constexpr int stage_slots() { return RUN_STAGE_BYTES / (int)sizeof(X); }

// In the F32-value / F64-vector mode the staged B shares the products'
// LDS buffer: every lane reads its B values into registers before the
// products overwrite them (one more barrier), so a workgroup needs 32 KB
// instead of 44 KB at 16 entries per lane and five workgroups fit a CU
// instead of three (on the 27-point matrix 184 against 202 us; the other
// modes, whose staging costs less, gain nothing from it).
template <int P> constexpr bool stage_shares_products() { return P == P_F32_F64; }
template <int P, int E> constexpr int staged_lds_elems() {
  using X = typename Ty<P>::X;
  return stage_shares_products<P>()
             ? (WG * E > stage_slots<X>() ? WG * E : stage_slots<X>())
             : WG * E + stage_slots<X>();
}

// One tile of the staged kernel; `rt` is its run-table row and s_prod holds
// staged_lds_elems<P, E>() elements.  `bias` as in tile_grouped.
template <int P, int E, bool NT, bool IND>
__device__ __forceinline__ void staged_tile(const int32_t *__restrict__ rp,
                                            const int32_t *__restrict__ col,
                                            const typename Ty<P>::V *__restrict__ val,
                                            const int32_t *__restrict__ row_ids, TileRP m0,
                                            TileRP m1, int bias, const int32_t *__restrict__ rt,
                                            const typename Ty<P>::X *__restrict__ x,
                                            typename Ty<P>::X *__restrict__ y,
                                            typename Ty<P>::X *s_prod) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  constexpr int G = group_of<V>();
  constexpr int NB = stage_slots<X>() / WG;
  constexpr bool share = stage_shares_products<P>();
  X *s_b = share ? s_prod : s_prod + WG * E;
  const int nr = rt[0];
  if (nr == 0) {
    tile_grouped<P, E, NT, IND>(rp, col, val, row_ids, m0, m1, bias, x, y, s_prod);
    return;
  }
  // nr in [1, RUN_MAX]; L in [1, WG * NB]; 1 <= nnz <= WG * E - 4 (planner)
  const int L = rt[1];
  const int d0 = rt[6], d1 = rt[7], d2 = rt[8], d3 = rt[9];
  const int s1 = nr > 1 ? rt[3] : INT_MAX, s2 = nr > 2 ? rt[4] : INT_MAX,
            s3 = nr > 3 ? rt[5] : INT_MAX;
  const int o1 = nr > 1 ? s1 + d1 : INT_MAX, o2 = nr > 2 ? s2 + d2 : INT_MAX,
            o3 = nr > 3 ? s3 + d3 : INT_MAX;
  const int tid = (int)threadIdx.x;
  // LDS slot i holds B[i - d_r], r the last run whose slots start at or
  // below i.  Passes wholly past L are skipped (a uniform branch); within the
  // last pass, slots past L load slot L - 1 again and are not stored.
  X bst[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i * WG >= L) break;
    const int slot = min(i * WG + tid, L - 1);
    int d = d0;
    if (slot >= o1) d = d1;
    if (slot >= o2) d = d2;
    if (slot >= o3) d = d3;
    bst[i] = x[slot - d];
  }
  const int nnz = m1.p - m0.p;
  const int nrows = m1.r - m0.r;
  const int off = (m0.p + bias) % G;
  const int base = m0.p - off;
  int c[E];
  V v[E];
  load_cv_groups<E, NT>(col, val, base, nnz, off, c, v);
  const RowSlot<X> slot = row_slot<X, IND>(rp, row_ids, m0.r, nrows, base, y);
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i * WG + tid < L) s_b[i * WG + tid] = bst[i];
  lds_barrier();
  X xg[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int cc = c[e];
    int d = d0;
    if (cc >= s1) d = d1;
    if (cc >= s2) d = d2;
    if (cc >= s3) d = d3;
    xg[e] = s_b[cc + d];
  }
  if constexpr (share) lds_barrier();  // B read by every lane before the products overwrite it
#pragma unroll
  for (int e = 0; e < E / G; ++e) {
    const int g = e * WG + tid;
#pragma unroll
    for (int j = 0; j < G; ++j) s_prod[G * g + j] = widen<X>(v[G * e + j]) * xg[G * e + j];
  }
  lds_barrier();
  tile_reduce<X, IND>(rp, row_ids, m0.r, nrows, base, slot, y, s_prod);
}

template <int P, int E, bool NT, bool IND>
__global__ __launch_bounds__(WG) void k_staged(CsrDev A, const TileRP *__restrict__ tiles,
                                               const int32_t *__restrict__ runs, int64_t n_tiles,
                                               int remap, const void *xv, void *yv) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  __shared__ X s_prod[staged_lds_elems<P, E>()];
  const int64_t t = xcd_tile(blockIdx.x, n_tiles, remap);
  staged_tile<P, E, NT, IND>(A.row_ptr, A.col, static_cast<const V *>(A.val), A.row_ids, tiles[t],
                             tiles[t + 1], 0, runs + t * RUN_WORDS, static_cast<const X *>(xv),
                             static_cast<X *>(yv), s_prod);
}

// ---------------------------------------------------------------------------
// Diagonal panels in one launch.  The panels of a part split its entries by
// their distance from the diagonal so that the workgroups running at one time
// gather from a narrow window of B (one that stays in L2); applied as K
// launches, every launch reads and writes C again.  Here workgroup b takes
// rows [b*R, b*R + R) and walks the K panels of those rows in turn: for each
// panel the block's entries are loaded as in the stream kernel (grouped,
// coalesced), their products go to LDS, and each lane adds the sums of its
// two rows (tid and tid + 256) to registers.  C is read once before the
// first panel and written once after the last; a row with no entry in any
// panel is left untouched.  Workgroups started together walk the panels
// together, so the window of B stays narrow.  A panel whose entries in the
// block exceed one tile is summed row by row from global memory (the
// planner sizes R so that this is rare).
// ---------------------------------------------------------------------------
template <int P, int E, bool NT>
__global__ __launch_bounds__(WG) void k_fused(PanelSetDev S, int R, int64_t n_blocks, int remap,
                                              const void *xv, void *yv) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  constexpr int TILE = WG * E;
  constexpr int G = group_of<V>();
  __shared__ X s_prod[TILE];
  const X *__restrict__ x = static_cast<const X *>(xv);
  X *__restrict__ y = static_cast<X *>(yv);
  const int64_t b = xcd_tile(blockIdx.x, n_blocks, remap);
  const int64_t r0 = b * R;
  const int64_t r1 = min(r0 + (int64_t)R, S.n_rows);
  const int nrows = (int)(r1 - r0);
  const int tid = (int)threadIdx.x;
  const bool has0 = tid < nrows, has1 = tid + WG < nrows;
  const int64_t row0 = r0 + (has0 ? tid : 0), row1 = r0 + (has1 ? tid + WG : 0);
  const X c0 = y[row0], c1 = y[row1];
  X acc0 = neg_zero<X>(), acc1 = neg_zero<X>();
  int cnt0 = 0, cnt1 = 0;
  for (int k = 0; k < S.K; ++k) {
    const int32_t *__restrict__ rp = S.rp[k];
    const int32_t *__restrict__ col = S.col[k];
    const V *__restrict__ val = static_cast<const V *>(S.val[k]);
    const int pa = rp[r0], pb = rp[r1];
    const int a0 = rp[row0], e0 = has0 ? rp[row0 + 1] : a0;
    const int a1 = rp[row1], e1 = has1 ? rp[row1 + 1] : a1;
    cnt0 += e0 - a0;
    cnt1 += e1 - a1;
    const int nnz = pb - pa;
    if (nnz == 0) continue;
    if (nnz > TILE - (G - 1)) {
      for (int j = a0; j < e0; ++j) acc0 += widen<X>(ld<V, NT>(val + j)) * x[ld<int32_t, NT>(col + j)];
      for (int j = a1; j < e1; ++j) acc1 += widen<X>(ld<V, NT>(val + j)) * x[ld<int32_t, NT>(col + j)];
      continue;
    }
    // each panel is an allocation of its own, so entry 0 is group-aligned
    const int off = pa % G;
    const int base = pa - off;
    int c[E];
    V v[E];
    load_cv_groups<E, NT>(col, val, base, nnz, off, c, v);
    X xg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) xg[e] = x[c[e]];
#pragma unroll
    for (int e = 0; e < E / G; ++e) {
      const int g = e * WG + tid;
#pragma unroll
      for (int j = 0; j < G; ++j) s_prod[G * g + j] = widen<X>(v[G * e + j]) * xg[G * e + j];
    }
    lds_barrier();
    acc0 += lds_row_sum(s_prod, a0 - base, e0 - base, 1);
    acc1 += lds_row_sum(s_prod, a1 - base, e1 - base, 1);
    lds_barrier();
  }
  if (has0 && cnt0 > 0) y[row0] = c0 + acc0;
  if (has1 && cnt1 > 0) y[row1] = c1 + acc1;
}

// ---------------------------------------------------------------------------
// Vector kernel: L lanes per row, rows_per_wg consecutive rows per workgroup.
// ---------------------------------------------------------------------------
template <int P, int L, bool NT>
__global__ __launch_bounds__(WG) void k_vector(CsrDev A, int64_t rows_per_wg, int64_t n_wg,
                                               int remap, const void *xv, void *yv) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  constexpr int G = WG / L;
  const V *__restrict__ val = static_cast<const V *>(A.val);
  const X *__restrict__ x = static_cast<const X *>(xv);
  X *__restrict__ y = static_cast<X *>(yv);
  const int64_t b = xcd_tile(blockIdx.x, n_wg, remap);
  const int64_t rb = b * rows_per_wg;
  const int64_t re = min(rb + rows_per_wg, A.n_rows);
  const int g = threadIdx.x / L;
  const int lane = threadIdx.x % L;
  for (int64_t base = rb; base < re; base += G) {
    const int64_t r = base + g;
    int a = 0, e = 0;
    if (r < re) {
      a = A.row_ptr[r];
      e = A.row_ptr[r + 1];
    }
    X acc = neg_zero<X>();
    for (int j = a + lane; j < e; j += L)
      acc += widen<X>(ld<V, NT>(val + j)) * x[ld<int32_t, NT>(A.col + j)];
    for (int off = L >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0 && e > a) {
      const int64_t o = A.row_ids ? A.row_ids[r] : r;
      y[o] = y[o] + acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Symmetric kernel (FP64): A = U + U^T - diag(U) from its upper triangle U,
// every stored column at or right of its row (the storage Sect. 1.3.1
// describes and sets aside).  L lanes share a row: each entry adds
// val * B[col] to the row's sum and, off the diagonal, scatters val * B[row]
// into C[col] with a device-scope atomic add.  Other rows scatter into
// C[row] at the same time, so the row's sum is added atomically too; the
// order of the additions into one C entry is not fixed.
// ---------------------------------------------------------------------------
template <int L, bool NT>
__global__ __launch_bounds__(WG) void k_sym(CsrDev A, int64_t rows_per_wg, int64_t n_wg, int remap,
                                            const double *__restrict__ x, double *y) {
  constexpr int G = WG / L;
  const double *__restrict__ val = static_cast<const double *>(A.val);
  const int64_t b = xcd_tile(blockIdx.x, n_wg, remap);
  const int64_t rb = b * rows_per_wg;
  const int64_t re = min(rb + rows_per_wg, A.n_rows);
  const int g = threadIdx.x / L;
  const int lane = threadIdx.x % L;
  for (int64_t base = rb; base < re; base += G) {
    const int64_t r = base + g;
    int a = 0, e = 0;
    double xr = 0.0;
    if (r < re) {
      a = A.row_ptr[r];
      e = A.row_ptr[r + 1];
      xr = x[r];
    }
    double acc = -0.0;
    for (int j = a + lane; j < e; j += L) {
      const int c = ld<int32_t, NT>(A.col + j);
      const double v = ld<double, NT>(val + j);
      acc += v * x[c];
      if (c != r) unsafeAtomicAdd(y + c, v * xr);
    }
    for (int off = L >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0 && e > a) unsafeAtomicAdd(y + r, acc);
  }
}

// ---------------------------------------------------------------------------
// Block kernel: columns [t0, t0 + KT) of k right-hand sides.  Each row is
// handled by G = KT / VW lanes; lane l owns columns t0 + l*VW .. + VW - 1.
// Every stored value is multiplied by `scale` as it is staged: 1 for
// C = C + A*B; a power of two (exact) for the recursions that need a
// multiple of A, e.g. -2 for the Chebyshev three-term recursion.
// ---------------------------------------------------------------------------
template <class X, int VW> struct VecT;
template <> struct VecT<double, 1> { using T = double; };
template <> struct VecT<double, 2> { using T = double2; };
template <> struct VecT<float, 1> { using T = float; };
template <> struct VecT<float, 2> { using T = float2; };
template <> struct VecT<float, 4> { using T = float4; };

template <class X, int VW>
__device__ __forceinline__ void load_vec(const X *p, X (&out)[VW]) {
  if constexpr (VW == 1) {
    out[0] = *p;
  } else {
    using T = typename VecT<X, VW>::T;
    const T t = *reinterpret_cast<const T *>(p);
    const X *q = reinterpret_cast<const X *>(&t);
#pragma unroll
    for (int i = 0; i < VW; ++i) out[i] = q[i];
  }
}

template <int P, int E, int KT, int VW, bool NT>
__global__ __launch_bounds__(WG) void k_block(CsrDev A, const TileRP *__restrict__ tiles,
                                              int64_t n_tiles, int remap, int k, int t0,
                                              const void *Bv, int64_t ldb, void *Cv, int64_t ldc,
                                              typename Ty<P>::X scale) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  constexpr int TILE = WG * E;
  constexpr int G = KT / VW;
  constexpr int NG = WG / G;
  static_assert(WG * VW <= TILE, "reduction buffer must fit in s_val");
  __shared__ int32_t s_col[TILE];
  __shared__ X s_val[TILE];
  const V *__restrict__ val = static_cast<const V *>(A.val);
  const X *__restrict__ B = static_cast<const X *>(Bv);
  X *__restrict__ C = static_cast<X *>(Cv);
  const int tid = threadIdx.x;
  const int64_t t = xcd_tile(blockIdx.x, n_tiles, remap);
  const int r0 = tiles[t].r, r1 = tiles[t + 1].r;
  const int p0 = tiles[t].p, p1 = tiles[t + 1].p;
  const int nnz = p1 - p0;
  const int g = tid / G;
  const int lane = tid % G;
  const int cb = t0 + lane * VW;
  const bool active = cb < k;  // VW divides k whenever VW > 1

  if (nnz > TILE) {
    // One long row: every group takes every NG-th entry, then the groups'
    // partial sums are combined in LDS in group order.
    X acc[VW];
#pragma unroll
    for (int i = 0; i < VW; ++i) acc[i] = neg_zero<X>();
    if (active) {
      for (int j = p0 + g; j < p1; j += NG) {
        const int c = ld<int32_t, NT>(A.col + j);
        const X a = widen<X>(ld<V, NT>(val + j)) * scale;
        X bv[VW];
        load_vec<X, VW>(B + (int64_t)c * ldb + cb, bv);
#pragma unroll
        for (int i = 0; i < VW; ++i) acc[i] += a * bv[i];
      }
    }
#pragma unroll
    for (int i = 0; i < VW; ++i) s_val[(g * G + lane) * VW + i] = acc[i];
    __syncthreads();
    if (g == 0 && active) {
      const int64_t o = A.row_ids ? A.row_ids[r0] : r0;
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        X s = neg_zero<X>();
        for (int q = 0; q < NG; ++q) s += s_val[(q * G + lane) * VW + i];
        C[o * ldc + cb + i] = C[o * ldc + cb + i] + s;
      }
    }
    return;
  }

  if (nnz > 0) {
    // clamped, unconditional staging (slots past the tile are never read)
    const int last = nnz - 1;
    int cc[E];
    V vv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kk = min(e * WG + tid, last);
      cc[e] = ld<int32_t, NT>(A.col + p0 + kk);
      vv[e] = ld<V, NT>(val + p0 + kk);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      s_col[e * WG + tid] = cc[e];
      s_val[e * WG + tid] = widen<X>(vv[e]) * scale;
    }
  }
  __syncthreads();
  if (!active) return;
  const int nrows = r1 - r0;
  for (int rr = g; rr < nrows; rr += NG) {
    const int a = A.row_ptr[r0 + rr] - p0;
    const int b = A.row_ptr[r0 + rr + 1] - p0;
    if (b == a) continue;
    X acc[VW];
#pragma unroll
    for (int i = 0; i < VW; ++i) acc[i] = neg_zero<X>();
    int j = a;
    for (; j + 2 <= b; j += 2) {
      const int c0 = s_col[j], c1 = s_col[j + 1];
      const X a0 = s_val[j], a1 = s_val[j + 1];
      X b0[VW], b1[VW];
      load_vec<X, VW>(B + (int64_t)c0 * ldb + cb, b0);
      load_vec<X, VW>(B + (int64_t)c1 * ldb + cb, b1);
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        acc[i] += a0 * b0[i];
        acc[i] += a1 * b1[i];
      }
    }
    if (j < b) {
      const int c0 = s_col[j];
      const X a0 = s_val[j];
      X b0[VW];
      load_vec<X, VW>(B + (int64_t)c0 * ldb + cb, b0);
#pragma unroll
      for (int i = 0; i < VW; ++i) acc[i] += a0 * b0[i];
    }
    const int64_t o = A.row_ids ? A.row_ids[r0 + rr] : (int64_t)(r0 + rr);
#pragma unroll
    for (int i = 0; i < VW; ++i) C[o * ldc + cb + i] = C[o * ldc + cb + i] + acc[i];
  }
}

// Block product over a panel set in one launch (see k_fused): workgroup b
// takes rows [b*R, b*R + R), R = NR * NG; lane group g (G = KT/VW lanes)
// owns rows g, g + NG, ..., g + (NR-1)*NG of the block and keeps their VW
// column sums in registers across the K panels.  Per panel the block's
// col_idx / val are staged in LDS (values scaled as in k_block) and each
// group walks its rows; C is read and written once, after the last panel.
template <int P, int E, int KT, int VW, int NR, bool NT>
__global__ __launch_bounds__(WG) void k_block_fused(PanelSetDev S, int64_t n_blocks, int remap,
                                                    int k, int t0, const void *Bv, int64_t ldb,
                                                    void *Cv, int64_t ldc,
                                                    typename Ty<P>::X scale) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  constexpr int TILE = WG * E;
  constexpr int G = KT / VW;
  constexpr int NG = WG / G;
  constexpr int R = NG * NR;
  constexpr int RB = (R + 1 + WG - 1) / WG;  // row bounds per lane to stage
  __shared__ int32_t s_col[TILE];
  __shared__ X s_val[TILE];
  __shared__ int32_t s_rp[R + 1];
  const X *__restrict__ B = static_cast<const X *>(Bv);
  X *__restrict__ C = static_cast<X *>(Cv);
  const int tid = threadIdx.x;
  const int64_t b = xcd_tile(blockIdx.x, n_blocks, remap);
  const int64_t r0 = b * R;
  const int64_t r1 = min(r0 + (int64_t)R, S.n_rows);
  const int nrows = (int)(r1 - r0);
  const int g = tid / G;
  const int lane = tid % G;
  const int cb = t0 + lane * VW;
  const bool active = cb < k;  // VW divides k whenever VW > 1
  X acc[NR][VW];
  int cnt[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    cnt[i] = 0;
#pragma unroll
    for (int w = 0; w < VW; ++w) acc[i][w] = neg_zero<X>();
  }
  for (int kk = 0; kk < S.K; ++kk) {
    const int32_t *__restrict__ rp = S.rp[kk];
    const int32_t *__restrict__ col = S.col[kk];
    const V *__restrict__ val = static_cast<const V *>(S.val[kk]);
    const int pa = rp[r0], pb = rp[r1];
    const int nnz = pb - pa;
    if (nnz == 0) continue;
    if (nnz > TILE) {
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int rr = g + i * NG;
        if (rr >= nrows) continue;
        const int a = rp[r0 + rr], e = rp[r0 + rr + 1];
        cnt[i] += e - a;
        if (!active) continue;
        for (int j = a; j < e; ++j) {
          const X av = widen<X>(ld<V, NT>(val + j)) * scale;
          X bv[VW];
          load_vec<X, VW>(B + (int64_t)ld<int32_t, NT>(col + j) * ldb + cb, bv);
#pragma unroll
          for (int w = 0; w < VW; ++w) acc[i][w] += av * bv[w];
        }
      }
      continue;
    }
    {
      // the block's entries of this panel and its row bounds, staged in LDS
      // (rows past the block's end take its last bound)
      const int last = nnz - 1;
      int cc[E];
      V vv[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int q = min(e * WG + tid, last);
        cc[e] = ld<int32_t, NT>(col + pa + q);
        vv[e] = ld<V, NT>(val + pa + q);
      }
      int rb[RB];
#pragma unroll
      for (int q = 0; q < RB; ++q) rb[q] = rp[r0 + min(q * WG + tid, nrows)];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        s_col[e * WG + tid] = cc[e];
        s_val[e * WG + tid] = widen<X>(vv[e]) * scale;
      }
#pragma unroll
      for (int q = 0; q < RB; ++q)
        if (q * WG + tid <= R) s_rp[q * WG + tid] = rb[q] - pa;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int rr = g + i * NG;
      if (rr >= nrows) continue;
      const int a = s_rp[rr], e = s_rp[rr + 1];
      cnt[i] += e - a;
      if (!active) continue;
      int j = a;
      for (; j + 2 <= e; j += 2) {
        const int c0 = s_col[j], c1 = s_col[j + 1];
        const X a0 = s_val[j], a1 = s_val[j + 1];
        X b0[VW], b1[VW];
        load_vec<X, VW>(B + (int64_t)c0 * ldb + cb, b0);
        load_vec<X, VW>(B + (int64_t)c1 * ldb + cb, b1);
#pragma unroll
        for (int w = 0; w < VW; ++w) {
          acc[i][w] += a0 * b0[w];
          acc[i][w] += a1 * b1[w];
        }
      }
      if (j < e) {
        const int c0 = s_col[j];
        const X a0 = s_val[j];
        X b0[VW];
        load_vec<X, VW>(B + (int64_t)c0 * ldb + cb, b0);
#pragma unroll
        for (int w = 0; w < VW; ++w) acc[i][w] += a0 * b0[w];
      }
    }
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int rr = g + i * NG;
    if (rr >= nrows || cnt[i] == 0) continue;
    const int64_t o = r0 + rr;
#pragma unroll
    for (int w = 0; w < VW; ++w) C[o * ldc + cb + w] = C[o * ldc + cb + w] + acc[i][w];
  }
}

// ---------------------------------------------------------------------------
// Sorted-block kernel.  On a matrix whose rows gather from scattered columns
// (a wide band), every gather of the stream kernel touches its own cache
// line.  Here one workgroup takes a block of R rows (R accumulators in at
// most 128 KB of LDS: up to 16384 rows in FP64, 32768 in FP32) whose entries the host
// sorted by column: the lanes of one load then gather neighbouring columns,
// several to a line.  The entries come in chunks of Q = 1024 * E slots in
// which no row appears twice, so each lane adds its product to its row's
// accumulator with a plain LDS read-add-write, and one barrier per chunk
// orders the chunks; the sums are therefore the same on every call.  Chunk
// c + 1's gathers and chunk c + 2's slot loads are in flight while chunk c
// is added.  C is read and written once, after the last chunk.
// ---------------------------------------------------------------------------
template <int P, int E, bool NT>
__global__ __launch_bounds__(SB_WG) void k_sorted(SortedDev S, int remap, const void *xv,
                                                  void *yv) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  constexpr int RMAX = SB_LDS_BYTES / (int)sizeof(X);
  constexpr int Q = SB_WG * E;
  __shared__ X acc[RMAX];
  const int R = S.R;  // rows per block, at most RMAX (checked by the launcher)
  const X *__restrict__ x = static_cast<const X *>(xv);
  X *__restrict__ y = static_cast<X *>(yv);
  const V *__restrict__ val = static_cast<const V *>(S.val);
  const int tid = (int)threadIdx.x;
  const int64_t b = S.b0 + xcd_tile(blockIdx.x, S.b1 - S.b0, remap);
  for (int i = tid; i < R; i += SB_WG) acc[i] = neg_zero<X>();
  lds_barrier();
  const int64_t c0 = S.cs[b], c1 = S.cs[b + 1];
  // slots of chunk c (uniform test: past the last chunk, empty slots)
  auto load = [&](int64_t c, int (&cc)[E], V (&vv)[E], int (&rr)[E]) {
    if (c < c1) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t j = c * Q + (int64_t)e * SB_WG + tid;
        cc[e] = ld<int32_t, NT>(S.col + j);
        vv[e] = ld<V, NT>(val + j);
        rr[e] = (int)ld<uint16_t, NT>(S.row + j);
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        cc[e] = 0;
        vv[e] = V(0);
        rr[e] = SB_PAD_ROW;
      }
    }
  };
  auto gather = [&](int64_t c, const int (&cc)[E], X (&g)[E]) {
    if (c < c1) {
#pragma unroll
      for (int e = 0; e < E; ++e) g[e] = x[cc[e]];
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) g[e] = X(0);
    }
  };
  int ca[E], ra[E], cb[E], rb[E];
  V va[E], vb[E];
  X ga[E], gb[E];
  load(c0, ca, va, ra);
  gather(c0, ca, ga);
  load(c0 + 1, cb, vb, rb);
  for (int64_t c = c0; c < c1; ++c) {
    gather(c + 1, cb, gb);
    int cn[E], rn[E];
    V vn[E];
    load(c + 2, cn, vn, rn);
    // rows are distinct within a chunk: no two lanes touch one accumulator
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (ra[e] != SB_PAD_ROW) acc[ra[e]] += widen<X>(va[e]) * ga[e];
    lds_barrier();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      ra[e] = rb[e];
      va[e] = vb[e];
      ga[e] = gb[e];
      rb[e] = rn[e];
      vb[e] = vn[e];
      cb[e] = cn[e];
    }
  }
  // (the last chunk's barrier has ordered every addition before this read)
  const int64_t r0 = b * R;
  const int nrow = (int)min((int64_t)R, S.n_rows - r0);
  for (int i = tid; i < nrow; i += SB_WG) y[r0 + i] = y[r0 + i] + acc[i];
}

// ---------------------------------------------------------------------------
// Sorted-block kernel for a block of right-hand sides: columns [j0, j0 + kk)
// of row-major B and C per launch (kk <= K).  A block of R rows keeps R * K
// sums in LDS; K / VW lanes share a slot, lane l gathering the VW columns
// j0 + l*VW .. + VW - 1 of the slot's row of B (one 16-byte load when
// VW > 1), so one entry's K values come from one contiguous stretch of B.
// A chunk of distinct rows is walked in H pieces of E * (1024 * VW / K)
// slots and closed by a barrier, as in k_sorted; the wide form (VW 2 in
// FP64, 4 in FP32) takes a chunk in one piece, the one-column form in VW
// pieces, so both read the same layout.  Every stored value is multiplied
// by `scale` first (as in k_block).  The layout is streamed with the
// nontemporal hint: it is read once per pass.
// ---------------------------------------------------------------------------
template <int P, int E, int K, int VW, int H>
__global__ __launch_bounds__(SB_WG) void k_sorted_blk(SortedDev S, int remap, const void *xv,
                                                      int64_t ldb, void *yv, int64_t ldc, int j0,
                                                      int kk, typename Ty<P>::X scale) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  constexpr bool NT = true;
  constexpr int RMAX = SB_LDS_BYTES / (int)sizeof(X);
  constexpr int LPS = K / VW;          // lanes per slot
  constexpr int SPW = SB_WG / LPS;     // slots per load step
  constexpr int PQ = SPW * E;          // slots per piece; a chunk is H pieces
  static_assert(K % VW == 0, "a lane's columns lie in one pass");
  __shared__ __align__(16) X acc[RMAX];
  const int R = S.R;  // rows per block; R * K <= RMAX (checked by the launcher)
  const X *__restrict__ x = static_cast<const X *>(xv);
  X *__restrict__ y = static_cast<X *>(yv);
  const V *__restrict__ val = static_cast<const V *>(S.val);
  const int tid = (int)threadIdx.x;
  const int jb = (tid % LPS) * VW, sl = tid / LPS;
  const bool jin = jb < kk;  // kk is a multiple of VW
  const int64_t b = S.b0 + xcd_tile(blockIdx.x, S.b1 - S.b0, remap);
  for (int i = tid; i < R * K; i += SB_WG) acc[i] = neg_zero<X>();
  lds_barrier();
  const int64_t p0 = S.cs[b] * H, p1 = S.cs[b + 1] * H;
  auto load = [&](int64_t p, int (&cc)[E], V (&vv)[E], int (&rr)[E]) {
    if (p < p1) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t q = p * PQ + (int64_t)e * SPW + sl;
        cc[e] = ld<int32_t, NT>(S.col + q);
        vv[e] = ld<V, NT>(val + q);
        rr[e] = (int)ld<uint16_t, NT>(S.row + q);
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        cc[e] = 0;
        vv[e] = V(0);
        rr[e] = SB_PAD_ROW;
      }
    }
  };
  auto gather = [&](int64_t p, const int (&cc)[E], X (&g)[E][VW]) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (p < p1 && jin) {
        load_vec<X, VW>(x + (int64_t)cc[e] * ldb + j0 + jb, g[e]);
      } else {
#pragma unroll
        for (int v = 0; v < VW; ++v) g[e][v] = X(0);
      }
    }
  };
  int ca[E], ra[E], cb[E], rb[E];
  V va[E], vb[E];
  X ga[E][VW], gb[E][VW];
  load(p0, ca, va, ra);
  gather(p0, ca, ga);
  load(p0 + 1, cb, vb, rb);
  for (int64_t p = p0; p < p1; ++p) {
    gather(p + 1, cb, gb);
    int cn[E], rn[E];
    V vn[E];
    load(p + 2, cn, vn, rn);
    // rows are distinct within a chunk: no two slots touch one row's sums
    // between the barriers that close the chunks
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (ra[e] != SB_PAD_ROW && jin) {
        const X a = widen<X>(va[e]) * scale;
        X *ap = &acc[ra[e] * K + jb];
#pragma unroll
        for (int v = 0; v < VW; ++v) ap[v] += a * ga[e][v];
      }
    if (H == 1 || (p - p0) % H == H - 1) lds_barrier();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      ra[e] = rb[e];
      va[e] = vb[e];
      rb[e] = rn[e];
      vb[e] = vn[e];
      cb[e] = cn[e];
#pragma unroll
      for (int v = 0; v < VW; ++v) ga[e][v] = gb[e][v];
    }
  }
  // (the last chunk's barrier has ordered every addition before this read)
  const int64_t r0 = b * R;
  const int nrow = (int)min((int64_t)R, S.n_rows - r0);
  for (int i = tid; i < nrow * K; i += SB_WG) {
    const int r = i / K, jj = i % K;
    if (jj < kk) {
      X *yp = y + (r0 + r) * ldc + j0 + jj;
      *yp = *yp + acc[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Batch kernels: tile t of the queue carries its member's row range, entry
// range and array offsets.
// ---------------------------------------------------------------------------
template <int P, int E, bool NT>
__device__ __forceinline__ void batch_tile(const int32_t *rp, const int32_t *col, const void *val,
                                           const BatchTile &T,
                                           const void *xv, void *yv,
                                           typename Ty<P>::X *s_prod) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  const int32_t *mrp = rp + T.rp_off;
  const TileRP m0{T.r0, T.p0}, m1{T.r1, T.p1};
  tile_grouped<P, E, NT, false>(mrp, col + T.nz_off, static_cast<const V *>(val) + T.nz_off, nullptr,
                               m0, m1, (int)(T.nz_off % group_of<V>()),
                               static_cast<const X *>(xv) + T.x_off,
                               static_cast<X *>(yv) + T.y_off, s_prod);
}

__global__ void k_batch_reset(int32_t *counters) {
  if (threadIdx.x < NXCD && blockIdx.x == 0) counters[threadIdx.x * QUEUE_STRIDE] = 0;
}

// Persistent grid with one work queue per XCD.  The tiles are cut into eight
// contiguous ranges (as xcd_tile does); workgroup g, placed on XCD g % 8,
// claims one tile at a time from its XCD's range through that range's
// counter, so the XCD's resident workgroups work on neighbouring tiles and
// its L2 sees one compact stretch of the batch.  The claim of the next tile
// is issued before the current tile's loads, so its latency hides under
// them.  Each counter has a 128-byte line of its own: counters sharing a
// line serialise the claims of all eight XCDs.  When its own range is used
// up a workgroup claims from the other ranges in turn; it exits once all
// eight are used up (counters only grow, so every workgroup reaches the
// exit).
template <int P, int E, bool NT>
__global__ __launch_bounds__(WG) void k_batch_persistent(const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ col,
                                                         const void *val,
                                                         const BatchTile *tiles, int64_t n_tiles,
                                                         int32_t *counters,
                                                         const void *xv, void *yv) {
  using X = typename Ty<P>::X;
  __shared__ X s_prod[WG * E];
  __shared__ int32_t s_claim;
  const int64_t q = n_tiles / NXCD, r = n_tiles % NXCD;
  int xq = (int)(blockIdx.x % NXCD);
  int tried = 0;
  if (threadIdx.x == 0) s_claim = atomicAdd(&counters[xq * QUEUE_STRIDE], 1);
  lds_barrier();
  int64_t c = s_claim;
  lds_barrier();
  while (true) {
    const int64_t start = xq * q + (xq < r ? xq : r);
    const int64_t size = q + (xq < r ? 1 : 0);
    if (c >= size) {
      if (++tried >= NXCD) break;
      xq = (xq + 1) % NXCD;
      if (threadIdx.x == 0) s_claim = atomicAdd(&counters[xq * QUEUE_STRIDE], 1);
      lds_barrier();
      c = s_claim;
      lds_barrier();
      continue;
    }
    int32_t next = 0;
    if (threadIdx.x == 0) next = atomicAdd(&counters[xq * QUEUE_STRIDE], 1);
    const BatchTile T = tiles[start + c];
    batch_tile<P, E, NT>(rp, col, val, T, xv, yv, s_prod);
    // LDS-only barriers: the tile's stores of C need not complete before
    // the next tile starts (each tile writes its own rows)
    if (threadIdx.x == 0) s_claim = next;
    lds_barrier();
    c = s_claim;
    lds_barrier();
  }
}

// One workgroup per tile (no counter).
template <int P, int E, bool NT>
__global__ __launch_bounds__(WG) void k_batch_flat(const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col,
                                                   const void *val,
                                                   const BatchTile *tiles, int64_t n_tiles,
                                                   const void *xv, void *yv) {
  using X = typename Ty<P>::X;
  __shared__ X s_prod[WG * E];
  const int64_t t = xcd_tile(blockIdx.x, n_tiles, 1);
  const BatchTile T = tiles[t];
  batch_tile<P, E, NT>(rp, col, val, T, xv, yv, s_prod);
}

// Batch tiles with the staged kernel's tile: one workgroup per tile, the run
// table row of tile t at runs + t * RUN_WORDS (member-local columns).
template <int P, int E, bool NT>
__global__ __launch_bounds__(WG) void k_batch_staged(const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const void *val,
                                                     const BatchTile *tiles,
                                                     const int32_t *__restrict__ runs,
                                                     int64_t n_tiles, const void *xv, void *yv) {
  using V = typename Ty<P>::V;
  using X = typename Ty<P>::X;
  __shared__ X s_prod[staged_lds_elems<P, E>()];
  const int64_t t = xcd_tile(blockIdx.x, n_tiles, 1);
  const BatchTile T = tiles[t];
  const int32_t *mrp = rp + T.rp_off;
  const TileRP m0{T.r0, T.p0}, m1{T.r1, T.p1};
  staged_tile<P, E, NT, false>(mrp, col + T.nz_off, static_cast<const V *>(val) + T.nz_off, nullptr,
                               m0, m1, (int)(T.nz_off % group_of<V>()), runs + t * RUN_WORDS,
                               static_cast<const X *>(xv) + T.x_off,
                               static_cast<X *>(yv) + T.y_off, s_prod);
}

// ---------------------------------------------------------------------------
// Dispatch helpers
// ---------------------------------------------------------------------------
template <int P, int E, bool NT, bool IND>
void launch_stream(const CsrDev &A, const PlanDev &pl, const TileRP *tiles, int64_t n_tiles, int tpw,
                   int64_t n_groups, const void *x, void *y, hipStream_t s) {
  if (tpw == 1)
    hipLaunchKernelGGL((k_stream1<P, E, NT, IND>), dim3((unsigned)n_tiles), dim3(WG), 0, s, A,
                       tiles, n_tiles, pl.xcd_remap, x, y);
  else
    hipLaunchKernelGGL((k_stream<P, E, NT, IND>), dim3((unsigned)n_groups), dim3(WG), 0, s, A,
                       tiles, n_tiles, tpw, n_groups, pl.xcd_remap, x, y);
}

template <int P, int E>
hipError_t run_stream(const CsrDev &A, const PlanDev &pl, const TileRP *tiles, int64_t n_tiles,
                      const void *x, void *y, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  const int tpw = pl.tiles_per_group < 1 ? 1 : pl.tiles_per_group;
  const int64_t n_groups = (n_tiles + tpw - 1) / tpw;
  const bool ind = A.row_ids != nullptr;
  if (pl.nontemporal) {
    if (ind) launch_stream<P, E, true, true>(A, pl, tiles, n_tiles, tpw, n_groups, x, y, s);
    else launch_stream<P, E, true, false>(A, pl, tiles, n_tiles, tpw, n_groups, x, y, s);
  } else {
    if (ind) launch_stream<P, E, false, true>(A, pl, tiles, n_tiles, tpw, n_groups, x, y, s);
    else launch_stream<P, E, false, false>(A, pl, tiles, n_tiles, tpw, n_groups, x, y, s);
  }
  return hipGetLastError();
}

template <int P, int L>
hipError_t run_vector(const CsrDev &A, const PlanDev &pl, const void *x, void *y, hipStream_t s) {
  if (A.n_rows <= 0) return hipSuccess;
  const int64_t rows_per_wg = (int64_t)(WG / L) * 8;
  const int64_t n_wg = (A.n_rows + rows_per_wg - 1) / rows_per_wg;
  if (pl.nontemporal)
    hipLaunchKernelGGL((k_vector<P, L, true>), dim3((unsigned)n_wg), dim3(WG), 0, s, A,
                       rows_per_wg, n_wg, pl.xcd_remap, x, y);
  else
    hipLaunchKernelGGL((k_vector<P, L, false>), dim3((unsigned)n_wg), dim3(WG), 0, s, A,
                       rows_per_wg, n_wg, pl.xcd_remap, x, y);
  return hipGetLastError();
}

template <int P, int E>
hipError_t run_staged(const CsrDev &A, const PlanDev &pl, const TileRP *tiles,
                      const int32_t *runs, int64_t n_tiles, const void *x, void *y,
                      hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (!runs) return hipErrorInvalidValue;
  if (A.row_ids) {
    if (pl.nontemporal)
      hipLaunchKernelGGL((k_staged<P, E, true, true>), dim3((unsigned)n_tiles), dim3(WG), 0, s, A,
                         tiles, runs, n_tiles, pl.xcd_remap, x, y);
    else
      hipLaunchKernelGGL((k_staged<P, E, false, true>), dim3((unsigned)n_tiles), dim3(WG), 0, s, A,
                         tiles, runs, n_tiles, pl.xcd_remap, x, y);
  } else {
    if (pl.nontemporal)
      hipLaunchKernelGGL((k_staged<P, E, true, false>), dim3((unsigned)n_tiles), dim3(WG), 0, s, A,
                         tiles, runs, n_tiles, pl.xcd_remap, x, y);
    else
      hipLaunchKernelGGL((k_staged<P, E, false, false>), dim3((unsigned)n_tiles), dim3(WG), 0, s,
                         A, tiles, runs, n_tiles, pl.xcd_remap, x, y);
  }
  return hipGetLastError();
}

template <int P>
hipError_t dispatch_spmv(const CsrDev &A, const PlanDev &pl, const TileRP *tiles,
                         const int32_t *runs, int64_t n_tiles, const void *x, void *y,
                         hipStream_t s) {
  if (pl.kernel == 4) {
    switch (pl.tile_items) {
      case 8: return run_staged<P, 8>(A, pl, tiles, runs, n_tiles, x, y, s);
      case 16: return run_staged<P, 16>(A, pl, tiles, runs, n_tiles, x, y, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (pl.kernel == 2) {
    switch (pl.lanes) {
      case 2: return run_vector<P, 2>(A, pl, x, y, s);
      case 4: return run_vector<P, 4>(A, pl, x, y, s);
      case 8: return run_vector<P, 8>(A, pl, x, y, s);
      case 16: return run_vector<P, 16>(A, pl, x, y, s);
      case 32: return run_vector<P, 32>(A, pl, x, y, s);
      case 64: return run_vector<P, 64>(A, pl, x, y, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (pl.tile_items) {
    case 4: return run_stream<P, 4>(A, pl, tiles, n_tiles, x, y, s);
    case 8: return run_stream<P, 8>(A, pl, tiles, n_tiles, x, y, s);
    case 16: return run_stream<P, 16>(A, pl, tiles, n_tiles, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P, int KT, int VW>
hipError_t run_block_kt(const CsrDev &A, const TileRP *tiles, int64_t n_tiles, int nt, int remap,
                        int k, int t0, const void *B, int64_t ldb, void *C, int64_t ldc,
                        double scale, hipStream_t s) {
  using X = typename Ty<P>::X;
  const X sc = static_cast<X>(scale);
  if (nt)
    hipLaunchKernelGGL((k_block<P, 4, KT, VW, true>), dim3((unsigned)n_tiles), dim3(WG), 0, s, A,
                       tiles, n_tiles, remap, k, t0, B, ldb, C, ldc, sc);
  else
    hipLaunchKernelGGL((k_block<P, 4, KT, VW, false>), dim3((unsigned)n_tiles), dim3(WG), 0, s, A,
                       tiles, n_tiles, remap, k, t0, B, ldb, C, ldc, sc);
  return hipGetLastError();
}

template <int P, int VW>
hipError_t run_block_vw(const CsrDev &A, const TileRP *tiles, int64_t n_tiles, int nt, int remap,
                        int kt, int k, int t0, const void *B, int64_t ldb, void *C, int64_t ldc,
                        double scale, hipStream_t s) {
  switch (kt) {
    case 4: return run_block_kt<P, 4, VW>(A, tiles, n_tiles, nt, remap, k, t0, B, ldb, C, ldc, scale, s);
    case 8: return run_block_kt<P, 8, VW>(A, tiles, n_tiles, nt, remap, k, t0, B, ldb, C, ldc, scale, s);
    case 16:
      return run_block_kt<P, 16, VW>(A, tiles, n_tiles, nt, remap, k, t0, B, ldb, C, ldc, scale, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P>
hipError_t dispatch_block(const CsrDev &A, const TileRP *tiles, int64_t n_tiles, int nt, int remap,
                          int kt, int k, const void *B, int64_t ldb, void *C, int64_t ldc,
                          double scale, hipStream_t s) {
  using X = typename Ty<P>::X;
  constexpr int VWIDE = sizeof(X) == 8 ? 2 : 4;
  // Wide column loads need every lane's first column aligned to VWIDE.
  const bool wide = (k % VWIDE == 0) && (ldb % VWIDE == 0) && (ldc % VWIDE == 0) &&
                    (kt % VWIDE == 0) &&
                    (reinterpret_cast<uintptr_t>(B) % (sizeof(X) * VWIDE) == 0) &&
                    (reinterpret_cast<uintptr_t>(C) % (sizeof(X) * VWIDE) == 0);
  for (int t0 = 0; t0 < k; t0 += kt) {
    hipError_t e = wide ? run_block_vw<P, VWIDE>(A, tiles, n_tiles, nt, remap, kt, k, t0, B, ldb, C,
                                                 ldc, scale, s)
                        : run_block_vw<P, 1>(A, tiles, n_tiles, nt, remap, kt, k, t0, B, ldb, C,
                                             ldc, scale, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int P, int E>
hipError_t run_persistent(const int32_t *rp, const int32_t *col, const void *val,
                          const BatchTile *tiles, int64_t n_tiles, int nt,
                          int32_t *counter, int grid, const void *x, void *y, hipStream_t s) {
  if (nt)
    hipLaunchKernelGGL((k_batch_persistent<P, E, true>), dim3(grid), dim3(WG), 0, s, rp, col, val,
                       tiles, n_tiles, counter, x, y);
  else
    hipLaunchKernelGGL((k_batch_persistent<P, E, false>), dim3(grid), dim3(WG), 0, s, rp, col, val,
                       tiles, n_tiles, counter, x, y);
  return hipGetLastError();
}

template <int P, int E>
hipError_t run_flat(const int32_t *rp, const int32_t *col, const void *val,
                    const BatchTile *tiles, int64_t n_tiles, int nt, const void *x, void *y,
                    hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (nt)
    hipLaunchKernelGGL((k_batch_flat<P, E, true>), dim3((unsigned)n_tiles), dim3(WG), 0, s, rp, col,
                       val, tiles, n_tiles, x, y);
  else
    hipLaunchKernelGGL((k_batch_flat<P, E, false>), dim3((unsigned)n_tiles), dim3(WG), 0, s, rp,
                       col, val, tiles, n_tiles, x, y);
  return hipGetLastError();
}

template <int P, int E>
int persistent_grid_for(int device) {
  int per_cu = 0, n_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent<P, E, true>, WG,
                                                   0) != hipSuccess)
    per_cu = 1;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    n_cu = 256;
  return (per_cu < 1 ? 1 : per_cu) * n_cu;
}

template <int P, int E>
hipError_t run_fused(const PanelSetDev &S, int R, int nt, int remap, const void *x, void *y,
                     hipStream_t s) {
  if (S.n_rows <= 0) return hipSuccess;
  const int64_t nb = (S.n_rows + R - 1) / R;
  if (nt)
    hipLaunchKernelGGL((k_fused<P, E, true>), dim3((unsigned)nb), dim3(WG), 0, s, S, R, nb, remap, x,
                       y);
  else
    hipLaunchKernelGGL((k_fused<P, E, false>), dim3((unsigned)nb), dim3(WG), 0, s, S, R, nb, remap, x,
                       y);
  return hipGetLastError();
}

template <int P>
hipError_t dispatch_fused(const PanelSetDev &S, int R, int items, int nt, int remap, const void *x,
                          void *y, hipStream_t s) {
  switch (items) {
    case 4: return run_fused<P, 4>(S, R, nt, remap, x, y, s);
    case 8: return run_fused<P, 8>(S, R, nt, remap, x, y, s);
    case 16: return run_fused<P, 16>(S, R, nt, remap, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

// Rows per lane group of the fused block kernel for a workgroup of at most
// want_rows rows (at least one pass of the NG lane groups).
constexpr int block_nr_for(int ng, int want_rows) {
  return want_rows >= 8 * ng ? 8 : want_rows >= 4 * ng ? 4 : want_rows >= 2 * ng ? 2 : 1;
}

template <int P, int KT, int VW, int NR>
hipError_t run_block_fused_nr(const PanelSetDev &S, int nt, int remap, int k, int t0, const void *B,
                              int64_t ldb, void *C, int64_t ldc, double scale, hipStream_t s) {
  using X = typename Ty<P>::X;
  constexpr int R = (WG / (KT / VW)) * NR;
  const int64_t nb = (S.n_rows + R - 1) / R;
  const X sc = static_cast<X>(scale);
  if (nt)
    hipLaunchKernelGGL((k_block_fused<P, 8, KT, VW, NR, true>), dim3((unsigned)nb), dim3(WG), 0, s, S,
                       nb, remap, k, t0, B, ldb, C, ldc, sc);
  else
    hipLaunchKernelGGL((k_block_fused<P, 8, KT, VW, NR, false>), dim3((unsigned)nb), dim3(WG), 0, s,
                       S, nb, remap, k, t0, B, ldb, C, ldc, sc);
  return hipGetLastError();
}

template <int P, int KT, int VW>
hipError_t run_block_fused_kt(const PanelSetDev &S, int want_rows, int nt, int remap, int k, int t0,
                              const void *B, int64_t ldb, void *C, int64_t ldc, double scale,
                              hipStream_t s) {
  switch (block_nr_for(WG / (KT / VW), want_rows)) {
    case 8: return run_block_fused_nr<P, KT, VW, 8>(S, nt, remap, k, t0, B, ldb, C, ldc, scale, s);
    case 4: return run_block_fused_nr<P, KT, VW, 4>(S, nt, remap, k, t0, B, ldb, C, ldc, scale, s);
    case 2: return run_block_fused_nr<P, KT, VW, 2>(S, nt, remap, k, t0, B, ldb, C, ldc, scale, s);
    default: return run_block_fused_nr<P, KT, VW, 1>(S, nt, remap, k, t0, B, ldb, C, ldc, scale, s);
  }
}

template <int P, int VW>
hipError_t run_block_fused_vw(const PanelSetDev &S, int want_rows, int nt, int remap, int kt, int k,
                              int t0, const void *B, int64_t ldb, void *C, int64_t ldc, double scale,
                              hipStream_t s) {
  switch (kt) {
    case 4:
      return run_block_fused_kt<P, 4, VW>(S, want_rows, nt, remap, k, t0, B, ldb, C, ldc, scale, s);
    case 8:
      return run_block_fused_kt<P, 8, VW>(S, want_rows, nt, remap, k, t0, B, ldb, C, ldc, scale, s);
    case 16:
      return run_block_fused_kt<P, 16, VW>(S, want_rows, nt, remap, k, t0, B, ldb, C, ldc, scale, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P>
bool block_wide(int kt, int k, int64_t ldb, int64_t ldc, const void *B, const void *C) {
  using X = typename Ty<P>::X;
  constexpr int VWIDE = sizeof(X) == 8 ? 2 : 4;
  return (k % VWIDE == 0) && (ldb % VWIDE == 0) && (ldc % VWIDE == 0) && (kt % VWIDE == 0) &&
         (reinterpret_cast<uintptr_t>(B) % (sizeof(X) * VWIDE) == 0) &&
         (reinterpret_cast<uintptr_t>(C) % (sizeof(X) * VWIDE) == 0);
}

template <int P>
hipError_t dispatch_block_fused(const PanelSetDev &S, int want_rows, int nt, int remap, int kt, int k,
                                const void *B, int64_t ldb, void *C, int64_t ldc, double scale,
                                hipStream_t s) {
  using X = typename Ty<P>::X;
  constexpr int VWIDE = sizeof(X) == 8 ? 2 : 4;
  const bool wide = block_wide<P>(kt, k, ldb, ldc, B, C);
  for (int t0 = 0; t0 < k; t0 += kt) {
    hipError_t e = wide ? run_block_fused_vw<P, VWIDE>(S, want_rows, nt, remap, kt, k, t0, B, ldb, C,
                                                       ldc, scale, s)
                        : run_block_fused_vw<P, 1>(S, want_rows, nt, remap, kt, k, t0, B, ldb, C,
                                                   ldc, scale, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int P>
int block_fused_rows_p(int kt, int k, int64_t ldb, int64_t ldc, const void *B, const void *C,
                       int want_rows) {
  using X = typename Ty<P>::X;
  constexpr int VWIDE = sizeof(X) == 8 ? 2 : 4;
  const int vw = block_wide<P>(kt, k, ldb, ldc, B, C) ? VWIDE : 1;
  const int ng = WG / (kt / vw);
  return ng * block_nr_for(ng, want_rows);
}

template <int P, int E, int K>
hipError_t run_sorted_blk(const SortedDev &S, int remap, const void *x, int64_t ldb, void *y,
                          int64_t ldc, int j0, int kk, double scale, hipStream_t s) {
  if (S.b1 <= S.b0) return hipSuccess;
  using X = typename Ty<P>::X;
  constexpr int VWIDE = sizeof(X) == 8 ? 2 : 4;
  const X sc = static_cast<X>(scale);
  const dim3 grid((unsigned)(S.b1 - S.b0));
  // wide column loads need every lane's first column aligned to VWIDE
  const bool wide = kk % VWIDE == 0 && ldb % VWIDE == 0 && j0 % VWIDE == 0 &&
                    reinterpret_cast<uintptr_t>(x) % (sizeof(X) * VWIDE) == 0;
  if (wide)
    hipLaunchKernelGGL((k_sorted_blk<P, E, K, VWIDE, 1>), grid, dim3(SB_WG), 0, s, S, remap, x,
                       ldb, y, ldc, j0, kk, sc);
  else
    hipLaunchKernelGGL((k_sorted_blk<P, E, K, 1, VWIDE>), grid, dim3(SB_WG), 0, s, S, remap, x,
                       ldb, y, ldc, j0, kk, sc);
  return hipGetLastError();
}

template <int P, int K>
hipError_t dispatch_sorted_blk_k(const SortedDev &S, int items, int remap, const void *x,
                                 int64_t ldb, void *y, int64_t ldc, int j0, int kk, double scale,
                                 hipStream_t s) {
  switch (items) {
    case 1: return run_sorted_blk<P, 1, K>(S, remap, x, ldb, y, ldc, j0, kk, scale, s);
    case 2: return run_sorted_blk<P, 2, K>(S, remap, x, ldb, y, ldc, j0, kk, scale, s);
    case 4: return run_sorted_blk<P, 4, K>(S, remap, x, ldb, y, ldc, j0, kk, scale, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P>
hipError_t dispatch_sorted_blk(const SortedDev &S, int items, int kt, int remap, const void *x,
                               int64_t ldb, void *y, int64_t ldc, int j0, int kk, double scale,
                               hipStream_t s) {
  switch (kt) {
    case 4: return dispatch_sorted_blk_k<P, 4>(S, items, remap, x, ldb, y, ldc, j0, kk, scale, s);
    case 8: return dispatch_sorted_blk_k<P, 8>(S, items, remap, x, ldb, y, ldc, j0, kk, scale, s);
    case 16: return dispatch_sorted_blk_k<P, 16>(S, items, remap, x, ldb, y, ldc, j0, kk, scale, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P, int E>
hipError_t run_sorted(const SortedDev &S, int nt, int remap, const void *x, void *y,
                      hipStream_t s) {
  if (S.b1 <= S.b0) return hipSuccess;
  const dim3 grid((unsigned)(S.b1 - S.b0));
  if (nt)
    hipLaunchKernelGGL((k_sorted<P, E, true>), grid, dim3(SB_WG), 0, s, S, remap, x, y);
  else
    hipLaunchKernelGGL((k_sorted<P, E, false>), grid, dim3(SB_WG), 0, s, S, remap, x, y);
  return hipGetLastError();
}

template <int P>
hipError_t dispatch_sorted(const SortedDev &S, int items, int nt, int remap, const void *x,
                           void *y, hipStream_t s) {
  switch (items) {
    case 1: return run_sorted<P, 1>(S, nt, remap, x, y, s);
    case 2: return run_sorted<P, 2>(S, nt, remap, x, y, s);
    case 4: return run_sorted<P, 4>(S, nt, remap, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

#define SPMV_PREC_SWITCH(prec, CALL) \
  switch (prec) {                    \
    case P_F64: { constexpr int PP = P_F64; return CALL; } \
    case P_F32: { constexpr int PP = P_F32; return CALL; } \
    case P_BF16: { constexpr int PP = P_BF16; return CALL; } \
    case P_F32_F64: { constexpr int PP = P_F32_F64; return CALL; } \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_spmv(int prec, const CsrDev &A, const PlanDev &plan, const TileRP *tiles,
                       const int32_t *runs, int64_t n_tiles, const void *x, void *y,
                       hipStream_t s) {
  SPMV_PREC_SWITCH(prec, (dispatch_spmv<PP>(A, plan, tiles, runs, n_tiles, x, y, s)))
}

template <int L>
hipError_t run_sym(const CsrDev &A, int nt, int remap, const double *x, double *y, hipStream_t s) {
  if (A.n_rows <= 0) return hipSuccess;
  const int64_t rows_per_wg = (int64_t)(WG / L) * 8;
  const int64_t n_wg = (A.n_rows + rows_per_wg - 1) / rows_per_wg;
  if (nt)
    hipLaunchKernelGGL((k_sym<L, true>), dim3((unsigned)n_wg), dim3(WG), 0, s, A, rows_per_wg, n_wg,
                       remap, x, y);
  else
    hipLaunchKernelGGL((k_sym<L, false>), dim3((unsigned)n_wg), dim3(WG), 0, s, A, rows_per_wg,
                       n_wg, remap, x, y);
  return hipGetLastError();
}

hipError_t launch_spmv_sym(const CsrDev &A, int lanes, int nontemporal, int xcd_remap,
                           const double *x, double *y, hipStream_t s) {
  switch (lanes) {
    case 2: return run_sym<2>(A, nontemporal, xcd_remap, x, y, s);
    case 4: return run_sym<4>(A, nontemporal, xcd_remap, x, y, s);
    case 8: return run_sym<8>(A, nontemporal, xcd_remap, x, y, s);
    case 16: return run_sym<16>(A, nontemporal, xcd_remap, x, y, s);
    case 32: return run_sym<32>(A, nontemporal, xcd_remap, x, y, s);
    case 64: return run_sym<64>(A, nontemporal, xcd_remap, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spmv_block(int prec, const CsrDev &A, const TileRP *tiles, int64_t n_tiles,
                             int tile_items, int nontemporal, int xcd_remap, int kt, int k,
                             const void *B, int64_t ldb, void *C, int64_t ldc, double scale,
                             hipStream_t s) {
  if (tile_items != 4) return hipErrorInvalidValue;
  if (n_tiles <= 0) return hipSuccess;
  SPMV_PREC_SWITCH(prec, (dispatch_block<PP>(A, tiles, n_tiles, nontemporal, xcd_remap, kt, k, B,
                                              ldb, C, ldc, scale, s)))
}

hipError_t launch_spmv_fused(int prec, const PanelSetDev &S, int R, int tile_items, int nontemporal,
                             int xcd_remap, const void *x, void *y, hipStream_t s) {
  if (R < 1 || R > 2 * WG || S.K < 1 || S.K > PANEL_MAX) return hipErrorInvalidValue;
  SPMV_PREC_SWITCH(prec, (dispatch_fused<PP>(S, R, tile_items, nontemporal, xcd_remap, x, y, s)))
}

hipError_t launch_spmv_sorted(int prec, const SortedDev &S, int tile_items, int nontemporal,
                              int xcd_remap, const void *x, void *y, hipStream_t s) {
  const int rmax = sorted_block_rows(prec);
  if (S.R < 1 || S.R > rmax || S.n_blocks != (S.n_rows + S.R - 1) / S.R || S.b0 < 0 ||
      S.b1 > S.n_blocks || S.b0 > S.b1 || S.q != sorted_chunk_slots(prec, 1, tile_items))
    return hipErrorInvalidValue;
  SPMV_PREC_SWITCH(prec, (dispatch_sorted<PP>(S, tile_items, nontemporal, xcd_remap, x, y, s)))
}

hipError_t launch_spmv_sorted_block(int prec, const SortedDev &S, int tile_items, int kt,
                                    int xcd_remap, const void *B, int64_t ldb, int j0, int kk,
                                    void *C, int64_t ldc, double scale, hipStream_t s) {
  if (kt != 4 && kt != 8 && kt != 16) return hipErrorInvalidValue;
  const int rmax = sorted_block_rows(prec) / kt;
  if (S.R < 1 || S.R > rmax || S.n_blocks != (S.n_rows + S.R - 1) / S.R || S.b0 < 0 ||
      S.b1 > S.n_blocks || S.b0 > S.b1 || S.q != sorted_chunk_slots(prec, kt, tile_items) ||
      j0 < 0 || kk < 1 || kk > kt || j0 + kk > ldb || j0 + kk > ldc)
    return hipErrorInvalidValue;
  SPMV_PREC_SWITCH(prec, (dispatch_sorted_blk<PP>(S, tile_items, kt, xcd_remap, B, ldb, C, ldc, j0,
                                                   kk, scale, s)))
}

int block_fused_rows(int prec, int kt, int k, int64_t ldb, int64_t ldc, const void *B, const void *C,
                     int want_rows) {
  if (kt != 4 && kt != 8 && kt != 16) return 0;
  SPMV_PREC_SWITCH(prec, (block_fused_rows_p<PP>(kt, k, ldb, ldc, B, C, want_rows)))
}

hipError_t launch_spmv_block_fused(int prec, const PanelSetDev &S, int want_rows, int nontemporal,
                                   int xcd_remap, int kt, int k, const void *B, int64_t ldb, void *C,
                                   int64_t ldc, double scale, hipStream_t s) {
  if (S.K < 1 || S.K > PANEL_MAX) return hipErrorInvalidValue;
  if (S.n_rows <= 0) return hipSuccess;
  SPMV_PREC_SWITCH(prec, (dispatch_block_fused<PP>(S, want_rows, nontemporal, xcd_remap, kt, k, B,
                                                    ldb, C, ldc, scale, s)))
}

hipError_t launch_batch_reset(int32_t *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, counter);
  return hipGetLastError();
}

template <int P>
static hipError_t persistent_e(const int32_t *rp, const int32_t *col, const void *val,
                               const BatchTile *tiles, int64_t n_tiles,
                               int tile_items, int nt, int32_t *counter, int grid, const void *x,
                               void *y, hipStream_t s) {
  switch (tile_items) {
    case 4: return run_persistent<P, 4>(rp, col, val, tiles, n_tiles, nt, counter, grid, x, y, s);
    case 8: return run_persistent<P, 8>(rp, col, val, tiles, n_tiles, nt, counter, grid, x, y, s);
    case 16: return run_persistent<P, 16>(rp, col, val, tiles, n_tiles, nt, counter, grid, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_persistent(int prec, const int32_t *rp, const int32_t *col, const void *val,
                                   const BatchTile *tiles, int64_t n_tiles,
                                   int tile_items, int nontemporal, int32_t *counter, int grid,
                                   const void *x, void *y, hipStream_t s) {
  SPMV_PREC_SWITCH(prec, (persistent_e<PP>(rp, col, val, tiles, n_tiles, tile_items,
                                           nontemporal, counter, grid, x, y, s)))
}

template <int P>
static hipError_t flat_e(const int32_t *rp, const int32_t *col, const void *val,
                         const BatchTile *tiles, int64_t n_tiles,
                         int tile_items, int nt, const void *x, void *y, hipStream_t s) {
  switch (tile_items) {
    case 4: return run_flat<P, 4>(rp, col, val, tiles, n_tiles, nt, x, y, s);
    case 8: return run_flat<P, 8>(rp, col, val, tiles, n_tiles, nt, x, y, s);
    case 16: return run_flat<P, 16>(rp, col, val, tiles, n_tiles, nt, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P, int E>
hipError_t run_batch_staged(const int32_t *rp, const int32_t *col, const void *val,
                            const BatchTile *tiles, const int32_t *runs,
                            int64_t n_tiles, int nt, const void *x, void *y, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (!runs) return hipErrorInvalidValue;
  if (nt)
    hipLaunchKernelGGL((k_batch_staged<P, E, true>), dim3((unsigned)n_tiles), dim3(WG), 0, s, rp,
                       col, val, tiles, runs, n_tiles, x, y);
  else
    hipLaunchKernelGGL((k_batch_staged<P, E, false>), dim3((unsigned)n_tiles), dim3(WG), 0, s, rp,
                       col, val, tiles, runs, n_tiles, x, y);
  return hipGetLastError();
}

template <int P>
static hipError_t batch_staged_e(const int32_t *rp, const int32_t *col, const void *val,
                                 const BatchTile *tiles,
                                 const int32_t *runs, int64_t n_tiles, int tile_items, int nt,
                                 const void *x, void *y, hipStream_t s) {
  switch (tile_items) {
    case 8: return run_batch_staged<P, 8>(rp, col, val, tiles, runs, n_tiles, nt, x, y, s);
    case 16: return run_batch_staged<P, 16>(rp, col, val, tiles, runs, n_tiles, nt, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_staged(int prec, const int32_t *rp, const int32_t *col, const void *val,
                               const BatchTile *tiles, const int32_t *runs,
                               int64_t n_tiles, int tile_items, int nontemporal, const void *x,
                               void *y, hipStream_t s) {
  SPMV_PREC_SWITCH(prec, (batch_staged_e<PP>(rp, col, val, tiles, runs, n_tiles, tile_items,
                                             nontemporal, x, y, s)))
}

hipError_t launch_batch_flat(int prec, const int32_t *rp, const int32_t *col, const void *val,
                             const BatchTile *tiles, int64_t n_tiles,
                             int tile_items, int nontemporal, const void *x, void *y,
                             hipStream_t s) {
  SPMV_PREC_SWITCH(prec, (flat_e<PP>(rp, col, val, tiles, n_tiles, tile_items, nontemporal,
                                     x, y, s)))
}

template <int P>
static int grid_e(int tile_items, int device) {
  switch (tile_items) {
    case 4: return persistent_grid_for<P, 4>(device);
    case 8: return persistent_grid_for<P, 8>(device);
    default: return persistent_grid_for<P, 16>(device);
  }
}

int sorted_chunk_slots(int prec, int kt, int items) {
  if (kt == 1) return SB_WG * items;
  const int vwide = sorted_block_rows(prec) == SB_LDS_BYTES / 8 ? 2 : 4;  // 8- or 4-byte sums
  return SB_WG / kt * items * vwide;
}

int sorted_block_rows(int prec) {
  switch (prec) {
    case P_F64: case P_F32_F64: return SB_LDS_BYTES / 8;
    case P_F32: case P_BF16: return SB_LDS_BYTES / 4;
    default: return 0;
  }
}

int batch_persistent_grid(int prec, int tile_items, int device) {
  switch (prec) {
    case P_F64: return grid_e<P_F64>(tile_items, device);
    case P_F32: return grid_e<P_F32>(tile_items, device);
    case P_BF16: return grid_e<P_BF16>(tile_items, device);
    default: return grid_e<P_F32_F64>(tile_items, device);
  }
}

}  // namespace spmv
