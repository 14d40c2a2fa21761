// Internal declarations shared by the host runtime (rt_*.cpp, rt_solvers.hip)
// and the gfx950 kernels (*.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace spmv {

// Element types of the four precision modes: stored value VT, vector XT
// (B and C), accumulator AT.  bfloat16 values are carried as uint16 codes.
enum Prec : int { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_F32_F64 = 3 };

inline int val_bytes(int p) { return p == P_F64 ? 8 : (p == P_BF16 ? 2 : 4); }
inline int vec_bytes(int p) { return (p == P_F64 || p == P_F32_F64) ? 8 : 4; }

// One CRS part on the device.  Row r of the part holds entries
// row_ptr[r] .. row_ptr[r+1]-1 and adds into C[row_ids ? row_ids[r] : r].
struct CsrDev {
  const int32_t *row_ptr;
  const int32_t *col;
  const void *val;
  const int32_t *row_ids;
  int64_t n_rows;
};

struct PlanDev {
  int kernel;       // 1 stream, 2 vector, 4 staged stream
  int tile_items;   // stream: products per thread (tile = 256 * tile_items)
  int lanes;        // vector: lanes per row
  int nontemporal;  // streaming hint on val / col
  int xcd_remap;    // place consecutive tiles on one XCD
  int tiles_per_group;  // stream: consecutive tiles per workgroup (software pipelined)
};

// Run table of the staged kernel: RUN_WORDS int32 per tile,
//   nr, L, s_0 .. s_3, d_0 .. d_3, 0, 0
// nr runs (1..RUN_MAX) of columns [s_r, s_r + len_r), ascending and
// disjoint, that cover every column the tile's entries read; run r fills
// LDS slots [s_r + d_r, s_r + d_r + len_r), L slots in all, at most
// RUN_STAGE_BYTES of B.  nr = 0: the tile is run as in the stream kernel.
constexpr int RUN_WORDS = 12;
constexpr int RUN_MAX = 4;
constexpr int RUN_STAGE_BYTES = 12288;

// Start of a tile: first row and first stored entry (row_ptr[r]).  A part
// with T tiles has T + 1 of these; the last one is (n_rows, nnz).
struct TileRP {
  int32_t r;
  int32_t p;
};

// Per-member offsets of a batch into the pooled arrays (host side; each tile
// carries a copy of its member's).
struct BatchDesc {
  int64_t rp_off;   // first row_ptr entry of the member (local row_ptr values)
  int64_t nz_off;   // first col / val entry
  int64_t x_off;    // first element of the member's B
  int64_t y_off;    // first element of the member's C
};

// Tile of a batch: member, row range [r0, r1) of that member and its entries
// [p0, p1) (the member's row_ptr at r0 and r1), with the member's offsets
// copied in, so a workgroup starts its tile's loads after one load of the
// tile instead of a chain of dependent loads.
struct BatchTile {
  int32_t member;
  int32_t r0;
  int32_t r1;
  int32_t p0;
  int32_t p1;
  int32_t pad;
  int64_t rp_off;
  int64_t nz_off;
  int64_t x_off;
  int64_t y_off;
};

// ---- launchers (kernels.hip) -------------------------------------------------
// All return hipSuccess or the launch error.  `tiles` (stream and block
// kernels) holds the n_tiles + 1 tile starts of `A`.
// `runs`: the run table of the tiles (staged kernel only, else unused).
hipError_t launch_spmv(int prec, const CsrDev &A, const PlanDev &plan, const TileRP *tiles,
                       const int32_t *runs, int64_t n_tiles, const void *x, void *y,
                       hipStream_t s);

// Symmetric product from the upper triangle (FP64; `lanes` a power of two in
// [2, 64]): C = C + (U + U^T - diag U) B with atomic adds into C.
hipError_t launch_spmv_sym(const CsrDev &A, int lanes, int nontemporal, int xcd_remap,
                           const double *x, double *y, hipStream_t s);

// Block product C = C + scale*A*B; `scale` is 1, or a power of two so that the
// scaled values are exact.
hipError_t launch_spmv_block(int prec, const CsrDev &A, const TileRP *tiles, int64_t n_tiles,
                             int tile_items, int nontemporal, int xcd_remap, int kt, int k,
                             const void *B, int64_t ldb, void *C, int64_t ldc, double scale,
                             hipStream_t s);

// counters: one int32 per XCD (8)
// The persistent batch grid's eight queue counters, QUEUE_STRIDE int32s
// apart (one 128-byte line each): a buffer of NXCD_QUEUES * QUEUE_STRIDE.
constexpr int QUEUE_STRIDE = 32;
constexpr int NXCD_QUEUES = 8;
hipError_t launch_batch_reset(int32_t *counters, hipStream_t s);

hipError_t launch_batch_persistent(int prec, const int32_t *rp, const int32_t *col, const void *val,
                                   const BatchTile *tiles, int64_t n_tiles,
                                   int tile_items, int nontemporal, int32_t *counter, int grid,
                                   const void *x, void *y, hipStream_t s);

hipError_t launch_batch_flat(int prec, const int32_t *rp, const int32_t *col, const void *val,
                             const BatchTile *tiles, int64_t n_tiles,
                             int tile_items, int nontemporal, const void *x, void *y, hipStream_t s);

// The staged kernel over batch tiles (tile_items 8 or 16): one workgroup per
// tile, `runs` the run table of the n_tiles batch tiles (member-local columns).
hipError_t launch_batch_staged(int prec, const int32_t *rp, const int32_t *col, const void *val,
                               const BatchTile *tiles, const int32_t *runs,
                               int64_t n_tiles, int tile_items, int nontemporal, const void *x,
                               void *y, hipStream_t s);

int batch_persistent_grid(int prec, int tile_items, int device);

// ---- split bookkeeping (split.hip) -------------------------------------------
struct SplitOut {
  int32_t *loc_row_ptr;  // [n_rows + 1]
  int32_t *loc_col;      // [nnz_loc]
  void *loc_val;         // [nnz_loc]
  int32_t *nl_rows;      // [R]
  int32_t *nl_ptr;       // [R + 1]
  int32_t *nl_col;       // [nnz_nl]
  void *nl_val;          // [nnz_nl]
};

// First pass: per-row counts and their exclusive scans into `work`
// (3 * (n_rows + 1) int32 plus scan scratch); returns the totals.
hipError_t split_count(const int32_t *row_ptr, const int32_t *col, int64_t n_rows, int32_t h,
                       int32_t *work, int32_t *scan_tmp, int64_t *nnz_loc, int64_t *nnz_nl,
                       int64_t *n_nl_rows, hipStream_t s);
int64_t split_work_elems(int64_t n_rows);
int64_t scan_tmp_elems(int64_t n);

hipError_t split_fill(int prec, const int32_t *row_ptr, const int32_t *col, const void *val,
                      int64_t n_rows, int32_t h, const int32_t *work, int64_t nnz_nl, int64_t R,
                      const SplitOut &out, hipStream_t s);

// ---- diagonal panels (split.hip) ------------------------------------------------
// Entries are grouped by their offset d = col - row into K <= PANEL_MAX equal
// slices of [dmin, dmin + span); each panel is a CRS over all rows.
constexpr int PANEL_MAX = 8;
struct PanelOut {
  int32_t *col[PANEL_MAX];
  void *val[PANEL_MAX];
};
// dev2: two int64 of device scratch.  Sets dmin / dmax of the part's offsets.
hipError_t panel_d_range(const int32_t *row_ptr, const int32_t *col, int64_t n_rows, int64_t *dev2,
                         int64_t *dmin, int64_t *dmax, hipStream_t s);
// counts: K * (n_rows + 1) int32; on return panel k's row_ptr is
// counts + k * (n_rows + 1).
hipError_t panel_count(const int32_t *row_ptr, const int32_t *col, int64_t n_rows, int64_t dmin,
                       int64_t span, int K, int32_t *counts, int32_t *scan_tmp, hipStream_t s);
hipError_t panel_fill(int prec, const int32_t *row_ptr, const int32_t *col, const void *val,
                      int64_t n_rows, int64_t dmin, int64_t span, int K, const int32_t *starts,
                      const PanelOut &out, hipStream_t s);

// ---- diagonal panels in one launch (kernels.hip) ---------------------------------
// The K diagonal panels of a part (each a CRS over all n_rows rows, see
// panel_fill) handed to one launch: a workgroup takes rows [b*R, b*R + R) and
// walks the K panels of those rows in turn, keeping the rows' sums in
// registers, so C is read and written once per call instead of once per panel.
struct PanelSetDev {
  const int32_t *rp[PANEL_MAX];
  const int32_t *col[PANEL_MAX];
  const void *val[PANEL_MAX];
  int K;
  int64_t n_rows;
};
// Sorted-block layout of a part (SPMV_KERNEL_SORTED_BLOCKS).  The rows are
// cut into blocks of R rows (at most sorted_block_rows(prec)); block b's entries, sorted
// by column, fill chunks [cs[b], cs[b+1]) of SB_WG * tile_items slots in
// which no row appears twice.  Slot s of the layout holds col[s], val[s] and
// the entry's row within its block, row[s]; an empty slot has row
// SB_PAD_ROW, val zero and a column some entry of its chunk has.
constexpr int SB_WG = 1024;
constexpr int SB_LDS_BYTES = 128 * 1024;
constexpr uint16_t SB_PAD_ROW = 0xFFFF;
struct SortedDev {
  const int64_t *cs;
  const int32_t *col;
  const void *val;
  const uint16_t *row;
  int64_t n_rows;
  int64_t n_blocks;
  int R;
  int q;           // slots per chunk (checked by the launchers)
  int64_t b0, b1;  // the launch covers blocks [b0, b1) of the n_blocks
};
// Most rows per block: their accumulators fill SB_LDS_BYTES of LDS.
int sorted_block_rows(int prec);
// tile_items 1, 2 or 4 (chunks of 1024, 2048 or 4096 slots).
hipError_t launch_spmv_sorted(int prec, const SortedDev &S, int tile_items, int nontemporal,
                              int xcd_remap, const void *x, void *y, hipStream_t s);
// Columns [j0, j0 + kk) of C += scale * A * B (row-major, kk <= kt) over a
// sorted-block layout whose chunks hold sorted_chunk_slots(prec, kt,
// tile_items) slots and whose blocks hold at most sorted_block_rows(prec) /
// kt rows.
hipError_t launch_spmv_sorted_block(int prec, const SortedDev &S, int tile_items, int kt,
                                    int xcd_remap, const void *B, int64_t ldb, int j0, int kk,
                                    void *C, int64_t ldc, double scale, hipStream_t s);
// Slots per chunk of a sorted-block layout: 1024 * items for one
// right-hand side (kt = 1); for the block form with kt columns per pass,
// the slots its wide form (2 FP64 or 4 FP32 columns per lane) takes in one
// load step per item.
int sorted_chunk_slots(int prec, int kt, int items);
// Plain product over a panel set: R <= 512 rows per workgroup, tile_items
// (4, 8, 16) entries per lane for the entries one panel holds in a row block
// (blocks holding more are summed row by row from global memory).
hipError_t launch_spmv_fused(int prec, const PanelSetDev &S, int R, int tile_items, int nontemporal,
                             int xcd_remap, const void *x, void *y, hipStream_t s);
// Block product C = C + scale*A*B over a panel set, 8 entries per lane
// staged per panel.  A workgroup takes block_fused_rows(...) consecutive
// rows: the largest supported count not above `want_rows` (at least the
// rows one pass of its lane groups covers); the host sizes want_rows so a
// panel's entries in a row block fit the 2048 staged (blocks holding more
// are summed row by row from global memory).
int block_fused_rows(int prec, int kt, int k, int64_t ldb, int64_t ldc, const void *B, const void *C,
                     int want_rows);
hipError_t launch_spmv_block_fused(int prec, const PanelSetDev &S, int want_rows, int nontemporal,
                                   int xcd_remap, int kt, int k, const void *B, int64_t ldb, void *C,
                                   int64_t ldc, double scale, hipStream_t s);


// ---- send side of the exchange (exchange.hip) -----------------------------------
// out[k] = B[idx[k]] for k < n, copying words of word_bytes (4 or 8) bytes.
hipError_t launch_pack(int word_bytes, const void *B, const int32_t *idx, int64_t n, void *out,
                       hipStream_t s);

// ---- Chebyshev moments (kpm.hip) -----------------------------------------------
// Blocks of R columns, row-major; part holds 2 * KPM_GRID * R doubles.  first:
// W1 = H v0 = z1 given, copies V0 into W2 and writes mu[0], mu[1].  step n: X = z_n,
// P = z_{n+1} given (z_n = c_n v_n, c = 1, 1, -1, -1, ...), writes mu[2n], mu[2n+1].
constexpr int KPM_GRID = 1024;
hipError_t launch_kpm_zero(double *p, int64_t n, hipStream_t s);
hipError_t launch_kpm_first(const double *V0, const double *W1, double *W2, int64_t n_rows, int R,
                            double *part, int M, double *mu, hipStream_t s);
hipError_t launch_kpm_step(const double *X, const double *P, int64_t n_rows, int R, double *part, int step,
                           int M, double *mu, hipStream_t s);

// ---- Lanczos (lanczos.hip) ---------------------------------------------------------
// part holds KPM_GRID + 1 doubles.  start: V = q / |q|.  step: with W = H v_j -
// beta_{j-1} v_{j-1} and V = v_j, writes *alpha, *beta, leaves v_{j+1} in W and
// -beta_j v_j in V.
hipError_t launch_lz_start(const double *q, double *V, int64_t n, double *part, hipStream_t s);
hipError_t launch_lz_step(double *W, double *V, int64_t n, double *part, double *alpha,
                          double *beta, hipStream_t s);

// ---- probes (probes.hip) -------------------------------------------------------
hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t s);
hipError_t launch_triad(double *a, const double *b, const double *c, double sc, int64_t n,
                        hipStream_t s);
hipError_t launch_spin(int64_t nanoseconds, hipStream_t s);
// Gather probe: for k < n, row clamp(idx[k]) of src viewed as n_rows rows of
// `width` doubles (1, 2, 4, 8 or 16); one partial sum per workgroup into sums,
// which must hold gather_sums_needed(n, width) doubles.
int64_t gather_sums_needed(int64_t n, int width);
hipError_t launch_gather(const double *src, int64_t n_rows, const int32_t *idx, int64_t n,
                         int width, int remap, double *sums, hipStream_t s);
// sums must hold read_sums_needed(n) doubles
int64_t read_sums_needed(int64_t n);
hipError_t launch_read(const double *src, int64_t n, double *sums, hipStream_t s);
// ATOMIC_BLOCKS * 256 threads each add 1.0 `iters` times into C[0, n), n a
// power of two >= 64.
constexpr int ATOMIC_BLOCKS = 2048;
hipError_t launch_atomic(double *C, int64_t n, int scattered, int iters, hipStream_t s);

}  // namespace spmv
