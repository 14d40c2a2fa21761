/*
 * libspmv -- CRS sparse matrix-vector multiplication C = C + A*B on AMD
 * Instinct MI355X (gfx950).
 *
 * The operation is the CRS kernel of Schubert, Fehske, Hager and Wellein,
 * "Hybrid-parallel sparse matrix-vector multiplication with explicit
 * communication overlap on current multicore-based systems" (2011):
 *   - storage (Sect. 1.2): val holds the stored entries row by row, row_ptr
 *     the offset of each row's first entry (N_r + 1 entries), col_idx the
 *     original column of each entry;
 *   - kernel (Listing 1): for every row i, C(i) = C(i) + sum over the row's
 *     entries j of val(j) * B(col_idx(j));
 *   - split of one process's share (Sect. 3.4): a local part that reads only
 *     the locally owned RHS elements and a nonlocal part that reads the halo
 *     elements received from other processes, applied one after the other so
 *     that the result vector is updated twice.
 *
 * Conventions shared by every entry point
 *   - Every function returns an spmv_status_t; on failure a description is
 *     available from spmv_last_error() (thread-local, valid until the next
 *     call from the same thread).  No C++ exception crosses this interface.
 *   - Host arrays passed to spmv_create_* are deep-copied; the caller may free
 *     them when the call returns.  All device memory a handle needs is owned
 *     by the handle and released by spmv_destroy.
 *   - B, C (and the block arrays) are caller-owned *device* pointers whose
 *     element type follows the handle's precision (see spmv_precision_t).
 *     C must not alias B.  The library cannot check that a device pointer is
 *     large enough: passing short buffers is undefined behaviour.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     spmv_run / spmv_run_block only enqueue work on it and return; results
 *     are visible once that stream has reached the enqueued work.
 *   - Asynchronous device faults surface at the caller's next
 *     synchronisation, not as a status from the call that enqueued them.
 *   - Different handles may be used concurrently from different threads; one
 *     handle must be used by one thread at a time.  Calls on one handle must
 *     also be ordered on the device (one stream, or streams ordered by
 *     events): a handle's internal buffers and streams serve every call.
 */
#ifndef LIBSPMV_SPMV_H
#define LIBSPMV_SPMV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spmv_handle_s *spmv_handle_t;

typedef enum spmv_status {
    SPMV_OK = 0,
    SPMV_ERR_INVALID_ARG = -1,     /* bad scalar argument or null pointer */
    SPMV_ERR_INVALID_MATRIX = -2,  /* CRS arrays violate the format */
    SPMV_ERR_ALLOC = -3,           /* device or host allocation failed */
    SPMV_ERR_HIP = -4,             /* a HIP runtime call failed */
    SPMV_ERR_UNSUPPORTED = -5,     /* valid request this handle cannot serve */
    SPMV_ERR_STATE = -6            /* destroyed or foreign handle */
} spmv_status_t;

/*
 * Storage and arithmetic precision of a handle.  Values are always given to
 * spmv_create_* as binary64 and rounded once, to nearest with ties to even,
 * into the storage type (NaN stays NaN, overflow gives +-Inf).
 *
 *   mode                    val      B and C   accumulation  bytes per entry
 *   SPMV_PREC_F64           f64      f64       f64           8 + 4
 *   SPMV_PREC_F32           f32      f32       f32           4 + 4
 *   SPMV_PREC_BF16_F32ACC   bfloat16 f32       f32           2 + 4
 *   SPMV_PREC_F32_F64ACC    f32      f64       f64           4 + 4
 */
typedef enum spmv_precision {
    SPMV_PREC_F64 = 0,
    SPMV_PREC_F32 = 1,
    SPMV_PREC_BF16_F32ACC = 2,
    SPMV_PREC_F32_F64ACC = 3
} spmv_precision_t;

/* flags for spmv_create_crs / spmv_create_sym_crs / spmv_create_batch */
#define SPMV_FLAG_ALLOW_PAGEABLE_HALO 0x1u /* accept a pageable B_halo_host (copy then loses overlap) */
#define SPMV_FLAG_NO_TUNE_CACHE 0x2u       /* ignore the persistent autotuner cache */

/* ---------------------------------------------------------------------------
 * a1: ingest (Sect. 1.2 storage; the one-time setup of Sect. 3.2)
 *
 * spmv_create_crs validates a CRS matrix, shifts it to 0-based indices,
 * encodes val into the storage precision, records row-length statistics,
 * picks a kernel plan and uploads the arrays to the current HIP device.
 *
 *   n_rows, n_cols  matrix shape, 0 <= n_rows < 2^31 - 1, 0 <= n_cols < 2^31
 *   nnz             number of stored entries, 0 <= nnz <= INT32_MAX
 *   row_ptr         host int32[n_rows + 1]; row i holds entries
 *                   row_ptr[i] - base ... row_ptr[i+1] - base - 1
 *   col_idx         host int32[nnz], columns in [base, n_cols + base)
 *   val             host double[nnz]
 *   index_base      0 or 1 (Listing 1 is written 1-based)
 *   prec            a spmv_precision_t value, passed as int32_t (any other
 *                   value gives SPMV_ERR_INVALID_ARG)
 *   flags           see above
 *   out             receives the new handle (set to NULL on failure)
 *
 * Unsorted columns, duplicate columns (summed), explicit zeros and empty rows
 * are allowed.  Errors: SPMV_ERR_INVALID_ARG for bad scalars or null
 * pointers; SPMV_ERR_INVALID_MATRIX, naming the first offending index, when
 * row_ptr[0] != base, row_ptr[n_rows] != nnz + base, row_ptr decreases, or a
 * column lies outside [base, n_cols + base).  Validation happens before any
 * device call.  SPMV_ERR_ALLOC / SPMV_ERR_HIP for device failures.
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_create_crs(int64_t n_rows, int64_t n_cols, int64_t nnz,
                              const int32_t *row_ptr, const int32_t *col_idx,
                              const double *val, int32_t index_base,
                              int32_t prec, uint32_t flags,
                              spmv_handle_t *out);

/* ---------------------------------------------------------------------------
 * a2: local / nonlocal split (Sect. 3.4; bookkeeping done once, Sect. 3.2)
 *
 * Builds, on the device, a new handle from plain handle `a` for one process's
 * share whose locally owned RHS elements are columns [0, halo_begin_col) and
 * whose halo is the column tail [halo_begin_col, n_cols):
 *   local part     every entry with column < halo_begin_col, in a CRS with
 *                  all n_rows rows (row_ptr of n_rows + 1 entries);
 *   nonlocal part  every entry with column >= halo_begin_col, for the R rows
 *                  that have one: nl_rows[R] (ascending), nl_ptr[R+1],
 *                  columns and values.
 * Entries keep their storage order and global column numbers.  `a` stays
 * valid and independent; both handles are destroyed separately.
 * Errors: SPMV_ERR_INVALID_ARG if halo_begin_col is outside [0, n_cols];
 * SPMV_ERR_UNSUPPORTED if `a` is itself a split or batch handle.
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_split_local_nonlocal(spmv_handle_t a, int64_t halo_begin_col,
                                        spmv_handle_t *out_split);

/* ---------------------------------------------------------------------------
 * a3-a7, a9: C = C + A*B (Listing 1) on `stream`.
 *
 * Plain handle: B has n_cols elements, C n_rows; B_halo_host must be NULL.
 *
 * Split handle (a4-a6): B has n_cols elements; its tail [h, n_cols) is the
 * receive area of the halo.  If B_halo_host is non-NULL it must point to
 * n_cols - h elements of pinned host memory (hipHostMalloc); they are copied
 * into B + h on the handle's own copy stream while the local-part kernel runs
 * on `stream`, and the nonlocal-part kernel runs on `stream` after the copy
 * has completed (the one-GPU analogue of the explicit overlap of Sect. 3.5).
 * Pageable memory is rejected with SPMV_ERR_INVALID_ARG unless the handle was
 * created with SPMV_FLAG_ALLOW_PAGEABLE_HALO, because a copy from pageable
 * memory does not overlap (nonblocking is not asynchronous, Sect. 3.1).  If
 * B_halo_host is NULL the tail of B is taken as already resident.  The local
 * kernel never reads B[h:].
 *
 * Batch handle (a9): B and C are the concatenation of every member's vector
 * in member order (member m's B starts at the sum of the earlier members'
 * n_cols, its C at the sum of their n_rows); B_halo_host must be NULL.  All
 * members run in one persistent launch replayed from a HIP graph.
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_run(spmv_handle_t h, const void *B, void *C,
                       const void *B_halo_host, void *stream);

/* ---------------------------------------------------------------------------
 * Send side of the exchange (Sect. 3.3: the elements another process needs
 * are gathered into one contiguous send buffer; Sect. 3.5: in task mode that
 * gather and the local part run while the communication proceeds).
 *
 * spmv_set_send_list (split handles only): send_idx[0 .. n_send) are
 * positions in B of locally owned elements, each in [0, h) with h the
 * handle's halo_begin_col, in send order; repeats are allowed.  The list is
 * copied to device memory owned by the handle; n_send = 0 clears it.  The
 * call first waits for all work on the device, since an exchange still in
 * flight may read the list it replaces.
 * Errors: SPMV_ERR_UNSUPPORTED for plain and batch handles;
 * SPMV_ERR_INVALID_ARG for n_send < 0, a NULL list with n_send > 0, or an
 * index outside [0, h) (the message names the first).
 *
 * spmv_send_list_symmetric (split handles only): sets the send list for a
 * structurally symmetric matrix to the rows i < h that hold an entry in a
 * halo column, ascending.  By symmetry these are exactly the locally owned
 * elements of B that the rows of the halo columns' owner reference.  *n_send
 * receives the count.  One-time bookkeeping (synchronous).
 *
 * spmv_run_exchange (split handles only): one exchange cycle and the
 * product, enqueued on `stream`:
 *   1. send_buf[k] = B[send_idx[k]] (the pack kernel) and the copy of
 *      send_buf to send_host, on the handle's send stream;
 *   2. B_halo_host -> B[h:], on the handle's copy stream, as spmv_run does;
 *   3. the local part on `stream`, while 1 and 2 proceed;
 *   4. the nonlocal part on `stream`, after 2;
 *   5. `stream` waits for 1, so send_host is complete once `stream` has
 *      reached the end of the call.
 * Under SPMV_SCHEDULE_SERIAL all five steps run in order on `stream`.
 * send_host holds n_send elements of the handle's vector type (f64 in the
 * F64 and F32_F64ACC modes, f32 otherwise) in pinned host memory; pageable
 * memory is rejected as for B_halo_host; it may be NULL only if n_send is 0.
 * The elements are copied bit for bit.  B_halo_host as for spmv_run.
 * Errors as for spmv_run, plus SPMV_ERR_UNSUPPORTED for non-split handles.
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_set_send_list(spmv_handle_t h, const int32_t *send_idx, int64_t n_send);
spmv_status_t spmv_send_list_symmetric(spmv_handle_t h, int64_t *n_send);
spmv_status_t spmv_run_exchange(spmv_handle_t h, const void *B, void *C,
                                const void *B_halo_host, void *send_host, void *stream);

/* ---------------------------------------------------------------------------
 * Phase timing of split handles: the one-GPU form of the paper's breakdown of
 * a process's time into communication, local and nonlocal calculation
 * (Sect. 3.3-3.5, Fig. 5).
 *
 * spmv_set_phase_timing(h, on): with on != 0, later spmv_run and
 * spmv_run_exchange calls on h record timing events at the start of the call
 * and around each phase, on the stream the phase runs on; on = 0 stops it.
 * spmv_phase_times(h, t): waits for the events of the last call and writes
 * eight times in milliseconds from that call's start:
 *   t[0], t[1] halo copy start / end      t[2], t[3] local part start / end
 *   t[4], t[5] nonlocal part start / end  t[6], t[7] send side start / end
 * (send side = pack kernel and copy of the send buffer); phases that did not
 * run give -1.  Errors: SPMV_ERR_UNSUPPORTED for non-split handles,
 * SPMV_ERR_STATE if timing is off or no call has run since it was switched
 * on, SPMV_ERR_INVALID_ARG for a NULL t.
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_set_phase_timing(spmv_handle_t h, int32_t on);
spmv_status_t spmv_phase_times(spmv_handle_t h, double *t);

/* ---------------------------------------------------------------------------
 * a8: block of k right-hand sides, C[:, t] = C[:, t] + A*B[:, t], t < k,
 * with A streamed once per column tile.  B is row-major [n_cols x ldb], C is
 * row-major [n_rows x ldc] (element (r, t) at r*ld + t), 1 <= k <= 64,
 * ldb >= k, ldc >= k.  Plain handles only (SPMV_ERR_UNSUPPORTED otherwise).
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_run_block(spmv_handle_t h, int32_t k, const void *B, int64_t ldb,
                             void *C, int64_t ldc, void *stream);

/* ---------------------------------------------------------------------------
 * Chebyshev moments of the kernel polynomial method: the polynomial-expansion
 * methods for spectral properties that the paper names among the algorithms
 * whose time goes into spMVM (Sect. 1.3).  For R start vectors v0 (the
 * columns of V0) and a matrix H whose spectrum the caller has scaled into
 * [-1, 1]:
 *   mu[m*R + r] = v0_r . T_m(H) v0_r,   m = 0 .. M-1,
 * with the Chebyshev recursion v_{n+1} = 2 H v_n - v_{n-1} (v_1 = H v0) and
 * the product relations mu_{2n} = 2 v_n.v_n - mu_0 and
 * mu_{2n+1} = 2 v_{n+1}.v_n - mu_1, so M moments cost ceil(M/2) block
 * products (the kernel of spmv_run_block with k = R).  The loop carries
 * z_n = c_n v_n with c_n = 1, 1, -1, -1, 1, 1, ...; each step is then one
 * product accumulating in place, z_{n+1} = z_{n-1} + (+-2 H) z_n, with the
 * values scaled by +-2 as they are staged (exact), and one read-only pass for
 * the two dot products.
 *
 * h: plain SPMV_PREC_F64 handle of a square matrix.  R: a power of two in
 * [1, 64].  1 <= M <= 2^20.  V0, W1, W2: device blocks of n_rows x R
 * doubles, row-major (element (i, r) at i*R + r); V0 is read only, W1 and W2
 * are work space overwritten by the call (on return they hold the last two
 * vectors of the recursion, each possibly negated).  mu: device array of M*R doubles.
 * Everything is enqueued on `stream`; the dot products are reduced in a fixed
 * order, so repeated calls give identical moments.  The handle keeps a small
 * device buffer of partial sums (grown on the first call with a larger R,
 * after a device synchronisation).
 * Errors: SPMV_ERR_UNSUPPORTED for split, batch or non-F64 handles;
 * SPMV_ERR_INVALID_ARG for a non-square matrix, R or M out of range, null or
 * equal buffers.
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_kpm_moments(spmv_handle_t h, int32_t R, int32_t M, const double *V0,
                               double *W1, double *W2, double *mu, void *stream);

/* ---------------------------------------------------------------------------
 * Lanczos: the iterative eigensolver the paper names first among the
 * algorithms whose time goes into spMVM (Sect. 1.3), in its plain three-term
 * form without reorthogonalisation:
 *   v_1 = q / |q|, beta_0 = 0, and for j = 1 .. m
 *   w = H v_j - beta_{j-1} v_{j-1}, alpha_j = w.v_j, w = w - alpha_j v_j,
 *   beta_j = |w|, v_{j+1} = w / beta_j (0 once beta_j = 0).
 * alpha[j-1] = alpha_j and beta[j-1] = beta_j, both written to device memory;
 * the tridiagonal matrix of the m steps has diagonal alpha[0 .. m-1] and
 * off-diagonal beta[0 .. m-2], whose eigenvalues (computed by the caller)
 * approximate the extreme eigenvalues of H.  One product (spmv_run's kernel
 * and plan) per step; everything is enqueued on `stream`, and dot products
 * and norms are reduced in a fixed order, so repeated runs agree bit for bit.
 *
 * h: plain SPMV_PREC_F64 handle of a square matrix (symmetric for the method
 * to make sense).  1 <= m <= 2^20.  q: start vector, n_rows doubles on the
 * device (read only); V1, V2: device work vectors of n_rows doubles,
 * overwritten; alpha, beta: device arrays of m doubles.  The handle's small
 * reduction buffer is shared with spmv_kpm_moments (allocated on first use,
 * after a device synchronisation).
 * Errors: SPMV_ERR_UNSUPPORTED for split, batch or non-F64 handles;
 * SPMV_ERR_INVALID_ARG for a non-square matrix, m out of range, null or
 * equal buffers.
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_lanczos(spmv_handle_t h, int32_t m, const double *q, double *V1, double *V2,
                           double *alpha, double *beta, void *stream);

/* ---------------------------------------------------------------------------
 * spmv_lanczos_noalloc: spmv_lanczos for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as spmv_lanczos, computed
 * by the same kernels; the call makes no allocation and no device
 * synchronisation, only enqueues work on `stream`.
 *
 * Its reductions keep their partial sums in a scratch array the library
 * holds in device memory for the life of the process, one per GPU, of
 * 2 * 1024 doubles (16 KiB).  The reductions use at most 1024 workgroups for
 * any n, so they need 1025 of those doubles whatever the matrix size; a build
 * whose reductions needed more than the array holds would fail with
 * SPMV_ERR_UNSUPPORTED.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (on streams not ordered with each other) race
 * and give wrong coefficients; order them on one stream or with events.  The
 * array's contents are overwritten by every call before they are read; each
 * call leaves its last partial sums there.
 * The product uses the kernels, tiles and panels prepared when the handle's
 * plan was set (spmv_create_crs, spmv_set_plan, spmv_tune); if they are not
 * there the call fails with SPMV_ERR_STATE instead of building them.
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_lanczos_noalloc(spmv_handle_t h, int32_t m, const double *q, double *V1,
                                   double *V2, double *alpha, double *beta, void *stream);

/* Releases a handle and its device memory after waiting for the handle's
 * internal copy stream.  spmv_destroy(NULL) is SPMV_OK; a destroyed or
 * foreign handle gives SPMV_ERR_STATE. */
spmv_status_t spmv_destroy(spmv_handle_t h);

/* Description of the last failure on the calling thread ("" if none). */
const char *spmv_last_error(void);

/* ---------------------------------------------------------------------------
 * a9: batch of independent products C_m = C_m + A_m * B_m (setup).
 *
 * count members; member m is given exactly as to spmv_create_crs by
 * n_rows[m], n_cols[m], nnz[m], row_ptr[m], col_idx[m], val[m].  All members
 * share index_base, prec and flags.  The members' arrays are pooled in one
 * device allocation and cut into tiles of bounded nonzero count; spmv_run
 * walks the tile queue with one persistent launch.  Errors as for
 * spmv_create_crs, naming the member.
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_create_batch(int32_t count, const int64_t *n_rows, const int64_t *n_cols,
                                const int64_t *nnz, const int32_t *const *row_ptr,
                                const int32_t *const *col_idx, const double *const *val,
                                int32_t index_base, int32_t prec, uint32_t flags,
                                spmv_handle_t *out);

/* ---------------------------------------------------------------------------
 * Symmetric storage: the upper triangle only, the variant Sect. 1.3.1
 * describes for symmetric matrices and sets aside, because the transposed
 * half of the product writes into entries of C that other rows (other
 * threads) also write.
 *
 * row_ptr / col_idx / val: the upper triangle U of a symmetric n x n matrix
 * A in CRS, as for spmv_create_crs (index_base, duplicates and empty rows as
 * there), with every column at or right of its row (col >= row).  spmv_run on
 * the handle computes C = C + A*B with A = U + U^T - diag(U): each stored
 * entry a_ij adds a_ij * B[j] to C[i] and, for j != i, a_ij * B[i] to C[j].
 * The additions into C are device-scope atomic adds, so their order, and the
 * rounding of C, may differ from call to call; B and C are as for plain
 * handles.  Plans: SPMV_KERNEL_VECTOR only (`lanes` lanes per row, the
 * streaming hint, the XCD remap); spmv_tune searches them.  Other entry
 * points (split, block, batch, moments, Lanczos) return
 * SPMV_ERR_UNSUPPORTED for symmetric handles.
 * Errors: as spmv_create_crs; SPMV_ERR_INVALID_MATRIX for an entry left of
 * the diagonal; SPMV_ERR_UNSUPPORTED for a precision other than
 * SPMV_PREC_F64.
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_create_sym_crs(int64_t n, int64_t nnz, const int32_t *row_ptr,
                                  const int32_t *col_idx, const double *val, int32_t index_base,
                                  int32_t prec, uint32_t flags, spmv_handle_t *out);

/* ---------------------------------------------------------------------------
 * a10: kernel plans and the autotuner.
 *
 * A plan says how rows are mapped to the GPU for one part of a handle
 * (SPMV_PART_MAIN: the whole matrix, the local part of a split handle, or
 * every member of a batch; SPMV_PART_NONLOCAL: the nonlocal part).
 *   kernel       SPMV_KERNEL_STREAM: rows are grouped into tiles of at most
 *                256 * tile_items stored entries; a 256-thread workgroup
 *                streams a tile's val and col_idx with coalesced loads, forms
 *                the products in LDS and reduces each row there.  For batch
 *                handles: a persistent grid drains per-XCD tile queues.
 *                SPMV_KERNEL_VECTOR: `lanes` lanes of a wavefront share one
 *                row and reduce it with cross-lane shuffles (not for batches).
 *                SPMV_KERNEL_TILE_GRID: batch handles only; one workgroup per
 *                tile of the whole batch in a single launch.
 *                SPMV_KERNEL_STAGED: the stream kernel's tiles, with the
 *                columns each tile reads merged into at most four runs
 *                (gaps of up to 16 columns filled) that the workgroup loads
 *                into LDS (up to 12 KB of B) before its val and col_idx, so
 *                the entries read B from LDS; a tile whose columns do not
 *                fit is run as in the stream kernel.  Stencil-like
 *                matrices, whose tiles read a few contiguous column ranges,
 *                gain; the run table (48 bytes per tile) is built on the host
 *                from a copy of col_idx read back once.  For batch handles:
 *                one workgroup per batch tile, as SPMV_KERNEL_TILE_GRID.
 *                SPMV_KERNEL_FUSED_PANELS: the diagonal panels of the plan
 *                (`panels`, 1 to 8) walked by one launch: a workgroup takes
 *                up to 512 consecutive rows and, panel after panel, streams
 *                that panel's entries of its rows as the stream kernel does,
 *                keeping the rows' sums in registers, so C is read and
 *                written once per call however many panels there are (parts
 *                that cover all rows; not for split nonlocal parts, batches or
 *                symmetric handles).  In a block plan (spmv_get_block_plan)
 *                the same walk with the block kernel's column layout.
 *                SPMV_KERNEL_SORTED_BLOCKS: the rows are cut into blocks of
 *                up to 16384 rows (FP64 accumulation) or 32768 (FP32),
 *                sized so that a part of about a full round or more (one
 *                block per CU) comes in whole rounds; a
 *                1024-thread workgroup takes one block, whose entries the
 *                library has sorted by column (each block's sweep starting at
 *                a column common to the blocks that run together) and dealt
 *                into chunks of 1024 * tile_items entries in which no row
 *                appears twice,
 *                and adds each entry's product to its row's sum in LDS, chunk
 *                after chunk; C is read and written once.  The lanes of one
 *                load gather neighbouring columns of B, so matrices whose
 *                rows gather from scattered columns (a wide band) gain.  The
 *                row sums are formed in a fixed order: the same result on
 *                every call.  The layout (column, value and a 2-byte row per
 *                entry, empty slots padded) is built on the host when the
 *                plan is set, from a copy of col_idx and val read back once.
 *                For parts that cover all rows (not split nonlocal parts,
 *                batches or symmetric handles); SPMV_ERR_UNSUPPORTED when a
 *                block's longest row would make the layout more than about
 *                four slots per entry.  Block products use the block kernel,
 *                unless block_kt is set: then they run a block form of this
 *                kernel, with block_kt columns of B per pass, R * block_kt
 *                sums per block in LDS (R at most 16384 / block_kt rows in
 *                FP64 and F32/F64, 32768 / block_kt in F32 and BF16), and
 *                block_kt / VW lanes per slot, each gathering VW adjacent
 *                columns of the slot's row of B in one 16-byte load (VW 2
 *                for 8-byte B, 4 for 4-byte B; 1, walking each chunk in VW
 *                pieces, when B's leading dimension, the pass's width or
 *                B's address do not allow it); chunks of
 *                (1024 * VW / block_kt) * tile_items slots.  Its layout is
 *                streamed with the nontemporal hint whatever the plan says,
 *                and built when the plan is set.  A plan whose layout is
 *                refused is not kept.
 *   tile_items   4, 8 or 16 (stream and fused-panel kernels); 8 or 16 (staged);
 *                1, 2 or 4 (sorted-block kernel)
 *   lanes        2, 4, 8, 16, 32 or 64 (vector kernel)
 *   nontemporal  1: val and col_idx are loaded with the streaming hint so
 *                they do not displace B from the caches
 *   xcd_remap    1: consecutive tiles are placed on the same XCD (each of
 *                MI355X's eight XCDs has its own L2)
 *   block_kt     columns of B processed per pass by spmv_run_block (4, 8,
 *                16); 0 lets the library choose
 *   tiles_per_group  stream kernel: consecutive tiles handled by one
 *                workgroup (1..64); with more than one, the next tile's
 *                val / col_idx loads are issued while the current tile is
 *                reduced (software pipelining)
 *   panels       1, 2, 4 or 8: the entries of a part that covers all rows are
 *                grouped by their offset from the diagonal (col - row) into
 *                this many equal slices, each a CRS applied in turn, so the
 *                window of B one slice gathers from is that many times
 *                narrower and can stay in the L2 cache (1 for the
 *                sorted-block kernel)
 * ------------------------------------------------------------------------- */
#define SPMV_KERNEL_STREAM 1
#define SPMV_KERNEL_VECTOR 2
#define SPMV_KERNEL_TILE_GRID 3
#define SPMV_KERNEL_STAGED 4
#define SPMV_KERNEL_FUSED_PANELS 5
#define SPMV_KERNEL_SORTED_BLOCKS 6
#define SPMV_PART_MAIN 0
#define SPMV_PART_NONLOCAL 1

typedef struct spmv_plan {
    int32_t kernel;
    int32_t tile_items;
    int32_t lanes;
    int32_t nontemporal;
    int32_t xcd_remap;
    int32_t block_kt;
    int32_t tiles_per_group;
    int32_t panels;
} spmv_plan_t;

spmv_status_t spmv_get_plan(spmv_handle_t h, int32_t part, spmv_plan_t *plan);
spmv_status_t spmv_set_plan(spmv_handle_t h, int32_t part, const spmv_plan_t *plan);

/* The plan spmv_run_block uses for blocks of k columns on plain handle h: the
 * one spmv_tune chose for this k, else the persistent cache's, else the main
 * part's plan (with block_kt = 4, 8 or 16 by k if it has none).  Its kernel
 * (the block kernel, the fused-panel walk, or the sorted-block kernel's block
 * form with tile_items), block_kt, nontemporal, xcd_remap and panels fields
 * apply.  Errors: SPMV_ERR_UNSUPPORTED for other handles, SPMV_ERR_INVALID_ARG
 * for k outside [1, 64] or a NULL plan. */
spmv_status_t spmv_get_block_plan(spmv_handle_t h, int32_t k, spmv_plan_t *plan);

/* Times candidate plans for every part of `h` (block products when k > 1)
 * on scratch vectors, keeps the fastest, and records it in the persistent
 * cache (file named by SPMV_TUNE_CACHE, default $HOME/.cache/libspmv_tune.json)
 * keyed by device, precision, k and the row-length statistics.  On a split
 * handle whose schedule the caller has not set (spmv_set_schedule), it also
 * times SPMV_SCHEDULE_OVERLAP against SPMV_SCHEDULE_OVERLAP_NONLOCAL and,
 * with a sorted-block local plan, SPMV_SCHEDULE_OVERLAP_MERGED, with the
 * plans chosen (halo resident), and keeps the fastest other schedule if it is
 * at least 1% faster than OVERLAP; the schedule is not cached.  Synchronous. */
spmv_status_t spmv_tune(spmv_handle_t h, int32_t k, void *stream);

/* ---------------------------------------------------------------------------
 * Introspection (for tests and tools).
 * ------------------------------------------------------------------------- */
#define SPMV_KIND_PLAIN 0
#define SPMV_KIND_SPLIT 1
#define SPMV_KIND_BATCH 2
#define SPMV_KIND_SYMMETRIC 3

typedef struct spmv_info {
    int32_t kind;          /* SPMV_KIND_* */
    int32_t precision;     /* spmv_precision_t */
    int64_t n_rows, n_cols, nnz;
    int64_t halo_begin;    /* split: first halo column; else n_cols */
    int64_t nnz_local, nnz_nonlocal, n_nonlocal_rows;
    int32_t batch_count;   /* batch: members; else 1 */
    int64_t n_tiles;       /* stream-kernel tiles of the main part (chunks
                              for a sorted-block plan) */
    double row_len_mean, row_len_cv;
    int64_t row_len_max;
    int64_t n_send;        /* split: entries of the send list; else 0 */
    int64_t n_staged_tiles; /* staged plan of the main part: tiles that read B
                               from LDS (the rest gather); else 0 */
} spmv_info_t;

spmv_status_t spmv_get_info(spmv_handle_t h, spmv_info_t *info);

/* Copies one of the handle's device arrays to host memory `dst` of `bytes`
 * bytes (synchronous).  If dst is NULL only *size_bytes is set.
 *   SPMV_ARR_ROW_PTR, _COL, _VAL: the matrix (split: the local part), 0-based,
 *     val in storage precision (f64, f32 or bfloat16 codes as uint16);
 *   SPMV_ARR_NL_ROWS, _NL_PTR, _NL_COL, _NL_VAL: the nonlocal part;
 *   SPMV_ARR_SEND_IDX: the send list (int32);
 *   SPMV_ARR_TILES: the main part's tiles for its plan's tile_items,
 *     n_tiles + 1 pairs (first row, first entry) of int32;
 *   SPMV_ARR_RUNS: its run table when the plan is SPMV_KERNEL_STAGED without
 *     panels: 12 int32 per tile, nr, L, s_0..s_3, d_0..d_3, 0, 0 -- nr runs of
 *     columns [s_r, s_r + len_r) (nr = 0: the tile gathers from B), run r in
 *     LDS slots s_r + d_r .. s_r + d_r + len_r - 1, L slots in all. */
#define SPMV_ARR_ROW_PTR 0
#define SPMV_ARR_COL 1
#define SPMV_ARR_VAL 2
#define SPMV_ARR_NL_ROWS 3
#define SPMV_ARR_NL_PTR 4
#define SPMV_ARR_NL_COL 5
#define SPMV_ARR_NL_VAL 6
#define SPMV_ARR_SEND_IDX 7
#define SPMV_ARR_TILES 8
#define SPMV_ARR_RUNS 9

spmv_status_t spmv_export(spmv_handle_t h, int32_t which, void *dst, int64_t bytes,
                          int64_t *size_bytes);

/* ---------------------------------------------------------------------------
 * Measurement probes (the GPU stand-ins for the STREAM benchmark of Sect. 2;
 * buffers must be 16-byte aligned
 * and the asynchrony test of Listing 2 / Sect. 3.1).
 *   spmv_probe_copy   dst[i] = src[i] for n doubles
 *   spmv_probe_triad  a[i] = b[i] + s * c[i] for n doubles
 *   spmv_probe_read   reads n doubles (n even contributes all of them; an odd
 *                     last one is skipped) and writes one partial sum per
 *                     workgroup to sums[0 .. (n/2 + 1023)/1024]; sums_len is
 *                     the capacity of sums in doubles
 *   spmv_probe_gather the indexed loads of the product alone: for k < n, the
 *                     `width` doubles of row idx[k] of src (viewed as n_rows
 *                     rows of width doubles, row-major; width 1 is one
 *                     right-hand side, width k a block of k) are loaded and
 *                     summed, the indices read with coalesced loads first;
 *                     indices outside [0, n_rows) are clamped into it.
 *                     xcd_remap places the index stream on the XCDs as the
 *                     stream kernel places its tiles.  One partial sum per
 *                     workgroup goes to sums[0 .. spmv_probe_gather_sums_needed
 *                     (n, width)); sums_len is its capacity.  With a matrix's
 *                     col_idx as idx it measures what the product's gathers
 *                     of B cost on their own (the source of kappa, Eq. (1));
 *                     with random indices in a window, the gather rate of the
 *                     cache level the window fits.  width > 1 needs src
 *                     16-byte aligned.
 *   spmv_probe_spin   one wavefront waits `nanoseconds` on the GPU's constant-rate
 *                     clock without touching memory (at most 10 s)
 *   spmv_probe_atomic 524288 threads each add 1.0 `iters` times (1 <= iters <=
 *                     4096) into C[0, n) with FP64 atomics, n a power of two in
 *                     [64, 2^31]; scattered = 0: each wavefront's 64 lanes hit
 *                     64 consecutive elements, 1: hashed positions.  The sum
 *                     of C grows by exactly 524288 * iters.
 * ------------------------------------------------------------------------- */
spmv_status_t spmv_probe_copy(double *dst, const double *src, int64_t n, void *stream);
spmv_status_t spmv_probe_triad(double *a, const double *b, const double *c, double s,
                               int64_t n, void *stream);
spmv_status_t spmv_probe_read(const double *src, int64_t n, double *sums, int64_t sums_len,
                              void *stream);
spmv_status_t spmv_probe_gather(const double *src, int64_t n_rows, int32_t width,
                                const int32_t *idx, int64_t n, int32_t xcd_remap, double *sums,
                                int64_t sums_len, void *stream);
/* Capacity spmv_probe_gather needs in sums (-1 for a bad n or width). */
int64_t spmv_probe_gather_sums_needed(int64_t n, int32_t width);
spmv_status_t spmv_probe_spin(int64_t nanoseconds, void *stream);
spmv_status_t spmv_probe_atomic(double *C, int64_t n, int32_t scattered, int32_t iters,
                                void *stream);

/* Schedule used by spmv_run (for measurement and for callers that need it).
 * Split handles:
 *   SPMV_SCHEDULE_OVERLAP       halo copy on the copy stream beside the local
 *                               kernel, then the nonlocal kernel on `stream`
 *                               (default)
 *   SPMV_SCHEDULE_OVERLAP_NONLOCAL  as OVERLAP, and the nonlocal kernel runs on
 *                               the handle's nonlocal stream beside the local
 *                               rows above the first row that has a nonlocal
 *                               entry, as soon as the halo is in; the
 *                               remaining local rows follow on `stream` (local
 *                               plans of the stream or staged kernel).  With a
 *                               sorted-block local plan the blocks above the
 *                               first nonlocal row run on `stream`, and on the
 *                               nonlocal stream the nonlocal kernel runs beside
 *                               them once the halo is in, followed there by
 *                               the blocks that hold nonlocal rows.  Other
 *                               local plans run as OVERLAP
 *   SPMV_SCHEDULE_OVERLAP_MERGED  sorted-block local plans: the blocks above
 *                               the first row that has a nonlocal entry run
 *                               on `stream` beside the halo copy; the blocks
 *                               from that row on run, as soon as the halo is
 *                               in, on the nonlocal stream over their rows'
 *                               local and nonlocal entries together (a second
 *                               layout of those blocks, built when the
 *                               schedule or the plan is set), and no separate
 *                               nonlocal kernel runs.  Each row's sum still
 *                               holds its local and nonlocal products, in the
 *                               merged layout's chunk order (deterministic).
 *                               Other local plans, or a merged layout refused
 *                               for rows too long, run as OVERLAP
 *   SPMV_SCHEDULE_SERIAL        halo copy, local and nonlocal kernels in order
 *                               on `stream` (split without asynchrony)
 * Batch handles:
 *   SPMV_SCHEDULE_BATCH_GRAPH   counter reset + persistent launch replayed from
 *                               a HIP graph captured per (B, C) (default)
 *   SPMV_SCHEDULE_BATCH_DIRECT  the same two launches without a graph
 *   SPMV_SCHEDULE_BATCH_FLAT    one workgroup per tile, no counter */
#define SPMV_SCHEDULE_OVERLAP 0
#define SPMV_SCHEDULE_SERIAL 1
#define SPMV_SCHEDULE_BATCH_GRAPH 0
#define SPMV_SCHEDULE_BATCH_DIRECT 2
#define SPMV_SCHEDULE_BATCH_FLAT 3
#define SPMV_SCHEDULE_OVERLAP_NONLOCAL 4
#define SPMV_SCHEDULE_OVERLAP_MERGED 5
spmv_status_t spmv_set_schedule(spmv_handle_t h, int32_t schedule);

#ifdef __cplusplus
}
#endif

#endif /* LIBSPMV_SPMV_H */
