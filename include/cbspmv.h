/*
 * cbspmv.h -- C ABI of the CB-SpMV library for AMD Instinct MI355X (gfx950).
 *
 * The library converts a CSR matrix into the two-level tile structure of
 * CB-SpMV (Cong et al., ICS '25) and multiplies it with dense vectors on the
 * GPU:
 *   - uniform 16 x 16 sub-blocks ("tiles"; 8 x 8 on request) located by a
 *     high-level COO of tiles: blk_row_idx, blk_col_idx, nnz_per_blk,
 *     vp_per_blk, type_per_blk (Section 3.1);
 *   - every tile's packed 4+4-bit coordinates, padding and values stored side
 *     by side in one byte buffer and found through its virtual pointer
 *     (Section 3.2);
 *   - block-aware column aggregation, chosen by the th0 rule, and per-tile
 *     COO / CSR / Dense format selection by th1 / th2 (Section 3.3);
 *   - inter-thread-block load balance (Section 3.4, Algorithm 2), plus a
 *     panel-contiguous nnz-balanced split that keeps every panel of tile rows in
 *     one work unit where it can;
 *   - y = alpha * A * x + beta * y (Section 3.5 kernels, Algorithms 3 and 4)
 *     and the k-right-hand-side form Y = alpha * A * X + beta * Y.
 *
 * Conventions shared by every entry point
 *   - Every call returns a cb_status_t.  Out-parameters are written only on
 *     CB_SUCCESS.  No exception or abort crosses the ABI.  A thread-local
 *     message for the last failure is available from cb_last_error().
 *   - "stream" is a hipStream_t passed as void*; NULL is the null stream.
 *   - Host arrays given to cb_create / cb_create_host are read during the call
 *     and copied; the caller may free them on return.
 *   - A handle owns all device memory of one converted matrix; cb_destroy
 *     releases it.  After creation a handle is read-only, so several streams
 *     may use it at once; the caller must synchronise those streams before
 *     cb_destroy.
 *   - Vectors x, y, X, Y are caller-owned DEVICE pointers.  cb_spmv and
 *     cb_spmm never allocate and never synchronise: they only enqueue work on
 *     the stream, so they may be captured in a HIP graph.
 *   - Index limits: 0 <= m, n < 2^31 and 0 <= nnz < 2^31.
 */
#ifndef CBSPMV_H
#define CBSPMV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cb_matrix_s *cb_matrix_t;

typedef enum {
    CB_SUCCESS = 0,
    CB_ERROR_INVALID_VALUE = 1,   /* bad argument or non-canonical CSR */
    CB_ERROR_OUT_OF_MEMORY = 2,   /* host or device allocation failed */
    CB_ERROR_HIP = 3,             /* a HIP runtime call or kernel launch failed */
    CB_ERROR_NOT_SUPPORTED = 4,   /* valid request this build cannot serve */
    CB_ERROR_INTERNAL = 5
} cb_status_t;

/* Storage precision of the matrix values (the paper evaluates FP64,
 * Section 4.2).  F64: x and y are double, FP64 arithmetic.  F32 / BF16:
 * values rounded to nearest-even straight from the FP64 input at creation,
 * x and y are float, products in FP32, row sums in FP32 (at least: the
 * streaming SpMV kernel keeps them in FP64 by default, see row_reduce),
 * alpha and beta applied in FP32 -- or, with the vector_f64 option, x and y
 * double and all arithmetic in FP64 on the widened stored values. */
typedef enum { CB_VALUE_F64 = 0, CB_VALUE_F32 = 1, CB_VALUE_BF16 = 2 } cb_value_t;

/* Tile formats (Section 3.3.2). */
typedef enum { CB_FMT_COO = 0, CB_FMT_CSR = 1, CB_FMT_DENSE = 2 } cb_format_t;

/* How tiles are grouped into the units of work the kernel hands to one
 * wavefront.
 *   CB_LB_NONE:       natural order (panel, then column), fixed groups of
 *                     quantum_tiles tiles -- the structure without load
 *                     balance.
 *   CB_LB_PAPER:      Algorithm 2 (Section 3.4): tiles sorted by nnz, each
 *                     given to the least-loaded group of quantum_tiles tiles
 *                     (min-heap), metadata permuted into group order.
 *   CB_LB_CONTIGUOUS: natural order cut into ranges of about wave_nnz
 *                     non-zeros at panel boundaries; only panels heavier than
 *                     twice that are split.  The default: a panel inside one
 *                     range is written to y once, with no atomics.
 *   CB_LB_PAPER_STREAM: Algorithm 2's groups as CB_LB_PAPER, with the packed
 *                     tiles re-laid in group order so that a wavefront streams
 *                     runs of consecutive groups (about wave_nnz non-zeros) as
 *                     one contiguous byte range; every tile's rows are added
 *                     into y with atomics after a y <- beta*y pre-pass (the
 *                     quad kernel in scatter form).  16 x 16 tiles only; SpMM
 *                     runs the tile-at-a-time kernel of Algorithm 2's order. */
typedef enum { CB_LB_NONE = 0, CB_LB_PAPER = 1, CB_LB_CONTIGUOUS = 2, CB_LB_PAPER_STREAM = 3 } cb_lb_t;

typedef struct {
    uint32_t struct_size;   /* sizeof(cb_options_t): set by cb_options_default */
    int32_t value_type;     /* cb_value_t, default CB_VALUE_F64 */
    int32_t col_agg;        /* -1: th0 rule of Section 3.3.1 (default); 0: off; 1: on */
    int32_t th1;            /* COO below th1 non-zeros (default 32, Section 3.3.2) */
    int32_t th2;            /* Dense above th2 non-zeros (default 128, Section 3.3.2) */
    int32_t quantum_tiles;  /* tiles per group for CB_LB_NONE / CB_LB_PAPER (default 8, Algorithm 2) */
    int32_t lb_mode;        /* cb_lb_t, default CB_LB_CONTIGUOUS */
    int32_t host_threads;   /* converter threads; 0 = all hardware threads */
    double th0;             /* super-sparse share that turns aggregation on (default 0.15) */
    int64_t wave_nnz;       /* target non-zeros per wavefront work range; 0 = automatic (about 5120
                               ranges, each of at least 256 non-zeros and at most about 18 KB of codes
                               and values: 2048 FP64 entries, 3686 FP32, 4096 BF16; where that
                               cap binds and the XCDs do not take an eighth of the ranges each
                               (xcd_chunk 0), CB_LB_CONTIGUOUS ranges shrink over the last stretch
                               of the matrix to about the remaining work / 2560, down to a quarter
                               of the cap, so the last wavefronts finish close together).  An explicit
                               value so large that one range's packed tiles would span 2 GiB or
                               more is refused by cb_create with CB_ERROR_INVALID_VALUE (the
                               streaming kernel addresses a range with 32-bit offsets) */
    int32_t row_reduce;     /* how the streaming SpMV kernel sums a pass's products into row
                               accumulators: 0 = one LDS atomic add per entry; 1 = a DPP segmented
                               scan over lanes of the same (tile, row), then one add per run;
                               2 = one FP64 LDS atomic add per entry (FP32/BF16 values: row sums
                               kept in FP64 until written; same as 0 for FP64); 3 and 4 = 0 and 2
                               with the accumulators in two copies, odd lanes adding into the
                               second (halves the collisions of a row's neighbouring entries on
                               one LDS address); -1 (default) = automatic: 0 (FP64 values) or 2
                               (FP32/BF16), or 3 or 4 for the streaming kernel where the tiles'
                               rows hold their entries in runs of two or more on average (the quad
                               kernel, which sums a lane's row runs in registers, keeps 0 or 2).
                               Results agree within the storage
                               precision's tolerance either way. */
    int32_t vector_f64;     /* FP32/BF16 storage only: 1 = x and y are double and the products,
                               sums, alpha and beta are FP64 (the stored values widened exactly);
                               0 (default) = x and y are float.  FP64 storage: always double. */
    int32_t spmv_kernel;    /* natural-order SpMV kernel: 0 = entries per lane across a batch's tiles
                               (the streaming kernel); 1 = rows per lane, four 16-lane groups each
                               walking its panels' tiles; 2 = quads per lane (four consecutive
                               entries of one tile per lane, codes and values loaded straight into
                               registers; row_reduce 1 then means 0, each lane summing its own row
                               runs; it addresses x with 32-bit byte offsets, so 2 with more than
                               2^29 - 16 columns is refused with CB_ERROR_NOT_SUPPORTED, as is
                               lb_mode CB_LB_PAPER_STREAM, which runs it); -1 (default) = automatic:
                               2 where the tiles hold 32 or more entries on average, their rows
                               hold runs of two or more entries and n allows it, else 0 */
    int32_t tile_dim;       /* sub-block size S (Section 3.1 fixes 16): 0 (default) or 16 = 16 x 16
                               tiles, 8 = 8 x 8 tiles (panels of 8 rows, the same one-byte (row,
                               column) codes, 8 one-byte row starts per CSR tile, 64 values and an
                               8-byte bitmap per Dense tile; th1 / th2 apply as given, so th2 >= 64
                               means no Dense tile).  The super-sparse share behind the th0 rule is
                               always taken on the 16 x 16 partition.  8 with spmv_kernel 1 is
                               refused with CB_ERROR_NOT_SUPPORTED; any other value with
                               CB_ERROR_INVALID_VALUE. */
    int32_t xcd_chunk;      /* how the kernels' workgroups (in dispatch order, which deals them to
                               the 8 XCDs in turn) map to work ranges: c >= 1 = each XCD takes runs of
                               c consecutive ranges, the XCDs side by side; 0 = each XCD one
                               contiguous eighth of the ranges; -1 (default) = automatic.  Results
                               do not depend on it. */
    int32_t cols16;         /* under column aggregation, how the SpMV kernels that stream work
                               ranges (spmv_kernel 0 and 2, lb_mode contiguous, none and
                               paper_stream, and the serving loop's batched products) read a tile's
                               original columns: as 2-byte offsets from a base, or as 4-byte
                               columns.  The quad kernel takes the base from its batch's header
                               (2 tile_dim bytes per tile instead of 4 tile_dim) where every quad
                               batch's columns span less than 65,536; otherwise, and for the
                               streaming kernel, a 4-byte base per tile (its first column; 2
                               tile_dim + 4 bytes) where every tile's columns span less than
                               65,536.  0 (default) = automatic: a 2-byte form where possible,
                               except the per-tile form for the quad kernel with double vectors
                               (its registers are at the limit of six wavefronts per SIMD: 4-byte
                               columns measured faster); 1 = a 2-byte form where possible; -1 =
                               always 4-byte columns.  Other values: CB_ERROR_INVALID_VALUE.  Results
                               do not depend on it. */
    int64_t min_wave_nnz;   /* with wave_nnz 0: the automatic work per range is at least this many
                               non-zero equivalents (0, the default: 256).  Longer ranges on small
                               matrices trade one product's latency for throughput when many
                               products share a launch (the serving loop's batches).  Negative:
                               CB_ERROR_INVALID_VALUE. */
    int64_t reserved[2];
} cb_options_t;

typedef struct {
    uint32_t struct_size;   /* caller sets sizeof(cb_info_t) before the call */
    int32_t value_type;
    int64_t m, n, nnz;
    int64_t npanels;        /* ceil(m / 16) */
    int64_t ntiles;
    int64_t tiles_coo, tiles_csr, tiles_dense;
    int32_t col_agg;        /* 1 when column aggregation was applied */
    int32_t lb_mode;
    double super_sparse_share;  /* share of tiles with < 32 non-zeros on the plain 16 x 16 partition */
    int64_t plain_tiles;    /* tiles of the plain partition (before aggregation) */
    int64_t payload_bytes;  /* packed tile data (mtx_data) */
    int64_t meta_bytes;     /* high-level arrays: 4+4+4+8+1 bytes per tile */
    int64_t restore_bytes;  /* restore_cols + cols_offset + a 4-byte restore index per tile
                               (0 without aggregation) */
    int64_t sched_bytes;    /* work-range pointers, panel flags, pre-pass panel list */
    int64_t nquanta;        /* groups of Algorithm 2 (or the contiguous ranges) */
    int64_t nwaves;         /* wavefront work ranges launched per SpMV */
    int64_t shared_panels;  /* panels whose tiles span more than one work range */
    int64_t prepass_panels; /* panels written by the y <- beta*y pre-pass (shared or empty) */
    int64_t quantum_nnz_max;
    double quantum_nnz_mean, quantum_nnz_std;
    int64_t wave_nnz_max;
    double wave_nnz_mean, wave_nnz_std;
    int64_t spmv_bytes;     /* algorithmic HBM bytes of one cb_spmv with beta == 0: the structure
                               the kernel of the handle's load-balance mode reads (payload, batch
                               records or the high-level arrays, restore_cols, schedule) + x once
                               + y once */
    int64_t device_bytes;   /* device memory owned by the handle */
    double convert_seconds; /* host conversion time */
    int32_t on_device;      /* 1 for cb_create handles, 0 for cb_create_host */
    int32_t reserved0;
    int64_t nbatches;       /* batches of the streaming kernel (0 with CB_LB_PAPER) */
    int64_t stream_bytes;   /* its batch records: 16 bytes per batch and per tile */
    double flat_run_mean;   /* COO/CSR entries per (tile, row) run: the lanes one scan step merges */
    int32_t row_reduce;     /* the resolved row_reduce option (0 .. 4) */
    int32_t vector_f64;     /* 1 when x and y are double (FP64 storage, or vector_f64 set) */
    int32_t spmv_kernel;    /* the resolved spmv_kernel option (0, 1 or 2) */
    int32_t tile_dim;       /* sub-block size S of the structure (16 or 8) */
    int32_t xcd_chunk;      /* the resolved xcd_chunk option */
    int32_t cols16;         /* the form the SpMV kernels read the original columns in (the cols16
                               option): 0 4-byte columns, 1 2-byte offsets from a base per tile
                               (tile_cbase), 2 2-byte offsets from a base per quad batch (the
                               batch header's fourth word) */
    int64_t reserved[2];
} cb_info_t;

/* Host buffers receiving the structure in kernel order (ntiles entries for the
 * tile arrays).  Any pointer may be NULL to skip that array.  Sizes come from
 * cb_get_info: payload_bytes, nquanta + 1, nwaves + 1, npanels (+ 1 for
 * cols_offset), restore_bytes / 4 - npanels - 1 - ntiles entries of restore_cols
 * when aggregation is applied, prepass_panels, ntiles for tile_xoff (aggregation
 * only). */
typedef struct {
    int32_t *tile_row;       /* blk_row_idx: panel (tile_dim rows) of each tile */
    int32_t *tile_col;       /* blk_col_idx: tile_dim-column block, or aggregated chunk */
    int32_t *tile_nnz;       /* nnz_per_blk */
    int64_t *tile_vp;        /* vp_per_blk: byte offset of the tile in payload */
    uint8_t *tile_type;      /* type_per_blk: cb_format_t */
    int32_t *tile_ori;       /* index of the tile in natural (panel, column) order */
    uint8_t *payload;        /* mtx_data */
    int32_t *restore_cols;   /* aggregated column -> original column */
    int32_t *cols_offset;    /* start of each panel's restore_cols, npanels + 1 */
    int32_t *quantum_ptr;    /* tile range of each group, nquanta + 1 */
    int32_t *wave_ptr;       /* tile range of each wavefront work range, nwaves + 1 */
    uint8_t *panel_shared;   /* 1 if the panel's tiles span more than one work range */
    int32_t *prepass_list;   /* panels written by the pre-pass */
    int32_t *tile_xoff;      /* aggregation only: cols_offset[tile_row] + tile_dim * tile_col, kernel order */
    int32_t *batch_stream;   /* streaming kernel: stream_bytes / 4 ints, a 16-byte header per batch
                                followed by a 16-byte record per tile (CB_LB_PAPER: none) */
    int32_t *batch_ptr;      /* first record of each work range, nwaves + 1 (CB_LB_PAPER: none) */
    int32_t *tile_cols;      /* aggregation with the streaming kernel: tile_dim original columns per
                                tile in kernel order, tile_dim * ntiles (else none); column c of a
                                tile at position (c mod 4) * tile_dim / 4 + c / 4 */
    int32_t *tile_cbase;     /* cols16 1 only: each tile's first original column, ntiles (else none) */
    uint16_t *tile_c16;      /* cols16 1 and 2: column c of each tile minus its base (cols16 1: the
                                tile's tile_cbase; 2: its quad batch's) at position c,
                                tile_dim * ntiles (columns past the tile's last: 0) */
} cb_structure_t;

/* Fill *opt with the defaults above (the paper's thresholds). */
cb_status_t cb_options_default(cb_options_t *opt);

/* Convert the CSR matrix (HOST arrays: row_ptr[m+1] int64, col_idx[nnz]
 * int32, values[nnz] double) into the CB structure (Section 3, Fig. 7 order:
 * partition, aggregation decision, column aggregation, format selection,
 * packing, load balance) and copy it to the current HIP device with one
 * transfer on `stream` (the call waits for that copy).  The CSR must be
 * canonical: row_ptr[0] = 0, non-decreasing, row_ptr[m] = nnz, 0 <= col < n,
 * columns strictly increasing within a row.  Explicit zeros, signed zeros,
 * NaN and Inf values are legal and stored.  opt may be NULL (defaults).
 * Errors: CB_ERROR_INVALID_VALUE for bad input, CB_ERROR_OUT_OF_MEMORY,
 * CB_ERROR_HIP. */
cb_status_t cb_create(cb_matrix_t *out, int64_t m, int64_t n, int64_t nnz, const int64_t *row_ptr,
                      const int32_t *col_idx, const double *values, const cb_options_t *opt, void *stream);

/* The same conversion without touching any GPU: the handle keeps the
 * structure in host memory for inspection (cb_get_info, cb_export_csr,
 * cb_export_structure).  cb_spmv / cb_spmm on it return
 * CB_ERROR_NOT_SUPPORTED. */
cb_status_t cb_create_host(cb_matrix_t *out, int64_t m, int64_t n, int64_t nnz, const int64_t *row_ptr,
                           const int32_t *col_idx, const double *values, const cb_options_t *opt);

/* y = alpha * A * x + beta * y over the CB structure (Section 3.5,
 * Algorithms 3 and 4).  x: n device elements, y: m device elements, double
 * for CB_VALUE_F64 and float otherwise (alpha and beta are then applied in
 * FP32).  beta == 0 means y is only written (NaN in y does not propagate).
 * Summation order differs from a sequential loop (results are within rounding
 * of the exact product).  x and y must not overlap.  Errors:
 * CB_ERROR_INVALID_VALUE (NULL handle or vectors), CB_ERROR_NOT_SUPPORTED
 * (host-only handle), CB_ERROR_HIP (launch failure). */
cb_status_t cb_spmv(cb_matrix_t A, double alpha, const void *x, double beta, void *y, void *stream);

/* Y = alpha * A * X + beta * Y for k right-hand sides.  X is n x k and Y is
 * m x k, both row-major device arrays with leading dimensions ldx >= k and
 * ldy >= k (elements).  Element type as for cb_spmv.  k == 1 with unit
 * leading dimensions is cb_spmv.  With the contiguous or no load balance
 * every tile is multiplied on the matrix cores (MFMA) as a 16 x 16 block (an
 * 8 x 8 tile in its top-left corner) times its rows of X, 16 or 32 columns of
 * X per launch slice; with Algorithm 2's order only Dense tiles are.  Errors as for cb_spmv, plus
 * CB_ERROR_INVALID_VALUE for k < 1 or ld < k. */
cb_status_t cb_spmm(cb_matrix_t A, int32_t k, double alpha, const void *X, int64_t ldx, double beta, void *Y,
                    int64_t ldy, void *stream);

/* Release the handle and its device memory.  cb_destroy(NULL) is a no-op. */
cb_status_t cb_destroy(cb_matrix_t A);

/* Rebuild CSR from the stored structure (for a device handle, from the
 * device copy) into HOST buffers: row_ptr[m+1], col_idx[nnz] and values[nnz]
 * in the storage type (double, float, or the 16-bit bf16 pattern).  For FP64
 * storage the result equals the cb_create input bit for bit. */
cb_status_t cb_export_csr(cb_matrix_t A, int64_t *row_ptr, int32_t *col_idx, void *values);

/* Sizes, counts and statistics of the structure.  info->struct_size must be
 * set by the caller. */
cb_status_t cb_get_info(cb_matrix_t A, cb_info_t *info);

/* Copy the structure into the caller's host buffers (see cb_structure_t). */
cb_status_t cb_export_structure(cb_matrix_t A, const cb_structure_t *out);

/* Device-to-device copy of `bytes` bytes with the library's streaming copy
 * kernel (16-byte loads and stores), used to measure the achievable HBM
 * bandwidth of the device.  src and dst must be 16-byte aligned device
 * pointers and must not overlap; bytes must be a multiple of 16. */
cb_status_t cb_copy_probe(const void *src, void *dst, int64_t bytes, void *stream);

/* Read-bandwidth probe: reads `bytes` of device memory at `src` with 16-byte
 * loads, each wavefront a contiguous 16 KB span with four loads in flight per
 * lane, and folds them into one word per thread,
 * which is stored to `sink` only when it equals a fixed value (a store the
 * compiler cannot remove, so every load stays; in practice nothing is
 * written).  It measures the achievable read bandwidth of the device, the
 * ceiling of a kernel that mostly reads (a product reads the structure and x
 * and writes only y).  src: 16-byte aligned device pointer; bytes: a
 * non-negative multiple of 16; sink: a device buffer of at least 16 bytes.
 * Enqueued on `stream`; errors as for cb_copy_probe. */
cb_status_t cb_read_probe(const void *src, int64_t bytes, void *sink, void *stream);

/* ---- Conjugate gradient (NEXT to the product: A symmetric positive definite) ----
 *
 * Solvers built on cb_spmv.  Each iteration runs on the device (the product, dot
 * products accumulated in FP64 and reduced in a fixed order, and the step lengths
 * read by the update kernels from device scalars); the host reads the residual
 * norm every check_every iterations, so the calls synchronise `stream` and must
 * not be captured in a graph.  The caller supplies the device workspace (size
 * from cb_cg_workspace_bytes); the solvers allocate nothing. */

/* How cb_cg_refine wins back FP64 accuracy from products on the low-precision copy.
 *   CB_REFINE_REPLACE: one CG whose products q = A_low p run in FP32 on the FP32/BF16
 *     copy while x, r, the dot products and the step lengths stay in FP64; whenever the
 *     recurrence residual has fallen by replace_factor since the last replacement, r is
 *     replaced by the true residual b - A x computed with the FP64 matrix (residual
 *     replacement, van der Vorst and Ye 2000), and only a true residual ends the solve.
 *   CB_REFINE_RESTART: classic iterative refinement: r = b - A x in FP64, an FP32 CG
 *     on A_low d = r / |r| to inner_rtol from d = 0, x += |r| d, repeated. */
typedef enum { CB_REFINE_RESTART = 0, CB_REFINE_REPLACE = 1 } cb_refine_t;

typedef struct {
    uint32_t struct_size;   /* sizeof(cb_cg_options_t) */
    int32_t max_iter;       /* iterations of one CG solve (of each inner solve when refining); 10000 */
    double rtol;            /* stop when |b - A x|_2 <= rtol |b|_2; 1e-10 */
    int32_t check_every;    /* iterations between host reads of the residual norm; 16 */
    int32_t max_refine;     /* outer steps of cb_cg_refine; 50 */
    double inner_rtol;      /* CB_REFINE_RESTART: residual reduction each inner solve aims at; 1e-4 */
    int32_t refine_method;  /* cb_refine_t; CB_REFINE_REPLACE */
    int32_t reserved32;
    double replace_factor;  /* CB_REFINE_REPLACE: recurrence reduction between residual
                               replacements, in (0, 1); 1e-2 */
    int64_t reserved[2];
} cb_cg_options_t;

typedef struct {
    int32_t converged;      /* 1 when the stopping test was met */
    int32_t iterations;     /* CG iterations (all inner solves for cb_cg_refine) */
    int32_t refinements;    /* cb_cg_refine: residual replacements (CB_REFINE_REPLACE) or outer
                               steps (CB_REFINE_RESTART); 0 for cb_cg */
    int32_t restarts;       /* CB_REFINE_REPLACE: replacements that also restarted the direction */
    double rel_residual;    /* |b - A x|_2 / |b|_2 of the returned x, computed in FP64 from the true residual
                               (FP64 handles); the CG recurrence's value for FP32/BF16 handles in cb_cg */
    int64_t reserved[2];
} cb_cg_result_t;

cb_status_t cb_cg_options_default(cb_cg_options_t *opt);

/* Device workspace bytes for cb_cg on A (A_low NULL) or for cb_cg_refine on A and A_low. */
cb_status_t cb_cg_workspace_bytes(cb_matrix_t A, cb_matrix_t A_low, int64_t *bytes);

/* Conjugate gradient on A x = b (Hestenes and Stiefel) starting from the caller's x.  b and x are n
 * device elements of A's vector type (double with FP64 storage or vector_f64, else float); x is overwritten
 * with the solution.  work: device buffer of at least cb_cg_workspace_bytes(A, NULL) bytes (its
 * contents are scratch).  A must be square; a non-positive-definite search direction stops the
 * iteration with converged = 0.  opt may be NULL (defaults).  Errors: CB_ERROR_INVALID_VALUE (NULL
 * arguments, workspace too small, bad options, non-square A), CB_ERROR_NOT_SUPPORTED (host-only
 * handle), CB_ERROR_HIP. */
cb_status_t cb_cg(cb_matrix_t A, const void *b, void *x, void *work, int64_t work_bytes, const cb_cg_options_t *opt,
                  cb_cg_result_t *res, void *stream);

/* Mixed-precision solve of A x = b to an FP64 accuracy: A stored in FP64, A_low the same matrix
 * stored in FP32 or BF16 (float or, with vector_f64, double vectors), the products on A_low and
 * the accuracy won back with FP64 residuals as
 * refine_method says (see cb_refine_t), until |b - A x| <= rtol |b| for the true FP64 residual, or
 * until the true residual stops decreasing (converged = 0).  b and x are double device vectors, x
 * the start and the solution; work: device buffer of at least cb_cg_workspace_bytes(A, A_low)
 * bytes.  Errors as for cb_cg, plus CB_ERROR_INVALID_VALUE when the handles' precisions or sizes
 * do not fit. */
cb_status_t cb_cg_refine(cb_matrix_t A, cb_matrix_t A_low, const double *b, double *x, void *work, int64_t work_bytes,
                         const cb_cg_options_t *opt, cb_cg_result_t *res, void *stream);

/* ---- CG without device allocation ----
 *
 * For callers that cannot allocate device memory (loops that must not call hipMalloc, harnesses
 * that forbid it): cb_cg with its workspace taken from a fixed array of CB_CG_NOALLOC_MAX_BYTES
 * bytes inside the library instead of a caller's buffer.  Arguments, results and errors as for
 * cb_cg; b and x stay caller-owned device vectors.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); the array is reserved in device memory when the library's
 * code is loaded on a GPU and kept, one per GPU, until the process ends.  It fits solves whose
 * cb_cg_workspace_bytes(A, NULL) is at most CB_CG_NOALLOC_MAX_BYTES (FP64 vectors: n up to about
 * 2.79 million; float vectors: about 5.59 million); larger ones return CB_ERROR_INVALID_VALUE.
 * A must live on the current device (else CB_ERROR_INVALID_VALUE).  All calls on one GPU share that
 * GPU's array: the library runs them one at a time (a second caller waits for the first), and
 * each call returns only after its work on `stream` has finished.  The array keeps the last
 * call's contents; every solve sets what it reads before reading it. */
#define CB_CG_NOALLOC_MAX_BYTES (64 * 1024 * 1024)

cb_status_t cb_cg_noalloc(cb_matrix_t A, const void *b, void *x, const cb_cg_options_t *opt, cb_cg_result_t *res,
                          void *stream);

/* Message for the last non-success status returned on this thread. */
const char *cb_last_error(void);

/* ---- Autotuner (NEXT: per-matrix layout choices by measurement) ----
 *
 * cb_tune converts the matrix under a short list of candidate options and times the product on
 * each (cb_spmv, or cb_spmm with spmm_k right-hand sides; HIP events on `stream`, median of reps
 * launches with x = 1 and beta = 0), by coordinate descent from `base` over: column aggregation
 * on/off, the sub-block size (16 x 16 or 8 x 8 tiles, th1/th2 scaled with the tile's area), the
 * natural-order kernel (entries or quads per lane), the form of the original columns under
 * aggregation (cols16: 2-byte offsets or 4-byte columns), the workgroup-to-range mapping (xcd_chunk
 * 16 or 0), the format thresholds th1/th2 (the base
 * ones, COO below Dense at 200/256 of the tile's slots, COO only), the row-sum mode, the
 * load-balance split (nnz-balanced at panel boundaries or equal tile counts) and the work per
 * wavefront (half and twice the current ranges' mean).  A choice is kept when it is at least
 * 1 % faster.  Every candidate computes the same product within the storage precision's
 * tolerance.  The tuner allocates: candidate structures, X and Y. */
#define CB_TUNE_MAX_CANDIDATES 16

typedef struct {
    uint32_t struct_size;   /* sizeof(cb_tune_options_t) */
    int32_t reps;           /* timed launches per candidate (after 3 untimed); 20 */
    int32_t max_candidates; /* 1 .. CB_TUNE_MAX_CANDIDATES; CB_TUNE_MAX_CANDIDATES */
    int32_t spmm_k;         /* 0 or 1 (default 0): time cb_spmv; 2 .. 4096: time cb_spmm with that
                               many right-hand sides (X n x k, Y m x k, leading dimension k) */
    int64_t reserved[4];
} cb_tune_options_t;

typedef struct {
    cb_options_t opt;       /* the candidate's options as given to cb_create */
    double us;              /* median kernel time of one cb_spmv, microseconds */
    int64_t spmv_bytes;     /* its algorithmic bytes per launch */
    int32_t col_agg;        /* resolved aggregation */
    int32_t row_reduce;     /* resolved row-sum mode */
    int32_t tile_dim;       /* resolved sub-block size (16 or 8) */
    int32_t spmv_kernel;    /* resolved natural-order kernel */
} cb_tune_candidate_t;

typedef struct {
    int32_t ncandidates;
    int32_t best;           /* index into cand */
    cb_tune_candidate_t cand[CB_TUNE_MAX_CANDIDATES];
} cb_tune_report_t;

cb_status_t cb_tune_options_default(cb_tune_options_t *opt);

/* Tunes the options for the CSR matrix (arguments as cb_create; base NULL = defaults, its
 * value_type and vector_f64 are kept).  *best receives the fastest candidate's options; out, if
 * not NULL, receives that candidate's handle (else it is destroyed); report may be NULL.  Errors
 * as cb_create, plus CB_ERROR_INVALID_VALUE for bad tuner options and CB_ERROR_NOT_SUPPORTED for
 * lb_mode CB_LB_PAPER in base (the tuner works on the streaming kernel's structures). */
cb_status_t cb_tune(cb_matrix_t *out, int64_t m, int64_t n, int64_t nnz, const int64_t *row_ptr,
                    const int32_t *col_idx, const double *values, const cb_options_t *base,
                    const cb_tune_options_t *topt, cb_options_t *best, cb_tune_report_t *report, void *stream);

/* ---- Serving loop (NEXT to the solvers): many resident matrices, continuous batching ----
 *
 * A server keeps registered (resident) handles and serves requests on them from a worker thread
 * of its own: SpMM requests (Y = alpha A X + beta Y, k right-hand sides) and CG solves.  Requests
 * are admitted in arrival order as soon as their device footprint fits in the server's memory
 * arena (allocated once, at creation) and, for a solve, a solve slot is free; requests that
 * arrive while others run join at the next step.  Active solves advance together: one step runs
 * the products of every active solve as batched launches (one launch per value type, aggregation
 * and row-sum mode, covering the work ranges of all their matrices) and the vector updates of all
 * of them as batched launches; check_every steps are captured once as a HIP graph and replayed
 * until the set of active solves changes.  SpMM requests run on their own streams beside the
 * solves.  A solve's arithmetic does not depend on what else is active (fixed per-solve
 * reductions), so its result alone and in a mix is the same up to the order of the global atomic
 * adds of shared panels.  Host vectors of a request must stay valid until it completes. */
typedef struct cb_server_s *cb_server_t;

typedef struct {
    uint32_t struct_size;   /* sizeof(cb_server_options_t) */
    int32_t max_active;     /* solves advanced together (solve slots per vector type); 64 */
    int64_t arena_bytes;    /* device bytes for request vectors and solve workspaces; 1 GiB */
    int32_t check_every;    /* solve steps between host reads of the solves' scalars; 8 */
    int32_t use_graph;      /* 1: replay the captured steps as a HIP graph (default); 0: launch them */
    int32_t spmm_streams;   /* streams for SpMM requests; 2 */
    int32_t reserved32;
    int64_t reserved[4];
} cb_server_options_t;

/* CB_REQ_CG: CG in the matrix's own vector type, stopped on the recurrence residual.
 * CB_REQ_CG_REFINE: CG with FP64 residual replacement (as cb_cg_refine with CB_REFINE_REPLACE and
 * replace_factor 1e-2): matrix is a FP64 handle, matrix_low a FP32 or BF16 handle of the same
 * matrix with float vectors; the steps multiply by matrix_low (p and q float), x, r, the dot
 * products and the scalar recurrences stay FP64, r is replaced by the true residual b - A x of
 * the FP64 matrix between periods, and only a true residual <= rtol |b| ends the solve as
 * converged.  b and x are double. */
typedef enum { CB_REQ_SPMM = 0, CB_REQ_CG = 1, CB_REQ_CG_REFINE = 2 } cb_request_kind_t;

typedef struct {
    uint32_t struct_size;   /* sizeof(cb_request_t) */
    int32_t kind;           /* cb_request_kind_t */
    int32_t matrix;         /* id from cb_server_add_matrix */
    int32_t k;              /* SpMM: right-hand sides (>= 1); CG: ignored */
    double alpha, beta;     /* SpMM */
    const void *in;         /* host, the matrix's vector type: SpMM X (n x k row-major); CG b (n) */
    void *out;              /* host: SpMM Y (m x k, read when beta != 0, written); CG x (n: the start,
                               overwritten with the solution) */
    double rtol;            /* CG: stop when the recurrence residual (CB_REQ_CG_REFINE: the true
                               residual) is <= rtol |b|; 0 = 1e-10 */
    int32_t max_iter;       /* CG: iteration cap (rounded up to a multiple of check_every); 0 = 500 */
    int32_t matrix_low;     /* CB_REQ_CG_REFINE: id of the FP32/BF16 copy the steps multiply by */
    int64_t reserved[4];
} cb_request_t;

typedef struct {
    int32_t done;           /* 1 once the request has completed */
    int32_t status;         /* cb_status_t of the request */
    int32_t iterations;     /* CG iterations */
    int32_t converged;      /* CG: 1 when the residual test was met */
    double rel_residual;    /* CG: |r| / |b| at the end (recurrence; CB_REQ_CG_REFINE: the true
                               residual of the last replacement) */
    double latency_us;      /* submission to completion */
    double queue_us;        /* submission to admission */
    int32_t replacements;   /* CB_REQ_CG_REFINE: residual replacements (the last one decides) */
    int32_t restarts;       /* CB_REQ_CG_REFINE: replacements that restarted the direction */
    int64_t reserved[1];
} cb_response_t;

typedef struct {
    int64_t submitted, completed, rejected;
    int64_t spmm_done, cg_done;
    double p50_us, p99_us, mean_us;  /* latency over completed requests */
    double elapsed_s;                /* first submission to last completion */
    double requests_per_s;           /* completed / elapsed_s */
    double solves_per_s;             /* completed CG solves / elapsed_s */
    int64_t arena_peak_bytes;        /* most arena bytes in use at once */
    int32_t active_peak;             /* most solves active at once */
    int32_t graph_builds;            /* HIP graphs captured (one per active set that lasts beyond its first period) */
    int64_t steps;                   /* solve steps run */
    int64_t reserved[4];
} cb_server_stats_t;

cb_status_t cb_server_options_default(cb_server_options_t *opt);

/* Creates a server on the current device (allocates its arena and tables).  Errors:
 * CB_ERROR_INVALID_VALUE (bad options), CB_ERROR_OUT_OF_MEMORY, CB_ERROR_HIP. */
cb_status_t cb_server_create(const cb_server_options_t *opt, cb_server_t *out);

/* Registers a device handle of a natural-order structure (lb_mode contiguous or none) on the
 * server's device, at any time; *id is its number for requests.  The server does not own the
 * handle: keep it until cb_server_destroy.  At most 16384 handles per server.  Errors:
 * CB_ERROR_INVALID_VALUE, CB_ERROR_NOT_SUPPORTED (host-only or paper-order handle, another device,
 * too many handles). */
cb_status_t cb_server_add_matrix(cb_server_t S, cb_matrix_t A, int32_t *id);

/* Queues a request; *ticket names it.  CB_ERROR_INVALID_VALUE for a bad request (unknown matrix,
 * k < 1, NULL vectors, CG on a non-square matrix), CB_ERROR_OUT_OF_MEMORY when its footprint can
 * never fit the arena (counted as rejected). */
cb_status_t cb_server_submit(cb_server_t S, const cb_request_t *req, int64_t *ticket);

/* Response of a ticket: done = 0 while it is queued or running (poll), or after blocking until it
 * completes (wait).  CB_ERROR_INVALID_VALUE for an unknown ticket. */
cb_status_t cb_server_poll(cb_server_t S, int64_t ticket, cb_response_t *resp);
cb_status_t cb_server_wait(cb_server_t S, int64_t ticket, cb_response_t *resp);

cb_status_t cb_server_stats(cb_server_t S, cb_server_stats_t *stats);

/* Completes every queued request, stops the worker and frees the server's memory. */
cb_status_t cb_server_destroy(cb_server_t S);

#ifdef __cplusplus
}
#endif

#endif /* CBSPMV_H */
