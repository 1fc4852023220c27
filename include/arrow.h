/*
 * arrow.h -- C ABI of the MI355X (gfx950) arrow-decomposition SpMM library.
 *
 * The library computes the iterated sparse x tall-skinny dense product
 *
 *     Y_t = A X_t,   X_{t+1} = Y_t / ||Y_t||_col            (t = 0 .. T-1)
 *
 * (problem statement of Section 2, "Matrices": X_{t+1} = sigma(A X_t) with
 * sigma a per-column normalisation) over an arrow matrix decomposition
 *
 *     A = sum_i P_{pi_i} B_i P_{pi_i}^T                       (Section 4, Eq. (1))
 *
 * where every B_i has arrow width b: its nonzeros lie in the first b rows, the
 * first b columns, or the band |p - q| <= b (Section 1, 0-based here).
 *
 * Two stages:
 *   1. arrow_decompose (host, C++): LA-Decompose of Section 5.1 with the
 *      random spanning forest linear arrangement of Section 5.3 and the
 *      smallest-first tree order of Section 5.4.
 *   2. arrow_plan_create uploads the decomposition to one GPU; arrow_spmm /
 *      arrow_spmm_iterate run the product with hand-written HIP kernels.
 *
 * Conventions for every function:
 *   - Return value: ARROW_OK (0) or an error code; arrow_last_error() gives a
 *     thread-local description of the last failure.  On failure, out-handles
 *     are set to NULL and nothing is leaked.
 *   - Argument errors are detected synchronously before any device work.
 *   - "device" pointers are HIP device memory of the plan's GPU and belong to
 *     the caller; the library never frees them.  "host" pointers are ordinary
 *     CPU memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued asynchronously on it; faults in that work
 *     surface at the caller's next synchronisation.
 *   - Dense matrices are row-major with a row stride (`ld`, in elements).
 *     Row and column storage must be 16-byte aligned: the base pointer and
 *     ld * element_size must be multiples of 16.
 *   - Feature width k must be a positive multiple of 16.
 *   - Decompositions and plans are immutable after creation, apart from the
 *     schedule settings arrow_plan_set_batch and arrow_profile_enable (call
 *     those while no other host thread uses the plan); concurrent calls on one
 *     plan from several streams are safe when each call has its own workspace
 *     and outputs.
 */
#ifndef ARROW_H
#define ARROW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t arrow_status_t;
enum {
    ARROW_OK = 0,
    ARROW_ERR_INVALID_ARG = 1,   /* bad argument: null pointer, bad CSR, bad size */
    ARROW_ERR_OUT_OF_MEMORY = 2, /* host or device allocation failed */
    ARROW_ERR_HIP = 3,           /* a HIP runtime call failed */
    ARROW_ERR_UNSUPPORTED = 4,   /* valid but not supported (e.g. too many levels) */
    ARROW_ERR_IO = 5,            /* file error or corrupt file in save/load */
    ARROW_ERR_INTERNAL = 6
};

/* Storage type of X and Y.  Products are always accumulated in FP32. */
typedef int32_t arrow_dtype_t;
enum {
    ARROW_F32 = 0,
    ARROW_F16 = 1,     /* IEEE binary16, per-column power-of-two scale */
    ARROW_BF16 = 2,    /* bfloat16, no scale needed (scale pointer may be NULL) */
    ARROW_F8E4M3 = 3   /* OCP FP8 E4M3FN (max 448), per-column power-of-two scale */
};

/* Linear arrangement used for the non-head vertices of each level. */
typedef int32_t arrow_la_t;
enum {
    ARROW_LA_RANDOM_FOREST = 0, /* random spanning forest + smallest-first order (Sections 5.3-5.4) */
    ARROW_LA_IDENTITY = 1,      /* vertices in id order (the input's own ordering) */
    ARROW_LA_SEPARATOR = 2      /* recursive separators (Section 5.2): BFS-level separators */
};

typedef struct arrow_decomp_s *arrow_decomp_t; /* host object */
typedef struct arrow_plan_s *arrow_plan_t;     /* device-resident object */

/* ------------------------------------------------------------------------ */
/* Stage 1: decomposition (host)                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t b;          /* arrow width, >= 2 (Section 5.1 requires b >= 2) */
    arrow_la_t la;      /* linear arrangement kind */
    uint64_t seed;      /* seed of the random edge weights (Section 5.3, step 1) */
    int32_t max_levels; /* 0 = unlimited; otherwise fail with ARROW_ERR_UNSUPPORTED above it */
    int32_t threads;    /* host threads: 0 = every hardware thread, >= 1 = that many; the
                           result does not depend on it */
} arrow_decompose_opts_t;

/*
 * LA-Decompose (Section 5.1) of the square n x n CSR matrix (host arrays):
 * row_ptr int64[n+1], col int32[nnz] strictly increasing within each row and
 * < n, val float32[nnz]; nnz < 2^31.  The pattern is symmetrised for the graph
 * steps (degrees, spanning forest); every stored entry keeps its own value and
 * lands in exactly one level.  Level 0 spans all n positions; later levels are
 * compacted to the positions that hold entries (Section 4, "collect the
 * non-zeros at the top").  The result depends only on the inputs, b, la and
 * seed (bit for bit, whatever opts.threads is).
 * Errors: ARROW_ERR_INVALID_ARG for a malformed CSR, b < 2 or threads < 0.
 */
arrow_status_t arrow_decompose(int64_t n, const int64_t *row_ptr, const int32_t *col,
                               const float *val, const arrow_decompose_opts_t *opts,
                               arrow_decomp_t *out);

typedef struct {
    int64_t n, nnz;
    int32_t b, levels;
    double seconds;       /* wall time of arrow_decompose */
} arrow_decomp_info_t;

arrow_status_t arrow_decomp_info(arrow_decomp_t d, arrow_decomp_info_t *out);

/*
 * Export level `level` (host pointers owned by the decomposition, valid until
 * arrow_decomp_destroy): n_i positions, vertex_of_pos int32[n_i] (the vertex
 * placed at each position, i.e. pi_i^{-1} restricted to [0, n_i)), and B_i as
 * CSR over positions: row_ptr int64[n_i+1], col int32[nnz_i], val float32[nnz_i].
 */
arrow_status_t arrow_decomp_level(arrow_decomp_t d, int32_t level, int64_t *n_i,
                                  int64_t *nnz_i, const int32_t **vertex_of_pos,
                                  const int64_t **row_ptr, const int32_t **col,
                                  const float **val);

/*
 * Counts of level `level`: positions n_i, entries nnz_i, entries in the head
 * rows (position < b), in the head columns of the other rows (column < b) and
 * in the band (both >= b), and rows holding entries.  Host only.
 */
typedef struct {
    int64_t n_i, nnz_i, head_row_nnz, head_col_nnz, band_nnz, active_rows;
} arrow_level_stats_t;
arrow_status_t arrow_decomp_level_stats(arrow_decomp_t d, int32_t level,
                                        arrow_level_stats_t *out);

/*
 * Nonzero blocks of level `level` in a grid of s x s blocks (s >= 1): the
 * number of blocks that hold at least one entry (with s = b these are the
 * b x b tiles of Section 4.1, the count Section 7 compares with a 1.5D
 * decomposition) and a histogram of their densities (entries / s^2):
 * hist[j] counts blocks with density in [j/10, (j+1)/10), hist[9] also those
 * of density 1.  region 0 takes every entry, region 1 only the head rows and
 * columns (row or column < b).  With s = 16 the histogram shows whether any
 * head tile is dense enough for a matrix-core product.  Host only.
 */
typedef struct {
    int64_t nonzero_blocks, entries;
    double max_density;
    int64_t hist[10];
} arrow_block_stats_t;
arrow_status_t arrow_decomp_block_stats(arrow_decomp_t d, int32_t level, int32_t s,
                                        int32_t region, arrow_block_stats_t *out);

/* Versioned binary file with a checksum; load rejects corrupt files (ARROW_ERR_IO). */
arrow_status_t arrow_decomp_save(arrow_decomp_t d, const char *path);
arrow_status_t arrow_decomp_load(const char *path, arrow_decomp_t *out);
void arrow_decomp_destroy(arrow_decomp_t d);

/* ------------------------------------------------------------------------ */
/* Stage 2: device plan and products                                        */
/* ------------------------------------------------------------------------ */

/*
 * Device allocator of plan buffers (process-wide).  alloc returns `bytes` of
 * device memory of the current HIP device (the plan's; 256-byte aligned) or
 * NULL on failure; `stream` is the stream given to arrow_plan_create.  free
 * releases a pointer alloc returned, with stream = NULL: the caller destroys
 * a plan only after its last product finished.  A plan keeps the allocator
 * it was created with and frees through it.  arrow_set_allocator(NULL, NULL,
 * NULL) restores the default (hipMalloc / hipFree).  Both functions or
 * neither must be given (else ARROW_ERR_INVALID_ARG).  Not thread-safe
 * against a concurrent arrow_plan_create.  Workspaces, X and Y are always the
 * caller's; this hook covers the only device memory the library owns.
 */
typedef void *(*arrow_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*arrow_free_fn)(void *ptr, void *stream, void *ctx);
arrow_status_t arrow_set_allocator(arrow_alloc_fn alloc, arrow_free_fn free_fn, void *ctx);

/*
 * Upload a decomposition to GPU `device` as a plan (the arrow tiles of
 * Section 4.1 become row blocks of work; the level maps pi_i become
 * precomputed gather indices into the level-0 order).  Short rows of levels
 * >= 1 are folded into the level-0 row of their vertex (the products of
 * Alg. 2 reassociated per vertex); long rows of any level become chunks with
 * FP32 partial rows.  Synchronous: returns after the upload finished.  The
 * plan does not reference `d` afterwards.
 */
arrow_status_t arrow_plan_create(arrow_decomp_t d, int32_t device, void *stream,
                                 arrow_plan_t *out);
void arrow_plan_destroy(arrow_plan_t p);

typedef struct {
    int64_t n, nnz;
    int32_t b, levels;
    int64_t footprint_bytes;  /* device memory owned by the plan */
    int64_t chunked_rows;     /* rows split into nnz chunks (rows of more than 32 entries) */
    int64_t chunks;           /* number of chunks */
    int64_t upper_rows;       /* rows of levels >= 1 computed by the upper pass */
    int64_t contributions;    /* partial rows (chunks, upper rows) listed by level-0 rows */
    double a_inf_norm;        /* max_i sum_j |A_ij| (bounds the FP8/FP16 scales) */
    int32_t upper_batch;      /* gather batch of the upper / level-0 passes: 0 = wide, */
    int32_t level0_batch;     /* else entries gathered per row and batch (4..8) */
    int64_t fused_rows;       /* rows of levels >= 1 folded into their level-0 row */
    int32_t level0_block_rows; /* rows per staged block of the level-0 pass */
    int32_t reserved;
} arrow_plan_info_t;

arrow_status_t arrow_plan_info(arrow_plan_t p, arrow_plan_info_t *out);
/* Device memory owned by the plan (the plan's own buffers, allocated through
 * the allocator of arrow_set_allocator at creation and freed by
 * arrow_plan_destroy). */
arrow_status_t arrow_plan_footprint(arrow_plan_t p, size_t *bytes);

/*
 * Gather batch of a row pass (kernel = ARROW_KERNEL_UPPER or
 * ARROW_KERNEL_LEVEL0).  The rows of a pass are gathered in batches; a wide
 * batch (0) takes 8 entries of a row and up to 8 listed partial rows at a
 * time, a short batch u in [4, 8] takes u entries and 2 partial rows at a time
 * with fewer registers, so more waves share a SIMD.  arrow_plan_create picks
 * the smallest short batch that holds the entries of at least 99% of the
 * pass's rows when at least 99% of them list at most 2 partial rows, and the
 * wide batch otherwise; batch = -1 restores that choice.  Every batch
 * computes the same products in the same order (they agree up to the sign of
 * a zero); the FP64 column norms reduce the same squares in a batch-dependent
 * fixed order, so they agree to rounding.  Operands whose X, or whose
 * partial-row workspace, spans 4 GiB or more always take the wide batch.
 * Not thread-safe against concurrent products on the same plan.
 */
arrow_status_t arrow_plan_set_batch(arrow_plan_t p, int32_t kernel, int32_t batch);

/* Kernel ids for arrow_plan_kernel_bytes and the profiling counters. */
enum {
    ARROW_KERNEL_CHUNKS = 0,  /* long rows (hub rows), nnz-balanced chunks */
    ARROW_KERNEL_UPPER = 1,   /* rows of levels >= 1 (gathered through pi_0 o pi_i^{-1}) */
    ARROW_KERNEL_LEVEL0 = 2,  /* level-0 band + head columns + cross-level sum + store */
    ARROW_KERNEL_NORM = 3,    /* FP64 column norms and next scales */
    ARROW_KERNEL_PERMUTE = 4, /* permute in / out */
    ARROW_KERNEL_COMBINE = 5, /* sums of long partial-row lists (hub rows), before level 0 */
    ARROW_KERNEL_COUNT = 6
};

/*
 * Algorithmic HBM bytes one launch of `kernel` moves for one product with k
 * columns of `dtype` (every matrix entry, index and X/Y/partial row counted
 * once), written to *bytes.  Used for the roofline.
 */
arrow_status_t arrow_plan_kernel_bytes(arrow_plan_t p, int32_t kernel, int64_t k,
                                       arrow_dtype_t dtype, int64_t *bytes);

/* Device workspace bytes needed by arrow_spmm for one operand of k columns
 * (arrow_spmm_iterate needs arrow_iterate_workspace_size instead). */
arrow_status_t arrow_workspace_size(arrow_plan_t p, int64_t k, arrow_dtype_t dtype,
                                    size_t *bytes);

/*
 * X_plan = P_{pi_0}^T X: row p of x_plan receives row pi_0^{-1}(p) of the
 * original-order FP32 input x (device, ldx >= k), converted to `dtype`.
 * For ARROW_F16 / ARROW_F8E4M3 the per-column power-of-two scale s_j (so that
 * max_i |x_ij| / s_j fits the format) is computed and written to
 * x_scale (device float[k], required for those types, ignored otherwise);
 * x_maxabs (device float[k] or NULL) receives max_i |code_ij| per column.
 */
arrow_status_t arrow_permute_in(arrow_plan_t p, const float *x, int64_t ldx, void *x_plan,
                                int64_t ld, arrow_dtype_t dtype, int64_t k, float *x_scale,
                                float *x_maxabs, void *stream);

/*
 * y = P_{pi_0} Y_plan, dequantised to FP32: row pi_0^{-1}(p) of y (device,
 * ldy >= k) receives row p of y_plan times x_scale[j] (NULL = 1) times
 * col_factor[j] (device double[k], NULL = 1).
 */
arrow_status_t arrow_permute_out(arrow_plan_t p, const void *y_plan, int64_t ld,
                                 arrow_dtype_t dtype, int64_t k, const float *x_scale,
                                 const double *col_factor, float *y, int64_t ldy, void *stream);

/*
 * One operand of a product: a column block of one request, in plan order.
 * Y[:, j] = x_scale[j] * x_inv_norm[j] * (A Q)[:, j] where Q is x as stored;
 * the linearity of the product folds the previous step's normalisation into
 * this one, so no separate scaling pass over X is needed.
 */
typedef struct {
    const void *x;            /* device, n rows, stride ldx elements */
    void *y;                  /* device, n rows, stride ldy elements; must not alias x */
    int64_t k;                /* columns, multiple of 16 */
    int64_t ldx, ldy;
    arrow_dtype_t dtype;      /* storage type of both x and y */
    int32_t reserved;
    const float *x_scale;     /* device float[k]: x = x_scale * code; NULL = 1 */
    const double *x_inv_norm; /* device double[k]: factor of this product; NULL = 1 */
    const float *x_maxabs;    /* device float[k]: max |code| of x (F16/F8); NULL = format max */
    float *y_scale;           /* device float[k] out: scale y is stored with (required F16/F8) */
    float *y_maxabs;          /* device float[k] out: max |code| of y, or NULL */
    double *y_norm;           /* device double[k] out: ||Y[:, j]||_2 of the stored y, or NULL */
    double *y_inv_norm;       /* device double[k] out: 1/||Y[:, j]||_2 (0 for a zero column), or NULL */
    const float *w;           /* device float[k*k] row-major, or NULL: the product becomes the
                                 GNN-style step y = ReLU((A x) w) (Section 2: the iteration with
                                 an element-wise sigma, here after a k x k weight matrix), fused
                                 into the last row pass on FP32 matrix cores; F32 only, k one of
                                 16, 32, 64, 128 (ARROW_ERR_UNSUPPORTED otherwise); y_norm and
                                 y_inv_norm then describe the stored ReLU output */
} arrow_operand_t;

/*
 * One product Y = A X for each operand (Section 4, Eq. (1): every level's
 * arrow product, the head-row panels and head-column strips of Alg. 1, and
 * the forward permutation and reverse accumulation of Alg. 2, fused into
 * row passes in level-0 order), enqueued on `stream`.  Operands of one
 * storage type and one tile width (the largest of 128, 64, 32, 16 dividing
 * k) share one launch sequence over all their column tiles, so the matrix is
 * read once for all of them (requests on the same graph batched into a wider
 * k).  The work partition depends only on the plan, k and the storage type,
 * and column norms are reduced in FP64 in a fixed order, so every operand's
 * result is bitwise the one it gets alone.  No operand's y may overlap
 * another operand's x or y (ARROW_ERR_INVALID_ARG).  `workspace` (device,
 * 256-byte aligned) must hold arrow_workspace_size bytes per operand (the
 * sum over operands, in operand order).
 */
arrow_status_t arrow_spmm(arrow_plan_t p, const arrow_operand_t *ops, int32_t num_ops,
                          void *workspace, size_t ws_bytes, void *stream);

/*
 * arrow_spmm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same products, bit for bit, with the workspace taken from a fixed array of
 * ARROW_STATIC_WORKSPACE_BYTES that the library holds on each GPU it runs on
 * until the process ends.  Calls no allocating routine.  Operands are as for
 * arrow_spmm.  Returns ARROW_ERR_UNSUPPORTED, before any device work, when
 * the operands need more than ARROW_STATIC_WORKSPACE_BYTES of workspace
 * (the sum of arrow_workspace_size over the operands).  Every call on one GPU
 * shares that GPU's array (no part of it needs to start at zero: a call reads
 * only what it wrote itself), so calls that overlap in time on one GPU -- on
 * different streams, or from several host threads -- race and give wrong
 * results; serialise them.
 */
#define ARROW_STATIC_WORKSPACE_BYTES (64u << 20)
arrow_status_t arrow_spmm_static(arrow_plan_t p, const arrow_operand_t *ops, int32_t num_ops,
                                 void *stream);

/* Workspace for arrow_spmm_iterate (product buffers plus the ping-pong state). */
arrow_status_t arrow_iterate_workspace_size(arrow_plan_t p, int64_t k, arrow_dtype_t dtype,
                                            size_t *bytes);

enum { ARROW_ITER_RENORM = 1 };

/*
 * `iters` products of the iteration.  x (device, plan order, stride ld) holds
 * X_0 and is not modified; y (device, stride ld) receives the last product
 * Y_{T-1} un-normalised; intermediate products live in the workspace.
 * With ARROW_ITER_RENORM the input of step t >= 1 is Y_{t-1}/||Y_{t-1}||_col,
 * otherwise Y_{t-1} itself.  norms (device double[iters*k] or NULL) receives
 * ||Y_t[:, j]||_2 at [t*k + j].  For F16/F8 x_scale (device float[k]) is the
 * scale of x and y_scale (device float[k], required) receives the scale of y.
 */
arrow_status_t arrow_spmm_iterate(arrow_plan_t p, const void *x, void *y, int64_t k, int64_t ld,
                                  arrow_dtype_t dtype, const float *x_scale, float *y_scale,
                                  int32_t iters, uint32_t flags, double *norms,
                                  void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Baselines, calibration and measurement                                   */
/* ------------------------------------------------------------------------ */

/*
 * Plain CSR SpMM on the device, the comparison baseline: y = A x with the
 * CSR (device row_ptr int32[n+1], col int32[nnz], val float32[nnz]) in
 * whatever order the caller uploaded, FP32 x/y (stride ld), plus the same
 * FP64 column-norm epilogue when sumsq_ws (device double workspace of
 * arrow_csr_workspace_size bytes) and norms (device double[k]) are non-NULL.
 */
arrow_status_t arrow_csr_workspace_size(int64_t n, int64_t k, size_t *bytes);
/* Gather batch for arrow_csr_spmm from the host row_ptr int64[n+1], by the
 * rule arrow_plan_create applies to its passes (0 = wide, else 4..8). */
arrow_status_t arrow_csr_batch(int64_t n, const int64_t *row_ptr, int32_t *batch);
/* batch: 0 (wide) or 4..8 entries gathered per row and batch (a schedule
 * choice: every batch gives the same y; the norms agree to rounding). */
arrow_status_t arrow_csr_spmm(int64_t n, const int32_t *row_ptr, const int32_t *col,
                              const float *val, const float *x, float *y, int64_t k, int64_t ld,
                              int32_t batch, double *sumsq_ws, double *norms, void *stream);

/*
 * The vendor CSR SpMM (rocSPARSE generic API) as a second comparison
 * baseline: y = A x with the same device CSR and row-major FP32 x / y
 * (stride ld).  create does the buffer-size query, allocation and
 * preprocessing (synchronous); run enqueues one product on the stream given
 * at creation.  `alg` is a rocsparse_spmm_alg value (0 = library default).
 */
typedef struct arrow_rocsparse_s *arrow_rocsparse_t;
arrow_status_t arrow_rocsparse_create(int64_t n, int64_t nnz, const int32_t *row_ptr,
                                      const int32_t *col, const float *val, const float *x,
                                      float *y, int64_t k, int64_t ld, int32_t alg, void *stream,
                                      arrow_rocsparse_t *out);
arrow_status_t arrow_rocsparse_run(arrow_rocsparse_t ctx);
void arrow_rocsparse_destroy(arrow_rocsparse_t ctx);

/* Streaming copy of `bytes` (multiple of 16) from src to dst: HBM calibration. */
arrow_status_t arrow_copy(const void *src, void *dst, int64_t bytes, void *stream);

/*
 * Per-kernel timing with HIP events around every launch the plan makes on
 * the stream it is launched on.  enable = 1 starts recording (clears the
 * totals), 0 stops.  Query returns the launch count and the summed event time
 * in milliseconds of one kernel id (synchronises the recorded events).
 */
arrow_status_t arrow_profile_enable(arrow_plan_t p, int32_t enable);
arrow_status_t arrow_profile_query(arrow_plan_t p, int32_t kernel, int64_t *launches,
                                   double *total_ms);

const char *arrow_status_string(arrow_status_t s);
const char *arrow_last_error(void);
/* Library version, e.g. "1.0.0". */
const char *arrow_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ARROW_H */
