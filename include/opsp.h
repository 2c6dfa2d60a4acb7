/*
 * opsp - row-wise sparse general matrix multiplication C = A * B on AMD
 * Instinct MI355X (gfx950), after OpSparse (Du et al., arXiv 2206.07244).
 *
 * C ABI.  No HIP or torch types appear in any signature: streams are passed
 * as `void*` (a hipStream_t, NULL = the default stream) and every matrix
 * array is a plain device pointer.
 *
 * Matrix format (Section 2.1.1, CSR): `rpt` int64[rows+1] holds absolute
 * offsets into `col` int32[nnz] and `val` double[nnz]; rpt[0] need not be 0,
 * so a range of rows of a matrix is itself a valid matrix (a zero-copy
 * view).  Inputs must be canonical: column indices strictly ascending inside
 * each row, all in [0, cols).  Outputs are canonical with rpt[0] == 0.
 *
 * Result definition (Section 2.1, Eq. 1 / Eq. 2): C_ij = sum_k A_ik * B_kj
 * over the *structural* product, i.e. C holds every (i,j) for which some k
 * has both A_ik and B_kj stored, even when the sum is exactly zero
 * (the symbolic step of Section 2.2 sees indices only).  Values are FP64 and
 * summed in an unspecified order (hash-table atomics), so they may differ
 * from a sequential sum in the last bits; rows and columns are exact.
 *
 * Errors: every call returns an opsp_status; nothing throws across the ABI.
 * On error no memory stays allocated by the call and *C is zeroed.
 * Thread safety: calls on distinct streams may run concurrently from
 * different host threads.
 */
#ifndef OPSP_H
#define OPSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OPSP_OK = 0,
    OPSP_ERR_INVALID = 1,   /* NULL pointer, negative size, bad argument, non-canonical input (validation mode) */
    OPSP_ERR_SHAPE = 2,     /* A.cols != B.rows, or a size beyond the index types */
    OPSP_ERR_ALLOC = 3,     /* device allocation failed */
    OPSP_ERR_OVERFLOW = 4,  /* a count exceeds its index type (e.g. a row of C above 2^31-1 entries) */
    OPSP_ERR_HIP = 5,       /* a HIP runtime call or kernel launch failed */
    OPSP_ERR_INTERNAL = 6,  /* internal consistency check failed */
    OPSP_ERR_NO_DEVICE = 7, /* no usable gfx950 device */
    OPSP_ERR_SCRATCH = 8    /* the product needs more scratch than the fixed buffer of
                               opsp_spgemm_numeric_noalloc holds */
} opsp_status;

/* A CSR matrix in device memory (see the format note above). */
typedef struct {
    int64_t rows, cols, nnz;
    int64_t *rpt;
    int32_t *col;
    double *val;
} opsp_csr;

/* Number of bins per step.  Symbolic: bins 0..7 use workgroup-local (LDS)
 * hash tables, and rows of bin 7 whose count crosses the abort threshold are
 * recomputed in global-memory tables ("bin 8").  Numeric: bins 0..6 use LDS
 * tables, bin 7 global-memory tables (Section 5.6, Tables of kernel
 * configuration). */
#define OPSP_SYM_BINS 9
#define OPSP_NUM_BINS 8

/* Optional tuning / test controls.  Pass NULL for the defaults.
 * Set `version` to OPSP_CONFIG_VERSION; zero-initialised fields take their
 * defaults.  Version 1 and 2 structs (without the explicit bin bounds, or
 * without the stream count) are still accepted. */
#define OPSP_CONFIG_VERSION 3
typedef struct {
    int32_t version;
    /* Binning ratio (Section 5.7): a row goes to the first table whose size is
     * at least `ratio` x its n_prod (symbolic) or nnz (numeric).
     * 0 = defaults 1.2 (symbolic) and 2.0 (numeric).  Must be >= 1. */
    double sym_ratio;
    double num_ratio;
    /* Route every row that fits bin b (value <= the bin's upper bound) to
     * bin b instead of its natural bin; larger rows keep their natural bin.
     * -1 = off.  Symbolic b in 0..8 (8 = global tables), numeric 0..7. */
    int32_t force_sym_bin;
    int32_t force_num_bin;
    /* Fraction of the largest symbolic LDS table at which a row is abandoned
     * and recomputed with a global table (Section 5.6.1: 0.8).  0 = default
     * 0.8; a negative value means "abort every row of that bin". */
    double sym_abort_fraction;
    /* Reserved, must be 0 (the lane mapping of products is chosen per chunk
     * of A entries from the lengths of the referenced B rows). */
    int32_t b_lanes;
    /* Record per-stage times in opsp_stats.ms_stage (adds device syncs). */
    int32_t stage_timing;
    /* Check the internal consistency counters after the call (adds a
     * device sync). */
    int32_t validate;
    /* Testing: > 0 launches the symbolic bin kernels (and numeric bin 0)
     * with this fixed grid, the workgroups walking the bin's rows with a
     * grid-stride loop (the launch form that captured graphs use for the
     * symbolic step); 0 = one team per row. */
    int32_t fixed_grid;
    /* Version >= 2: explicit inclusive upper bounds of bins 0..6 of each
     * step (symbolic: on n_prod, bin 7 takes larger rows; numeric: on nnz,
     * bin 7 = global tables takes larger rows).  0 = from the ratio,
     * -1 = the bin takes no rows, otherwise at most the bin's table size
     * (opsp_table_sizes).  A row goes to the first bin whose bound it does
     * not exceed, so the bounds need not be monotone.  This is what the
     * autotuner searches. */
    int64_t sym_bounds[7];
    int64_t num_bounds[7];
    /* Version >= 2: 1 = every row takes the hash tables, as in the paper;
     * 0 = rows whose output columns span a short range are counted in a
     * bitmap of that range (symbolic) and accumulated in a dense array of it
     * (numeric), which gives the same result without probing. */
    int32_t hash_all_rows;
    /* Version >= 3: streams that the bin kernels of each step are spread
     * over (Section 5, computation flow: bins run concurrently, the longest
     * rows' kernels launched first): the calling stream takes the longest-row
     * bins, up to three library-owned side streams of default priority take
     * the others, and the calling stream waits for them before the step's
     * result is used.  0 = the library default (1: the calling stream
     * only), at most 4. */
    int32_t streams;
    /* Version >= 3: lanes per row of bin 0, the bin that packs several short
     * rows into one 256-lane workgroup: 4, 8 or 16, with per-row tables of
     * 64 / 128 / 256 keys (symbolic) and 19 / 39 / 79 entries (numeric), the
     * same LDS per workgroup.  0 = 8.  The one-phase product always uses 8.
     * Bin 0's ratio bound follows the table size; explicit bounds of bin 0
     * may not exceed it. */
    int32_t group_lanes;
} opsp_config;

/* Counters of one call (filled when a stats pointer is given). */
typedef struct {
    int64_t nprod;                         /* total intermediate products, sum_i n_prod_i */
    int64_t nnz;                           /* nnz(C) */
    int64_t max_row_nprod;
    int64_t max_row_nnz;
    int64_t sym_bin_rows[OPSP_SYM_BINS];   /* rows per symbolic bin; [8] = rows recomputed globally */
    int64_t num_bin_rows[OPSP_NUM_BINS];
    /* Stage times in ms when config.stage_timing != 0:
     * two-phase calls: 0 setup+binning, 1 symbolic, 2 numeric
     *   binning+scan+allocation, 3 numeric, 4 total, 5 the numeric
     *   kernel of the longest rows (bin 7) alone (0 when it did not run),
     *   6 the setup kernels alone (within 0; the first binning pass is
     *   fused into the setup kernel);
     * opsp_spgemm_learned: 0 setup+capacities+binning+slot scan,
     *   1 one-phase numeric, 2 recompute+row-pointer scan+allocation of C,
     *   3 copy into C, 4 total */
    float ms_stage[8];
    /* opsp_spgemm_learned only (0 otherwise): */
    int64_t cap_total;            /* sum of the row capacities (temporary slots) */
    int64_t arena_entries;        /* entries stored in the overflow arena */
    int64_t slot_overflow_rows;   /* rows with nnz above their capacity, stored in the arena */
    int64_t table_overflow_rows;  /* rows whose hash table filled up (recomputed exactly) */
    int64_t retry_rows;           /* rows recomputed exactly (table full or arena exhausted) */
    double calib_scale;           /* calibration sample: sum of exact sizes / sum of the
                                   * estimates over all counted rows (1 = none) */
} opsp_stats;

typedef struct opsp_plan opsp_plan;       /* opaque */

/* Version string of the library. */
const char *opsp_version(void);

/* Human-readable name of a status code (static storage). */
const char *opsp_status_string(opsp_status s);

/* C = A * B (two-phase method of Section 2.2 with the six steps of
 * Section 5: setup, symbolic binning, symbolic, numeric binning + scan +
 * allocation of C, numeric, cleanup).
 *   A, B   : read-only device inputs, borrowed until the stream work ends.
 *   C      : output; C->rpt/col/val are allocated by the library from its
 *            device-memory cache and owned by the caller afterwards
 *            (release with opsp_csr_free).  nnz(C) == 0 gives col = val =
 *            NULL and a valid rpt of zeros.
 *   stream : hipStream_t or NULL.  The host blocks once, to read nnz(C)
 *            and the numeric bin sizes (the symbolic bin kernels take their
 *            row counts from device memory); with config.hash_all_rows or
 *            B.cols above 2^23 it blocks once more, to size the global hash
 *            tables.  C is complete once the stream reaches the point of
 *            return. */
opsp_status opsp_spgemm(const opsp_csr *A, const opsp_csr *B, opsp_csr *C, void *stream);

/* As opsp_spgemm, with tuning/test controls and counters (either may be
 * NULL). */
opsp_status opsp_spgemm_ex(const opsp_csr *A, const opsp_csr *B, opsp_csr *C,
                           const opsp_config *config, opsp_stats *stats, void *stream);

/* Symbolic phase only (Section 2.2): runs setup, symbolic binning, the
 * symbolic step, numeric binning and the row-pointer scan.  Returns nnz(C)
 * in *nnzC and a plan that keeps C's row pointer and the numeric bins.
 * A and B must keep their structure (rpt/col) until the plan is destroyed. */
opsp_status opsp_spgemm_symbolic(const opsp_csr *A, const opsp_csr *B, const opsp_config *config,
                                 opsp_plan **plan, int64_t *nnzC, void *stream);

/* Numeric phase for a plan (Section 2.2): may be called repeatedly when A and
 * B change values but not structure.  For each of C->rpt/col/val: NULL means
 * "allocate it" (caller owns it afterwards); non-NULL means a caller device
 * buffer of rows+1 / nnzC / nnzC elements that is filled in. */
opsp_status opsp_spgemm_numeric(opsp_plan *plan, const opsp_csr *A, const opsp_csr *B,
                                opsp_csr *C, void *stream);

/* Numeric phase for a plan that allocates nothing, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  Same result as opsp_spgemm_numeric.
 *   C      : caller buffers, all required: C->rpt int64[rows+1], C->col
 *            int32[nnzC] and C->val double[nnzC] (col/val may be NULL when
 *            nnzC == 0).  On success C->rows/cols/nnz are set; on error the
 *            pointers are left as they were.
 *   scratch: the long-row bin (numeric bin 7: staging of the bucketed kernel,
 *            or the global hash tables) works in one fixed device buffer of
 *            OPSP_NOALLOC_SCRATCH_BYTES per GPU, reserved when the library is
 *            loaded and held until the process ends.  Its grid is cut to what
 *            fits; a product whose single workgroup needs more (bucketed:
 *            12 (max row n_prod + 1) + 512 bytes; hashed: 12 next_pow2(2 max
 *            row nnz) + 512 bytes) returns OPSP_ERR_SCRATCH.  Every call on
 *            a GPU shares that GPU's buffer: calls that overlap in time on one
 *            GPU (two streams, two threads) race and give wrong results.
 *   No hipMalloc, hipFree, pool or cache allocation and no host
 *   synchronisation happen inside the call; the internal consistency check
 *   of a validating plan is not run.  C is complete when the stream reaches
 *   the point of return. */
#define OPSP_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
opsp_status opsp_spgemm_numeric_noalloc(opsp_plan *plan, const opsp_csr *A, const opsp_csr *B,
                                        opsp_csr *C, void *stream);

/* Release a plan (stream-ordered on the plan's last stream). NULL is a no-op. */
void opsp_plan_destroy(opsp_plan *plan);

/* Release the arrays of a C produced by this library (stream-ordered) and
 * zero *C.  NULL arrays are skipped. */
opsp_status opsp_csr_free(opsp_csr *C, void *stream);

/* ---- FP32 values --------------------------------------------------------
 * The same product with single-precision values (the paper evaluates FP64
 * only, Section 6.1; the method is the same for any value type): a CSR
 * matrix whose val is float[nnz], otherwise laid out as opsp_csr.  Products
 * a_ik * b_kj are rounded to float, summed in double in an unspecified order
 * and rounded to float once, so each value of C lies within (number of its
 * terms + 1) units of float rounding of sum_k |a_ik b_kj| from the exact sum
 * of the float inputs; rows and columns are exact.  Structure, allocation,
 * ownership, errors and the single host wait are those of opsp_spgemm_ex
 * (release C with opsp_csr_f32_free). */
typedef struct {
    int64_t rows, cols, nnz;
    int64_t *rpt;
    int32_t *col;
    float *val;
} opsp_csr_f32;
opsp_status opsp_spgemm_f32(const opsp_csr_f32 *A, const opsp_csr_f32 *B, opsp_csr_f32 *C,
                            const opsp_config *config, opsp_stats *stats, void *stream);
opsp_status opsp_csr_f32_free(opsp_csr_f32 *C, void *stream);

/* ---- Batched products --------------------------------------------------
 * `count` independent products C_p = A_p * B_p computed as ONE block-diagonal
 * product over the concatenation of their rows (rows of C are independent,
 * Section 2.1): one pass of setup, binning, symbolic, scan and numeric covers
 * all problems.  The work runs as two captured graphs: the structure graph
 * (everything up to the row pointer, with the symbolic bin kernels launched
 * persistently because their bin sizes are only known on the device) and,
 * after one host read-back of nnz and the numeric bin sizes, the value graph
 * (value gather + numeric kernels).  Both graphs are replayed by later
 * executions of the same batch object.
 *
 * opsp_batch_create: A[p], B[p] (device CSR, A[p].cols == B[p].rows) are
 *   borrowed by the batch object until it is destroyed; their structure must
 *   not change, their values may (each execution reads them).  Problems may
 *   be empty.  1 <= count <= 65535.
 * opsp_batch_execute: fills C[0..count) with views into storage owned by the
 *   batch: C[p].rpt points into a shared row pointer holding absolute offsets
 *   (C[p].rpt[0] is generally not 0), C[p].col / C[p].val are the shared
 *   arrays.  Views stay valid until the next execution or destroy.  The host
 *   blocks once per execution (the read-back); C is complete when the stream
 *   reaches the point of return.  stats may be NULL.
 * opsp_spgemm_batched: create + execute; *owner receives the batch object
 *   that owns the views (release with opsp_batch_destroy). */
typedef struct opsp_batch opsp_batch;
opsp_status opsp_batch_create(int32_t count, const opsp_csr *A, const opsp_csr *B,
                              const opsp_config *config, opsp_batch **batch, void *stream);
opsp_status opsp_batch_execute(opsp_batch *batch, opsp_csr *C, opsp_stats *stats, void *stream);
void opsp_batch_destroy(opsp_batch *batch);
opsp_status opsp_spgemm_batched(int32_t count, const opsp_csr *A, const opsp_csr *B, opsp_csr *C,
                                const opsp_config *config, opsp_batch **owner, void *stream);

/* ---- Row-size predictor and the one-phase product ------------------------
 * An extension beyond the paper.  Section 2.2 names the one-phase
 * alternative to the two-phase method: each row is computed straight into
 * space reserved from a bound on its size, and the rows are then copied into
 * a compact C (temporary space and a copy are its two costs).  Here the bound
 * of row i comes from a small network that predicts nnz(C_i*) from three
 * features of the row, so no symbolic pass runs:
 *   features  x_i = log2(1 + v) for v = (a_len_i, n_prod_i, b_max_i), float32:
 *             the entries of A's row i, its intermediate products, and the
 *             longest row of B that it references;
 *   network   3 -> 64 -> 64 -> 1, ReLU, bfloat16 parameters packed as
 *             W1[64][3], b1[64], W2[64][64], b2[64], W3[64], b3 (row-major,
 *             OPSP_MLP_NPARAM bit patterns), predicting y_i = log2(1 + nnz_i):
 *               z1 = ((b1 + w0 x0) + w1 x1) + w2 x2   float32, no fused ops
 *               h1 = bf16(relu(z1))                   nearest, ties to even
 *               y  = W3 relu(W2 h1 + b2) + b3        float32 accumulation
 *   capacity  cap_i = ceil((2^y_i - 1) c (1 + margin)) clamped to
 *             [min(b_max_i, U_i), U_i] with U_i = min(n_prod_i, N); a row
 *             with a_len_i <= 1 gets n_prod_i (exact); c is the calibration
 *             factor of the row's n_prod octave from a small exactly counted
 *             sample of rows (see calib_rows), which corrects the network's
 *             bias on the input at hand (1 where the sample has too few rows).
 * Whatever the capacities, the result is the C of opsp_spgemm (same
 * structure; values summed in unspecified order): a row that outgrows its
 * capacity is stored in an overflow arena, and a row whose hash table fills
 * up is recomputed exactly with a table sized from U_i. */
#define OPSP_MLP_NPARAM 4481
#define OPSP_PREDICTOR_VERSION 1
typedef enum {
    OPSP_PRED_MLP = 0,    /* the network above */
    OPSP_PRED_UPPER = 1,  /* cap_i = U_i: the upper-bound one-phase method */
    OPSP_PRED_RATIO = 2   /* cap_i = ceil(n_prod_i / ratio * (1 + margin)), clamped as above */
} opsp_predictor_kind;

typedef struct {
    int32_t version;          /* OPSP_PREDICTOR_VERSION */
    int32_t kind;             /* opsp_predictor_kind */
    const uint16_t *params;   /* device; OPSP_MLP_NPARAM bfloat16 bit patterns (kind MLP) */
    double margin;            /* >= 0 */
    double ratio;             /* kind RATIO: assumed n_prod / nnz, > 0 */
    double cap_scale;         /* testing: capacities multiplied by this and floored
                               * after clamping (0 = 1), e.g. 0.1 to overflow rows */
    float *pred_out;          /* optional device float[A.rows]: network outputs y_i */
    int64_t *cap_out;         /* optional device int64[A.rows]: capacities */
    /* Kind MLP: calibration, the most rows sampled per octave of n_prod.
     * Rows with a_len >= 2, 1 <= n_prod < 2^21 and an output column range
     * of at most 2^23 columns are grouped by o = floor(log2 n_prod); of an octave's
     * c rows, about K = min(c, clamp(2^24 >> o, 4, calib_rows)) are picked
     * (row i with probability K / c: when u(i) * c < K * 2^32, u(i) the
     * high 32 bits of MurmurHash3's 64-bit finalizer fmix64(i); every row
     * when c <= K) and counted exactly on the device.  In an
     * octave with at least 4 counted rows every row's estimate 2^y_i - 1 is
     * multiplied by the largest size / estimate (clamped as above) of the
     * counted rows before the margin; other rows are not scaled.
     * 0 = 64; negative = no calibration. */
    int32_t calib_rows;
    int32_t reserved;
} opsp_predictor;

/* Integer features of every row of A*B into device arrays of A->rows
 * elements (any may be NULL). */
opsp_status opsp_row_features(const opsp_csr *A, const opsp_csr *B, int32_t *a_len,
                              int64_t *n_prod, int32_t *b_max, void *stream);

/* Network inputs x_i (float32 [A->rows][3], device) of every row of A*B. */
opsp_status opsp_mlp_features(const opsp_csr *A, const opsp_csr *B, float *X, void *stream);

/* y[i] = network(X[i]) for n rows (device arrays float[n][3] -> float[n]). */
opsp_status opsp_mlp_forward(const uint16_t *params, const float *X, int64_t n, float *y,
                             void *stream);

/* Loss over n >= 1 rows and its gradient with respect to the OPSP_MLP_NPARAM
 * parameters (float32, same packing), evaluated at the bfloat16 parameters,
 * with the rounding of h1 passed straight through.  tau == 0: mean squared
 * error L = sum_i (y_i - target_i)^2 / n; 0 < tau < 1: mean pinball loss of
 * level tau, L = sum_i rho(target_i - y_i) / n with rho(r) = tau r for r > 0
 * and (tau - 1) r otherwise (the network then estimates the tau-quantile of
 * the row size).  grad: device float[OPSP_MLP_NPARAM]; loss: device float[1]
 * or NULL. */
opsp_status opsp_mlp_grad(const uint16_t *params, const float *X, const float *target, int64_t n,
                          float tau, float *grad, float *loss, void *stream);

/* One Adam step (Kingma and Ba, 2015) on float32 master parameters with
 * moments m, v (device float[OPSP_MLP_NPARAM] each, updated in place), step
 * counted from 1; writes the rounded bfloat16 copy into params. */
opsp_status opsp_mlp_adam(float *master, float *m, float *v, const float *grad, int64_t step,
                          float lr, float beta1, float beta2, float eps, uint16_t *params,
                          void *stream);

/* C = A * B by the one-phase method with predicted capacities (see above):
 * setup with the three features, capacities (network inference on the
 * matrix cores), numeric binning by capacity and a scan of the capacities
 * into slot offsets, one read-back, the numeric hash-accumulate kernels
 * writing each row into its slot or the arena, the exact recompute of rows
 * whose tables filled up, the scan of the exact row sizes, one read-back,
 * allocation of C and the copy into C.  The host blocks two times (three
 * when rows are recomputed).  Ownership and errors as for opsp_spgemm;
 * config fields sym_* and fixed_grid are ignored.  stats may be NULL. */
opsp_status opsp_spgemm_learned(const opsp_csr *A, const opsp_csr *B, opsp_csr *C,
                                const opsp_predictor *predictor, const opsp_config *config,
                                opsp_stats *stats, void *stream);

/* Device memory of the library (workspaces and C arrays) comes from a
 * per-device cache: blocks released by the library or by opsp_csr_free are
 * kept, per stream and size class, and handed out again to later calls on the
 * same stream without any HIP allocation call (on this stack a pool
 * allocation or release costs tens to hundreds of microseconds of host
 * time).  opsp_cache_release() synchronises the current device, returns
 * every cached block to HIP and trims the device's default memory pool, so
 * that the memory is free for other allocators of the process;
 * opsp_cache_bytes() reports what is cached on the current device. */
opsp_status opsp_cache_release(void);
int64_t opsp_cache_bytes(void);

/* Bytes of the blocks that the cache has handed out on the current device
 * and not yet taken back (C arrays a caller still holds included).  A call
 * that fails leaves this where it was before the call. */
int64_t opsp_cache_live_bytes(void);

/* Testing hook: after the next n successful allocations of the library,
 * the following one fails as if the device were out of memory (once);
 * n < 0 switches the hook off.  Lets a test drive every error exit of a
 * call and check that nothing stays allocated. */
void opsp_debug_fail_alloc(int64_t n);

/* Host-side helpers (no device work; usable without a GPU).
 * Table sizes of the per-bin hash tables, in entries (-1 = global-memory
 * table), for step 0 = symbolic (OPSP_SYM_BINS entries) or 1 = numeric
 * (OPSP_NUM_BINS entries). */
opsp_status opsp_table_sizes(int32_t step, int64_t *out, int32_t n);

/* Inclusive upper bounds of bins 0..n-2 for table sizes `tsize[0..n-2]` and
 * a ratio (Section 5.7): symbolic floor(t/ratio), numeric
 * min(t, floor((t+1)/ratio)); the last bin is unbounded. */
opsp_status opsp_bin_bounds(int32_t step, const int64_t *tsize, int32_t n, double ratio,
                            int64_t *out);

#ifdef __cplusplus
}
#endif
#endif /* OPSP_H */
