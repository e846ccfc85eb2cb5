/*
 * spk.h -- C ABI of libspk, autotuned bandwidth-bound sparse and vector
 * kernels for AMD Instinct MI355X (gfx950).
 *
 * The library implements, as hand-written HIP kernels, the operations the
 * paper's annotation-based autotuning targets (Mametjanov & Norris,
 * "Software Autotuning for Sustainable Performance Portability"):
 *   - the vector update of Figure 1, read as WAXPY  w = alpha*x + y, with its
 *     in-place form AXPY and the dot product;
 *   - the sparse kernels of the prior GPU work cited in Section 3 (CSR
 *     sparse matrix-vector product y = A*x), in several storage formats;
 *   - one Krylov-style step fusing both: y = A*x, w = alpha*y + x;
 *   - the tuning method of Section 2: enumerate code variants over the
 *     parameters listed in Section 3 (threads per block, blocks per grid,
 *     asynchronous streams, cache-sized staging, unroll factor), run each,
 *     compare its outputs with a reference run, and keep the fastest;
 *   - batched and served execution driven by the tuned variants.
 *
 * General conventions (apply to every function below)
 *   - Every function is extern "C", returns spk_status and never throws.
 *   - Arrays named "device" are GPU memory owned by the caller (e.g. torch
 *     tensors).  The library never frees them; a call borrows them until its
 *     work on the given stream has completed.
 *   - Kernels are enqueued asynchronously on the caller's stream (a
 *     hipStream_t passed as spk_stream; NULL is the null stream).  Only
 *     spk_tune*, spk_matrix_register, spk_batch_plan and spk_serve_*
 *     synchronise.
 *   - Argument, shape and dtype errors are reported before any HIP call.
 *     HIP failures map to SPK_ERR_HIP; spk_last_error() then holds the HIP
 *     message.  A device fault in asynchronous work surfaces at the caller's
 *     next synchronisation (or spk_check()).
 *   - Indices are int32 (nnz < 2^31); sizes are int64.
 *   - Floating point is IEEE round-to-nearest without flush-to-zero; every
 *     multiply-add is fused.  FP32 data are accumulated in FP64 and rounded
 *     once per output.
 *   - n == 0 or nrows == 0 is valid and launches nothing.
 *   - HIP graph capture: spk_spmv_*, spk_waxpy, spk_axpy, spk_dot, spk_run
 *     and spk_cg may be captured into a graph on the caller's stream.  What
 *     they build on first use (a matrix's derived formats, and the dot
 *     partials, column-block partials and CG scratch, which are kept per
 *     stream) is allocated then,
 *     so make one eager call with the same matrix, size and stream before
 *     capturing: a first use inside a capture fails with SPK_ERR_HIP.  The
 *     captured launches record no memset nodes.
 */
#ifndef SPK_H
#define SPK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPK_ABI_VERSION 1

typedef enum {
    SPK_OK = 0,
    SPK_ERR_NULL = 1,        /* a required pointer or handle is NULL */
    SPK_ERR_SHAPE = 2,       /* negative or inconsistent sizes */
    SPK_ERR_DTYPE = 3,       /* unknown dtype or mixed dtypes */
    SPK_ERR_ALIAS = 4,       /* forbidden overlap between inputs and outputs */
    SPK_ERR_CSR = 5,         /* malformed row_ptr / col_idx (registration only) */
    SPK_ERR_OOM = 6,         /* device allocation failed */
    SPK_ERR_BUDGET = 7,      /* request exceeds the server's HBM budget */
    SPK_ERR_HIP = 8,         /* a HIP runtime call failed */
    SPK_ERR_VALIDATION = 9,  /* no variant reproduced the reference output */
    SPK_ERR_NOT_FOUND = 10,  /* unknown id or variant */
    SPK_ERR_ARG = 11,        /* other invalid argument (options, variant fields) */
    SPK_ERR_STATE = 12,      /* call not allowed in the object's current state */
    SPK_ERR_INTERRUPTED = 13 /* a search stopped after opts->stop_after new
                              * points (those points are in the journal) */
} spk_status;

typedef enum { SPK_F32 = 0, SPK_F64 = 1 } spk_dtype;

typedef enum {
    SPK_OP_SPMV = 0,        /* y = A*x */
    SPK_OP_WAXPY = 1,       /* w = alpha*x + y */
    SPK_OP_AXPY = 2,        /* y = alpha*x + y */
    SPK_OP_DOT = 3,         /* d = sum x_i*y_i */
    SPK_OP_SPMV_WAXPY = 4   /* y = A*x; w = alpha*y + x */
} spk_op;

/* Storage format / kernel family of a SpMV variant. */
typedef enum {
    SPK_FMT_AUTO = 0,       /* let the library choose (tuned plan or default) */
    SPK_FMT_SCALAR = 1,     /* CSR, one lane per row */
    SPK_FMT_VECTOR = 2,     /* CSR, `group` lanes per row (64 = one wavefront) */
    SPK_FMT_SELL = 3,       /* sliced ELL, `group` rows per slice, column-major slices */
    SPK_FMT_ADAPTIVE = 4,   /* CSR wavefront tiles staged through LDS (`lds` entries per wavefront) */
    /* Structured formats (registered matrices whose structure qualifies,
     * see spk_matrix_formats; not listed by spk_variant_get, searched by
     * spk_tune when they apply).  They store less than CSR, so their
     * algorithmic bytes differ from the CSR count (spk_matrix_format_bytes). */
    SPK_FMT_DIA = 5,        /* diagonal storage: at most 16 diagonals, one value per
                             * (diagonal, row) plus a 16-bit presence mask per row;
                             * `block` threads, `unroll` rows per lane (1, 2) */
    SPK_FMT_STENCIL = 6,    /* matrix-free: a constant-coefficient 3-, 5- or 7-point
                             * stencil on a 1-, 2- or 3-D grid with Dirichlet
                             * truncation (only the coefficients are stored);
                             * `block` threads, `unroll` rows per lane (1..8),
                             * `lds` 1 = x staged through LDS */
    SPK_FMT_COLBLOCK = 7    /* column-blocked CSR (FP64 registered matrices): the
                             * matrix split by column ranges into `group` (2 or 4)
                             * sub-matrices of all rows, built on first use; one
                             * pass per block with the ADAPTIVE kernel (`block`
                             * threads, `lds` entries per wavefront) into FP64
                             * partials kept per stream, then one pass adds them
                             * in block order (and forms w).  Each pass gathers
                             * from one slice of x only, which pays when x is
                             * larger than an XCD's L2.  Same algorithmic bytes
                             * as CSR; not listed by spk_variant_get, searched
                             * by spk_tune (`formats`) when x exceeds 4 MiB */,
    SPK_FMT_XWIN = 8        /* x staged in LDS by column window (registered
                             * matrices, FP64 and FP32): the columns cut into
                             * windows of `group` KiB of x (128 or 64); the
                             * entries regrouped at first use into (row, window)
                             * pairs, window-major, with 16-bit column indices
                             * inside the window; one pass in which each
                             * workgroup (`block` threads, `lds` row-stream
                             * entries per wavefront) copies one window of x to
                             * LDS and writes an FP64 partial per pair of its
                             * chunk (about `grid` chunks per compute unit), then
                             * one pass adds each row's partials in window order
                             * (and forms w).  The gathers of x never leave the
                             * compute unit.  Not listed by spk_variant_get,
                             * searched by spk_tune (`formats`) when x exceeds
                             * 4 MiB */
} spk_format;

typedef void *spk_stream;                 /* hipStream_t */
typedef struct spk_ctx *spk_handle;       /* library-owned: device, plan DB, scratch */
typedef struct spk_mat *spk_matrix;       /* library-owned resident matrix */
typedef struct spk_batch_s *spk_batch;    /* library-owned batched plan */
typedef struct spk_server_s *spk_server;  /* library-owned serving loop */

/* Borrowed view of a CSR matrix.  row_ptr[nrows+1] (row_ptr[0] == 0,
 * non-decreasing, row_ptr[nrows] == nnz), col_idx[nnz] in [0, ncols),
 * val[nnz] of `dtype`.  Unsorted rows, duplicate columns and explicit zeros
 * are allowed: every stored entry contributes.  Whether the arrays are host
 * or device memory is stated by each function. */
typedef struct {
    int64_t nrows, ncols, nnz;
    int32_t dtype;                 /* spk_dtype */
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const void *val;
} spk_csr;

/* One point of the tuning space (Section 3 lists the parameters: threads per
 * block, blocks per grid, streams, cache size, unroll).  Fields that do not
 * apply to an operation must be 0.
 *   format  spk_format (SpMV only)
 *   block   threads per workgroup (64..1024, power of two)
 *   group   SpMV VECTOR: lanes per row (2..64); SELL: rows per slice
 *   unroll  independent loads in flight per lane (1, 2, 4 or 8)
 *   vec     vector ops: elements per lane load (1, 2 or 4; at most 16 bytes);
 *           SpMV SCALAR/VECTOR: entries per value/index access (0 = one);
 *           ADAPTIVE: 2 = two-byte columns (each row-stream block whose
 *           columns span at most 65,536 reads its columns as offsets from
 *           its first column, a copy the matrix keeps once made; 0 = the
 *           CSR's four-byte columns)
 *   grid    vector ops: 0 = one pass, else workgroups per compute unit of a
 *           grid-stride launch (either way at most 2^30 work-items: past
 *           that the kernels loop over the grid, so any n is covered)
 *   streams SpMV: split rows over this many streams (1, 2 or 4)
 *   lds     SpMV VECTOR: 1 = stage row_ptr in LDS; ADAPTIVE: LDS row-stream
 *           capacity in entries per wavefront (the "L1 size" knob; gfx950
 *           has no L1/LDS split, so the staged tile size takes its place);
 *           STENCIL: 1 = stage each workgroup's x values and one grid line
 *           of halo in LDS (applies while they fit 64 KiB) */
typedef struct {
    int32_t format, block, group, unroll, vec, grid, streams, lds;
} spk_variant;

/* ------------------------------------------------------------- library -- */

/* SPK_ABI_VERSION of the loaded library.  Library plumbing, not in the
 * paper. */
int spk_abi_version(void);

/* Human-readable name of a status code (static storage).  Library plumbing,
 * not in the paper. */
const char *spk_status_str(spk_status s);

/* Creates a handle on HIP device `device`.  `db_path` (nullable) names a
 * tuning database file, where the outcome of Section 2's search is kept:
 * winners found by spk_tune are appended there and loaded by later handles;
 * entries from another GPU architecture or library build are ignored.
 * Environment: SPK_PLAIN=1
 * makes every call use the fixed plain variants; SPK_DB_PATH supplies
 * db_path when it is NULL.  SPK_ERR_NULL without `out`; SPK_ERR_HIP when the
 * device cannot be selected. */
spk_status spk_create(int device, const char *db_path, spk_handle *out);

/* Releases the handle and everything it owns (matrices and batches created
 * from it must be released first).  Library plumbing, not in the paper. */
spk_status spk_destroy(spk_handle h);

/* Message of the calling thread's last non-OK status (static per thread).
 * Library plumbing, not in the paper. */
const char *spk_last_error(void);

/* Waits for `stream` and reports any asynchronous HIP error.  Library
 * plumbing, not in the paper. */
spk_status spk_check(spk_handle h, spk_stream stream);

/* Selects how untuned calls pick variants: 0 = plan DB, else built-in
 * default; 1 = always the fixed plain variants, the analogue of Figure 1's
 * baseline kernel without directives. */
spk_status spk_set_plain(spk_handle h, int plain);

/* Number of compute units and device name (name_cap bytes, NUL-terminated).
 * Library plumbing, not in the paper. */
spk_status spk_device_info(spk_handle h, int32_t *num_cu, char *name, int32_t name_cap);

/* ------------------------------------------------------- vector kernels -- */

/* WAXPY (the vector update of Figure 1): w_i = alpha*x_i + y_i, one fused
 * rounding.  x, y, w: device arrays of n elements of `dtype`.  w may be
 * identical to x or y (element-wise update); any other overlap is
 * SPK_ERR_ALIAS.  For SPK_F32, alpha is rounded to float first.  alpha == 0
 * is not special-cased (0*Inf = NaN propagates). */
spk_status spk_waxpy(spk_handle h, int32_t dtype, int64_t n, double alpha,
                     const void *x, const void *y, void *w, spk_stream stream);

/* AXPY: y_i <- alpha*x_i + y_i, the vector update of Figure 1 done in
 * place (WAXPY with w == y), one fused rounding per element.  x, y: device
 * arrays of n elements of `dtype`; x may equal y (then y_i <- (alpha+1)*y_i
 * rounded once); any partial overlap is SPK_ERR_ALIAS.  For SPK_F32 alpha is
 * rounded to float first.  n == 0 launches nothing; SPK_ERR_NULL for a NULL
 * array with n > 0. */
spk_status spk_axpy(spk_handle h, int32_t dtype, int64_t n, double alpha,
                    const void *x, void *y, spk_stream stream);

/* Dot product d = sum_i x_i*y_i.  Not in the paper: one of the vector
 * operations of the configured vector sweep, kept beside WAXPY/AXPY because
 * a Krylov step needs it.  x, y: device arrays of n elements of `dtype`
 * (may be the same array); the sum is accumulated in FP64 and written to
 * d_result[0] (device, one double, also for SPK_F32; n == 0 writes 0).  The
 * reduction order is fixed for a given (n, variant), so repeated calls are
 * bit-identical.  The per-workgroup partial sums live in scratch the handle
 * allocates per stream on first use.  Calls on one handle and one stream are
 * serialised by the stream; calls on different streams use separate
 * scratch. */
spk_status spk_dot(spk_handle h, int32_t dtype, int64_t n, const void *x, const void *y,
                   double *d_result, spk_stream stream);

/* spk_dot for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels, variant and result bits as spk_dot, but the
 * partial sums and the ticket live in a fixed per-GPU array of the library
 * (65,536 partials, 512 KiB plus one 256-byte line, held by each GPU the
 * library runs on until the process ends) instead of scratch the handle
 * allocates; the call allocates nothing, launches a small kernel that zeroes
 * the ticket, then the dot.  A dot whose variant needs more than 65,536
 * workgroups (only the one-pass plain variant, above 16.7M elements) is
 * rejected with SPK_ERR_SHAPE.  Every call on a GPU, from any handle or
 * stream, shares that GPU's array: calls that overlap on one GPU race and
 * give wrong results, so serialise them (one stream, or events). */
spk_status spk_dot_noalloc(spk_handle h, int32_t dtype, int64_t n, const void *x, const void *y,
                           double *d_result, spk_stream stream);

/* ----------------------------------------------------------------- SpMV -- */

/* y = A*x for a borrowed CSR matrix: the sparse matrix-vector product of
 * the prior GPU work that Section 3 cites (the paper's spmv_csr(A, x, y)).
 * All arrays are device memory owned by the caller: row_ptr int32[nrows+1],
 * col_idx int32[nnz], val[nnz], x[ncols] and y[nrows], all of A->dtype.
 * y_i = sum over row i's stored entries of val_k * x[col_k], FP64
 * accumulation (FP32 data rounded once); an empty row gives +0.  y must not
 * overlap x (SPK_ERR_ALIAS).  Only O(1) facts are checked (pointers, sizes,
 * dtype, aliasing); row_ptr/col_idx contents are trusted (use
 * spk_matrix_register(validate=1) to check them).  nrows == 0 or
 * ncols == 0 is valid (y is set to zeros when ncols == 0).  Formats that need
 * derived data (SELL, ADAPTIVE, structured) are only available on
 * registered matrices, so this call uses the SCALAR/VECTOR families. */
spk_status spk_spmv_csr(spk_handle h, const spk_csr *A, const void *x, void *y, spk_stream stream);

/* Copies a CSR matrix into library-owned device memory and derives the
 * metadata its formats need (row statistics, LDS row blocks, sliced ELL on
 * first use): the operand A of the sparse kernels of Section 3, kept
 * resident so that repeated products (and the tuner's variant runs of
 * Section 2) do not upload it again.  Beyond the spmv_csr(A, x, y)
 * interface, the arrays may come from either side: `where` 0 = the arrays
 * of A are host memory, 1 = device memory.  validate != 0 checks row_ptr
 * monotonicity, row_ptr[0] == 0, row_ptr[nrows] == nnz and
 * 0 <= col_idx < ncols (SPK_ERR_CSR otherwise).  The caller may free its
 * arrays when this returns; the matrix is owned by the handle until
 * spk_matrix_release.  Synchronises.  SPK_ERR_OOM when device memory runs
 * out. */
spk_status spk_matrix_register(spk_handle h, const spk_csr *A, int32_t where, int32_t validate,
                               spk_matrix *out);

/* Frees a registered matrix and its derived formats.  Library plumbing, not
 * in the paper. */
spk_status spk_matrix_release(spk_handle h, spk_matrix A);

/* Bytes of device memory held by a registered matrix (CSR plus derived
 * formats built so far).  Library plumbing, not in the paper. */
spk_status spk_matrix_bytes(spk_handle h, spk_matrix A, int64_t *bytes);

/* Formats that apply to A, as a bitmask of (1 << spk_format): SCALAR,
 * VECTOR, SELL and ADAPTIVE always; DIA when every stored entry lies on at
 * most 16 diagonals with no duplicate (row, column); STENCIL when A is
 * exactly a constant-coefficient grid stencil: offsets {0, +-1} (1-D),
 * {0, +-1, +-s} (2-D, s | n) or {0, +-1, +-s, +-t} (3-D, s | t, t | n),
 * every neighbour inside the grid present, none outside, and one value per
 * offset.  The structure is detected at registration (Section 3's prior
 * GPU work counts the storage format among the choices a tuner makes). */
spk_status spk_matrix_formats(spk_handle h, spk_matrix A, uint32_t *mask);

/* The structure spk_matrix_register detects, computed from host arrays
 * alone (no GPU, no handle): `formats` as spk_matrix_formats reports it,
 * the diagonal offsets when DIA applies, and the grid and coefficients
 * (ascending offset order -N2*N3, -N3, -1, 0, +1, +N3, +N2*N3; absent
 * slots 0) when STENCIL applies.  row_ptr, col_idx and val of `csr` are
 * host pointers here.  Structure detection for the storage-format choice of
 * Section 3. */
typedef struct {
    uint32_t formats;
    int32_t ndiag;
    int32_t offsets[16];
    int32_t dim;             /* 0 (no stencil), 1, 2 or 3 */
    int32_t n1, n2, n3;      /* grid, slowest to fastest axis */
    double coef[7];
} spk_structure;

spk_status spk_csr_structure(const spk_csr *csr, spk_structure *out);

/* Measurement, not in the paper.  Algorithmic bytes of one SpMV (fused: +
 * the w stream) of A in `format`
 * (SCALAR/VECTOR/ADAPTIVE: the CSR count; SELL: the CSR count; DIA:
 * ndiag*m values + 2m mask bytes; STENCIL: none for the matrix) plus x and
 * y.  SPK_ERR_ARG when the format does not apply to A. */
spk_status spk_matrix_format_bytes(spk_handle h, spk_matrix A, int32_t format, int32_t fused, int64_t *bytes);

/* y = A*x on a registered matrix (the sparse product of Section 3's prior
 * GPU work), with the variant Section 2's search recorded for its shape
 * class, or the built-in default when none is recorded.  x: device,
 * A.ncols elements; y: device, A.nrows elements; both of A's dtype; y must
 * not overlap x (SPK_ERR_ALIAS).  Asynchronous on `stream`; a format built
 * on first use (sliced ELL, DIA, column blocks) is built then, on the same
 * stream. */
spk_status spk_spmv_mat(spk_handle h, spk_matrix A, const void *x, void *y, spk_stream stream);

/* One Krylov-style step on a square registered matrix: the sparse product
 * of Section 3 followed by the vector update of Figure 1, fused: y = A*x,
 * then w_i = alpha*y_i + x_i (one rounding) from the rounded y_i, in one
 * kernel.  x, y, w: device, A.nrows elements of A's dtype.  w must not
 * overlap x or y; y must not overlap x (SPK_ERR_ALIAS); a non-square matrix
 * is SPK_ERR_SHAPE. */
spk_status spk_spmv_waxpy(spk_handle h, spk_matrix A, double alpha, const void *x, void *y,
                          void *w, spk_stream stream);

/* ------------------------------------------------- conjugate gradients -- */

/* Conjugate gradients on a square symmetric positive definite registered
 * FP64 matrix: `iters` iterations of the textbook recurrence (r = b - A x,
 * p = r; per iteration q = A p, alpha = r.r / p.q, x += alpha p,
 * r -= alpha q, beta = r'.r' / r.r, p = r + beta p), a step size whose
 * denominator is exactly zero being taken as zero.  The iteration is not in
 * the paper: it is the Krylov solver whose per-iteration kernels are the
 * vector update of Figure 1 and the SpMV of Section 3, i.e. the hotspot
 * kernels Section 1 sets out to specialize.  Each iteration is three
 * launches with the scalars kept on the device (no host round trip): the
 * SpMV fused with p.q, the residual update fused with r.r, and the x and
 * direction updates in one pass over p.  The SpMV+dot kernel is the one
 * spk_cg_tune recorded for A's class (a CSR wavefront-tile shape, or the
 * matrix-free form when A is a constant-coefficient grid stencil), else a
 * default tile shape.
 *   b        device, n doubles (right-hand side), read only
 *   x        device, n doubles, 8-byte aligned: initial guess on entry, the
 *            iterate after `iters` iterations on return
 *   d_rr_hist device, iters + 1 doubles: r_k.r_k for k = 0..iters
 * Asynchronous on `stream`; the solve's working vectors are owned by the
 * handle (one set per stream, grown on demand), so solves on one stream run
 * one after another and must not be issued from several threads at once.  Errors: SPK_ERR_DTYPE for
 * FP32 matrices, SPK_ERR_SHAPE for a non-square matrix or iters < 0,
 * SPK_ERR_ALIAS when x overlaps b or the history. */
spk_status spk_cg(spk_handle h, spk_matrix A, const void *b, void *x, int32_t iters, double *d_rr_hist,
                  spk_stream stream);

/* ------------------------------------------------- variants and tuning -- */

/* A problem for spk_run / spk_tune: one call of an operation above, the
 * unit Section 2's search runs, compares and times.  SPMV/SPMV_WAXPY use A
 * (registered) and x, y (and w); WAXPY uses x, y, w; AXPY x, y; DOT x, y and
 * d_result.  The operation travels inside the problem (`op`) rather than as
 * a separate argument of spk_tune, so that spk_run and spk_tune share one
 * description of it. */
typedef struct {
    int32_t op;          /* spk_op */
    int32_t dtype;       /* vector ops; SpMV takes A's dtype */
    int64_t n;           /* vector ops */
    double alpha;
    spk_matrix A;
    const void *x;
    void *y;
    void *w;
    double *d_result;
} spk_problem;

/* Runs `problem` with an explicit variant (NULL = the dispatcher's choice):
 * one code variant of Section 2's search.  Used by the tuner and by tests
 * that exercise every compiled variant.  SPK_ERR_ARG for a variant outside
 * the compiled space. */
spk_status spk_run(spk_handle h, const spk_problem *problem, const spk_variant *variant,
                   spk_stream stream);

/* The variant space compiled into the library for an op and dtype (the
 * parameter variations of Section 3: threads per block, unroll, streams,
 * cache-sized staging, plus the storage format): spk_variant_count gives
 * its size, spk_variant_get the i-th point. */
spk_status spk_variant_count(int32_t op, int32_t dtype, int32_t *count);
spk_status spk_variant_get(int32_t op, int32_t dtype, int32_t index, spk_variant *out);

/* The fixed "plain" variants, the analogue of the paper's unannotated
 * -O3 baseline (Figure 1): one element per thread and 256 threads for the
 * vector ops; for SpMV index 0 = one lane per row, 1 = one wavefront per
 * row, both 256 threads, no unroll, no LDS, plain CSR. */
spk_status spk_plain_variant(int32_t op, int32_t which, spk_variant *out);

typedef struct {
    int32_t reps;            /* timed repetitions per variant (0 -> 10) */
    int32_t warmup;          /* untimed runs per variant (0 -> 2) */
    int32_t flush;           /* 1: evict the last-level cache before each timed rep */
    int32_t max_variants;    /* 0 = the whole pruned space */
    double tau;              /* per-row tolerance factor (0 -> 1e-12 FP64, 1e-5 FP32) */
    const double *ref_host;  /* optional host reference: y (SpMV), w (WAXPY/AXPY,
                              * as doubles), d (DOT, one double); NULL = a run of
                              * the plain variant is the reference (Section 2) */
    const double *ref_scale; /* with ref_host: per-output tolerance scale
                              * (SpMV: sum_k |a_ik x_k|; DOT: sum |x_i y_i|);
                              * NULL = computed on the device */
    int32_t record;          /* 1: store the winner in the handle's plan DB */
    int32_t verbose;         /* 1: print one line per variant to stderr */
    uint32_t formats;        /* SpMV: bitmask (1 << spk_format) of the formats to
                              * search; 0 = every format that applies to A */
    int32_t resume;          /* spk_tune / spk_batch_tune: 1 = journal every timed
                              * point (search key, variant, median) as one line
                              * of the plan DB as soon as it is measured, and
                              * take points journaled before (same search key,
                              * arch and build) instead of running them again;
                              * 0 = neither.  spk_cg_tune: must be 0 */
    int32_t stop_after;      /* >0: validate and time at most this many points
                              * not already journaled, then stop with
                              * SPK_ERR_INTERRUPTED, recording no winner (a
                              * search cut short); 0 = no limit */
} spk_tune_opts;

typedef struct {
    spk_variant best;
    double best_us;          /* median time of the winner */
    double plain_us;         /* median time of the better plain variant */
    int32_t tried;           /* variants timed */
    int32_t rejected;        /* variants whose output failed validation */
    int32_t pruned;          /* variants skipped by the byte model */
    char class_key[96];      /* plan DB key the winner is filed under */
    int32_t resumed;         /* points taken from the journal, not timed again */
} spk_tune_report;

/* The tuning loop of Section 2: for every variant of the (pruned) space run
 * the problem, compare its output with the reference (per row
 * |out - ref| <= tau*scale; NaN/Inf positions must match; WAXPY/AXPY within
 * one ulp), discard it on mismatch, otherwise time it (median of reps,
 * HIP events) and keep the fastest.  Work buffers y/w/d_result are
 * overwritten.  Synchronises the handle's internal stream. */
spk_status spk_tune(spk_handle h, const spk_problem *problem, const spk_tune_opts *opts,
                    spk_tune_report *report);

/* Shape class a problem is filed under in the plan DB (for inspection):
 * where Section 2's selected variant is kept. */
spk_status spk_class_key(spk_handle h, const spk_problem *problem, char *out, int32_t cap);

/* Looks up / stores a plan DB entry directly (the record of Section 2's
 * selected variant for a class). */
spk_status spk_plan_get(spk_handle h, const char *class_key, spk_variant *out);
spk_status spk_plan_put(spk_handle h, const char *class_key, const spk_variant *v);

/* Section 2's search applied to the solve.  The knob is the SpMV+dot
 * kernel: a CSR wavefront-tile shape (threads per workgroup and row-stream
 * entries per wavefront, reported as an SPK_FMT_ADAPTIVE variant with
 * `block` and `lds`; `vec` 2 = the tiles read two-byte columns, as the
 * SpMV row-block kernel with vec 2), which sets the number of partial sums every workgroup
 * of the residual kernel adds, so the solve's best shape can differ from a
 * lone SpMV's; or, when A is a grid stencil (spk_matrix_formats), the
 * matrix-free kernel (SPK_FMT_STENCIL, `block` threads, `unroll` rows per
 * lane, `lds` 1 = p staged through LDS).  opts->formats
 * limits the search (bits 1 << SPK_FMT_ADAPTIVE, 1 << SPK_FMT_STENCIL; 0 =
 * all that apply).  Every candidate runs `iters` iterations
 * from x = 0 on b (device, n doubles); its r.r history and x must match
 * the default shape's run within tau (relative per entry of the history,
 * relative to max |x| for x; opts->tau, 0 -> 1e-10) or it is discarded
 * before it is timed (median of opts->reps solves after opts->warmup).
 * The winner is filed under "cg:" + the SpMV class key of A (spk_class_key)
 * and used by later spk_cg calls on that class.  On matrices whose CG
 * trajectories separate quickly in rounding (an isolated extreme
 * eigenvalue) keep iters small.  Synchronises the handle's internal
 * stream; opts may be NULL. */
spk_status spk_cg_tune(spk_handle h, spk_matrix A, const void *b, int32_t iters, const spk_tune_opts *opts,
                       spk_tune_report *report);

/* ------------------------------------------------------------- batching -- */

/* Batched execution is not in the paper: it is the configured batched
 * workload, thousands of independent instances of Section 3's sparse
 * product followed by Figure 1's update, run as one launch.
 * Many independent square CSR instances stored back to back (instance i:
 * row_ptr[rp_off[i] .. rp_off[i]+m[i]] with values local to the instance,
 * entries col_idx/val[nz_off[i] .. nz_off[i]+nnz[i]) with local column
 * indices, vectors x/y/w[vec_off[i] .. vec_off[i]+m[i])).  Size and offset
 * arrays are host memory; row_ptr, col_idx and val are device memory;
 * row_ptr_host (nullable) is a host copy of row_ptr used for planning. */
typedef struct {
    int64_t count;
    int32_t dtype;
    const int64_t *m, *nnz, *rp_off, *nz_off, *vec_off;   /* host */
    const int32_t *row_ptr, *col_idx;                       /* device */
    const void *val;                                        /* device */
    const int32_t *row_ptr_host;                            /* host, nullable */
} spk_batch_desc;

typedef struct {
    int32_t persistent;      /* launch kind: 1 (default) one persistent launch
                              * pulling tiles from per-XCD queues; 0 one
                              * workgroup per group of wavefront tiles; other
                              * values are rejected (SPK_ERR_ARG) */
    int32_t use_graph;       /* 1 (default): replay a captured hipGraph */
    int32_t block;           /* threads per workgroup; 0 -> the launch shape
                              * spk_batch_tune recorded for the dtype
                              * (workgroup size, LDS tile and launch kind,
                              * which then replaces `persistent`), else 256
                              * threads with 2048-entry tiles */
    int32_t tile_nnz;        /* target entries per tile of the lane-group
                              * modes (0 -> 1024) */
    int32_t waves_per_cu;    /* persistent residency (0 -> from occupancy) */
    int32_t x_window;        /* LDS room for x per wavefront (entries; 0 or 256)
                              * of the kernel used with an explicit block; a
                              * kernel with room runs the tiles of classes
                              * tuned to mode 1 (or 3) with the tile's window
                              * of x staged in LDS (block 0 takes the
                              * recorded value) */
} spk_batch_opts;

/* Plans the batch (not in the paper; the configured batched workload):
 * instances -> shape classes -> tiles, each class served by
 * the variant recorded for it (see spk_batch_tune), tiles ordered largest
 * first.  The descriptor arrays are copied; the device arrays are borrowed
 * for the batch's lifetime.  Classes planned with compact columns (mode 3)
 * read a one-byte copy of their column indices (each entry's place in its
 * tile's window of x; two bytes, the offset from the tile's first column,
 * for tiles whose window is wider than the kernel's room for x) that the
 * plan makes from col_idx and owns: col_idx must not change while the plan
 * lives.  Each instance's row_ptr is checked (starts at
 * 0, never decreases, ends at nnz: SPK_ERR_CSR otherwise); column indices
 * are not (as in spk_spmv_csr, one outside [0, m_i) reads outside the
 * instance's x).  A batch runs as one launch of at most 2^24
 * wavefront tiles (a dispatch counts its work-items in 32 bits); one that
 * needs more is rejected with SPK_ERR_SHAPE and should be split. */
spk_status spk_batch_plan(spk_handle h, const spk_batch_desc *desc, const spk_batch_opts *opts,
                          spk_batch *out);

/* One step over every instance: Section 3's sparse product y = A_i*x_i,
 * then Figure 1's update w = alpha*y + x (w may be NULL for SpMV only), all
 * instances in one launch.  With use_graph the launch is
 * captured once per (stream, x, y, w, alpha) and replayed.  The batch keeps
 * its persistent queue counters and its captured graph per stream, so runs
 * on different streams (with distinct y / w) may overlap; the first run on a
 * stream allocates that stream's counters and synchronises, so a caller
 * capturing runs into its own graph makes one eager run on the capture
 * stream first.  Calls on one batch from several host threads are
 * serialised by the library only for that per-stream state: runs that share
 * y or w race as any two writers do. */
spk_status spk_batch_run(spk_handle h, spk_batch b, double alpha, const void *x, void *y, void *w,
                         spk_stream stream);

/* Tunes the batch (Section 2's search): the launch shape (workgroup size,
 * LDS tile per workgroup, room for x in LDS, grid or persistent kind) on
 * the whole batch, then the tile kernel of each shape class under it (LDS
 * row stream, the same with the tile's x window staged in LDS when the
 * kernel has room for it, the same again with compact columns -- one byte
 * per entry, its offset in the window, instead of four, or two bytes for
 * tiles whose window is wider than the room: a storage-format choice of
 * the tuner, not a knob the paper lists -- or G lanes per row),
 * then the launch shape again
 * with the tuned kernels.  Every candidate is validated before it is timed
 * against the unannotated program's output: the plain kernel (one lane per
 * row, fused with the update when w is given) run instance by instance,
 * per row within tau * sum_k |a_ik x_k| (tau from opts, else 1e-12 FP64 /
 * 1e-5 FP32), w within |alpha| times that plus two rounding units.
 * opts->ref_host (nullable, host, FP64, one entry per vector element up to
 * the last instance's end) replaces the plain kernels' y as the reference;
 * when no candidate matches the reference the call fails with
 * SPK_ERR_VALIDATION.  Re-plans the tiles.  With
 * opts->record the winners go to the plan DB: one plan per class
 * ("batch:<dtype>:c<class>") and the launch shape ("batch:<dtype>:launch":
 * block, lds = LDS tile entries per workgroup, unroll = LDS room for x per
 * wavefront, grid = 1 for the persistent kind), which later plans with
 * block 0 take. */
spk_status spk_batch_tune(spk_handle h, spk_batch b, double alpha, const void *x, void *y, void *w,
                          const spk_tune_opts *opts, spk_tune_report *report);

/* Number of tiles and classes and the algorithmic bytes of one step.
 * Library plumbing, not in the paper. */
spk_status spk_batch_info(spk_handle h, spk_batch b, int64_t *tiles, int32_t *classes,
                          int64_t *bytes);

/* Tiles and matrix entries per kernel mode as planned on the device (after
 * the x windows are found, so a mode-3 tile whose window did not fit counts
 * as mode 5 or 1): tiles[mode] and entries[mode] for mode 0..64 (host
 * arrays of 65; entries nullable; 0 = LDS row stream, 1 = with the tile's
 * window of x in LDS, 3 = the same with one-byte compact columns, 5 = the
 * row stream with two-byte compact columns and x from memory, G = G lanes
 * per row).
 * Synchronises with the device.  Library plumbing, not in the paper. */
spk_status spk_batch_tile_modes(spk_handle h, spk_batch b, int64_t *tiles, int64_t *entries);

/* The launch configuration the batch currently uses (after planning or
 * tuning, Section 3's threads per block and blocks per grid): persistence,
 * graph use and workgroup size; here tile_nnz is the kernel's LDS tile in
 * entries per workgroup and waves_per_cu the persistent kind's residency. */
spk_status spk_batch_config(spk_handle h, spk_batch b, spk_batch_opts *out);

/* Frees a batch plan (its tiles, counters and captured graphs).  Library
 * plumbing, not in the paper. */
spk_status spk_batch_free(spk_handle h, spk_batch b);

/* -------------------------------------------------------------- serving -- */

/* Serving is not in the paper: it is the configured serving workload,
 * requests for one Krylov-style step (Section 3's sparse product, then
 * Figure 1's update) arriving over time and batched continuously. */
typedef struct {
    int32_t streams;          /* device streams used concurrently (0 -> 4) */
    int32_t max_inflight;     /* request slots (0 -> 256) */
    int32_t max_batch;        /* requests per launch (0 -> 64) */
    int32_t mode;             /* 0 = continuous batching; 1 = FIFO, one request per
                               * launch with the plain kernels (baseline) */
    int64_t hbm_budget;       /* bytes for resident matrices + in-flight vectors
                               * (0 -> 200 GB), counted at their exact sizes;
                               * the device blocks behind them are pooled by
                               * power-of-two size, and the pool keeps idle
                               * blocks up to a quarter of the budget for
                               * later uploads */
    double alpha;             /* step coefficient (w = alpha*y + x) */
    int32_t max_launches;     /* launches in flight (0 -> one per stream): while
                               * they run, arrivals queue and are admitted
                               * together into the next launch */
    int32_t reserved;         /* 0 */
} spk_serve_opts;

typedef struct {
    int64_t submitted, completed, rejected;
    int64_t batches;          /* launches issued */
    int64_t uploads, evictions;
    int64_t resident_bytes, peak_bytes;
    double p50_us, p99_us, mean_us, max_us;   /* arrival -> result on host */
    double wall_s;            /* first arrival -> last completion */
    double bytes_moved;       /* algorithmic bytes of completed requests */
    /* where the scheduler thread's time goes, summed over launches: */
    double stage_in_s;        /* copying requests' x into pinned staging */
    double stage_out_s;       /* copying results out of pinned staging */
    double device_s;          /* from a launch's first enqueued copy until its
                               * completion is seen (stream queueing, copies
                               * over the host link, kernel) */
    int64_t direct;           /* requests whose vectors skipped the staging
                               * copies (pinned caller buffers) */
} spk_serve_stats;

/* Starts a serving loop (not in the paper; the configured serving
 * workload) on the handle's device: a scheduler thread, which
 * owns the GPU side, and three threads that share its host copies between
 * the callers' buffers and pinned staging memory.  spk_serve_destroy joins
 * them all.  The server keeps a small record of every request submitted
 * (arrival and completion times, under 64 bytes) for spk_serve_stats_get and
 * spk_serve_latencies until it is destroyed. */
spk_status spk_serve_create(spk_handle h, const spk_serve_opts *opts, spk_server *out);

/* Adds a matrix to the server's pool (the operand of Section 3's sparse
 * product, kept resident while the budget allows).  A's arrays are host
 * memory and are
 * copied; the matrix is uploaded (made resident) when a request needs it
 * and evicted, least recently used first, only while idle.  SPK_ERR_SHAPE
 * for a non-square matrix, nnz >= 2^31, nrows >= 2^30 or more than 2^24
 * wavefront tiles (the most one launch takes; a launch's requests together
 * stay within it). */
spk_status spk_serve_add_matrix(spk_server s, const spk_csr *A, int32_t *id);

/* Submits one request: y = A_id*x (Section 3's product), w = alpha*y + x
 * (Figure 1's update).  x is host memory of
 * ncols elements (copied at admission); y and w are host memory of nrows
 * elements filled in before the request is reported complete.  The buffers
 * stay borrowed until then.  *req receives the request id.  Vectors of
 * 128 KiB or more whose three buffers (two without w) are each inside one
 * pinned host allocation (hipHostMalloc) move between those buffers and the
 * device by the copy engines, without the server's staging copies. */
spk_status spk_serve_submit(spk_server s, int32_t mat_id, const void *x, void *y, void *w,
                            int64_t *req);

/* Completed request ids since the last poll (up to cap).  Serving plumbing,
 * not in the paper. */
spk_status spk_serve_poll(spk_server s, int64_t *ids, int32_t cap, int32_t *n);

/* Blocks until every submitted request has completed.  Serving plumbing,
 * not in the paper. */
spk_status spk_serve_drain(spk_server s);

/* Open-loop replay (measurement of the configured serving workload, not in
 * the paper): submits request i at arrival_s[i] seconds after the call (by
 * the library's own clock) and returns when all have completed. */
spk_status spk_serve_replay(spk_server s, int64_t n, const double *arrival_s, const int32_t *mat_ids,
                            const void *const *x, void *const *y, void *const *w);

/* Counters and latency percentiles of the server so far.  Measurement, not
 * in the paper. */
spk_status spk_serve_stats_get(spk_server s, spk_serve_stats *out);

/* Per-request latency in microseconds, by request id (cap entries).
 * Measurement, not in the paper. */
spk_status spk_serve_latencies(spk_server s, double *out_us, int64_t cap, int64_t *n);

/* Each request's latency split at its admission, by request id (cap
 * entries): wait_us = from its arrival until the scheduler admitted it to a
 * launch (queueing, including waits for memory), run_us = from admission
 * until its results were in the caller's buffers (copies, launch, kernel).
 * -1 for requests not finished.  Measurement, not in the paper. */
spk_status spk_serve_latency_split(spk_server s, double *wait_us, double *run_us, int64_t cap, int64_t *n);

/* Drains and stops the server, joins its threads and frees its device
 * memory.  Serving plumbing, not in the paper. */
spk_status spk_serve_destroy(spk_server s);

/* --------------------------------------------------------- measurement -- */

/* Measurement, not in the paper.  STREAM-style probes on device arrays of
 * n doubles: kind 0 = copy
 * (c = a; b unused), 1 = triad (c = a + 3*b).  Used for the measured
 * bandwidth roofline and to calibrate byte counters. */
spk_status spk_stream_probe(spk_handle h, int32_t kind, int64_t n, const double *a, const double *b,
                            double *c, spk_stream stream);

/* Measurement, not in the paper.  Reads a library-owned 512 MiB buffer
 * (twice the last-level cache) so the
 * next kernel starts with cold caches holding only clean lines: it pays for
 * its own misses and not for writing back someone else's dirty lines. */
spk_status spk_flush_cache(spk_handle h, spk_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* SPK_H */
