/*
 * fespmv -- FP64 sparse matrix-vector products and conjugate-gradient solves
 * for matrices assembled from unstructured finite element meshes, on AMD
 * Instinct MI355X (gfx950).
 *
 * The operation is y = A x for a sparse A given in CSR form (paper: section
 * "Description of Current GPU Methods", statement of the SpMV problem), and
 * the Jacobi-preconditioned conjugate-gradient solve of A x = b built around
 * it (paper: sections "Computational Cost of the Finite Element Method" and
 * "Description of Current GPU Methods": the solver performs at least one
 * SpMV per iteration).  The matrix is re-packed once into a row-grouped,
 * column-interleaved layout (paper: section "Development of Novel GPU
 * Algorithms"; the pattern is fixed and only values change between Newton
 * steps, section "Cost of Reordering Matrix Values").
 *
 * Conventions for every entry point:
 *  - Every call returns an fs_status (int32_t).  FS_OK is 0.  The library
 *    never aborts and never throws across this interface; fs_last_error()
 *    returns a thread-local description of the last non-OK status.
 *  - Vector and CSR array pointers are DEVICE pointers on the device that
 *    is current when the call is made (the device the handle was created
 *    on).  They stay owned by the caller; the library never frees them and
 *    keeps no reference to them after the call (blocking calls) or after
 *    the stream reaches the call (asynchronous calls).
 *  - Indices are 0-based int32.  nnz must be below 2^31.
 *  - Asynchronous calls are ordered on the given stream (0 = the null
 *    stream).  A device fault raised by an asynchronous call is reported as
 *    FS_E_HIP by the next call that synchronises.
 *  - One handle must not be used from two streams at the same time;
 *    different handles are independent.
 */
#ifndef FESPMV_H
#define FESPMV_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef int32_t fs_status;
enum {
    FS_OK = 0,
    FS_E_ARG = 1,            /* NULL pointer, negative size, k out of range  */
    FS_E_BAD_CSR = 2,        /* malformed row pointer, column out of range,
                                duplicate column in a row                   */
    FS_E_NOT_SQUARE = 3,     /* operation needs a square matrix             */
    FS_E_OOM = 4,            /* device or host allocation failed            */
    FS_E_BUDGET = 5,         /* request exceeds the configured memory budget */
    FS_E_HIP = 6,            /* HIP runtime error (message has the details) */
    FS_E_NOT_CONVERGED = 7,  /* maxit reached; x holds the last iterate     */
    FS_E_BREAKDOWN = 8,      /* p^T A p <= 0 or a non-finite CG scalar      */
    FS_E_UNSUPPORTED = 9     /* option combination not implemented          */
};

/* Thread-local message for the last non-OK status returned on this thread
 * (empty string if none).  The pointer stays valid until the next call on
 * the same thread. */
const char *fs_last_error(void);

/* ----------------------------------------------------------- the matrix */
typedef struct fs_csr *fs_csr_t;

enum {  /* fs_csr_opts.reorder */
    FS_REORDER_AUTO = 0,  /* reverse Cuthill-McKee when it shortens the mean
                             |i - j| of the non-zeros, else none           */
    FS_REORDER_NONE = 1,  /* keep the caller's numbering (rows may still be
                             sorted by length inside sort windows)         */
    FS_REORDER_RCM = 2,   /* reverse Cuthill-McKee on the pattern of A+A^T */
    FS_REORDER_USER = 3   /* use opts.perm                                 */
};

enum {  /* fs_csr_opts.build: where the per-non-zero phases of the layout
           build run (validation of the columns, slot assignment, CSR ->
           slot map, 16-bit offsets, bandwidth statistics).  The row order
           and the row groups are computed on the host either way (they
           need the row lengths, or the graph for reverse Cuthill-McKee).
           Both builders produce the same layout, bit for bit.  (Paper:
           section "Cost of Reordering Matrix Values" -- the value map comes
           from one scan of the pattern, done here by either builder.) */
    FS_BUILD_DEVICE = 0,  /* device kernels (default); the host build runs
                             instead when a row has more than
                             FS_BUILD_DEVICE_MAX_ROW entries or autotune is
                             set (fs_csr_stats.build tells which ran)      */
    FS_BUILD_HOST = 1     /* multi-threaded host build                     */
};
#define FS_BUILD_DEVICE_MAX_ROW 4096

enum {  /* bit mask, fs_csr_opts.dtypes and csr_add_dtype() */
    FS_DT_F64 = 1,
    FS_DT_F32 = 2,        /* FP32 copy of the values, rounded to nearest  */
    FS_DT_BF16 = 4        /* BF16 copy: FP64 -> FP32 -> BF16, each to
                             nearest, ties to even                         */
};

typedef struct fs_csr_opts {
    int32_t reorder;       /* FS_REORDER_*                                   */
    const int32_t *perm;   /* HOST array of n_rows entries for
                              FS_REORDER_USER: new row i is old row perm[i] */
    int32_t sort_window;   /* rows are ordered longest-first (stable) inside
                              consecutive windows of this many rows, after
                              the reordering; 1 disables; 0 = auto: the
                              narrowest of 256, 1024, 4096, 16384 whose
                              padded slot count is within 2% of the fewest */
    int32_t threshold;     /* most slots one lane may own before the row is
                              spread over more lanes; 0 = default 48       */
    int32_t lanes_min;     /* lanes per row bounds, powers of two in 1..64; */
    int32_t lanes_max;     /*   0 = defaults 1 and 64                       */
    int32_t dtypes;        /* extra low-precision copies (FS_DT_F32/BF16)   */
    int32_t vec;           /* slots each lane loads at once: 1 or 2; 0 =
                              auto (2 unless it adds > 6% padded slots)    */
    int32_t index_bits;    /* column indices in the slot stream: 0 = auto
                              (16-bit offsets from a per-group base when
                              every row group's columns span fewer than
                              65535, else 32-bit); 32 = always 32-bit      */
    int32_t autotune;      /* 1: time the product for several lanes-per-row
                              and slots-per-load shapes on this matrix and
                              keep the fastest (results cached per matrix
                              signature for the process); lanes_min/max and
                              vec are then ignored                          */
    int32_t build;         /* FS_BUILD_DEVICE (0) or FS_BUILD_HOST (autotune
                              always builds on the host)                   */
    int32_t reserved[4];   /* must be zero                                   */
} fs_csr_opts;

/* Fill *o with the defaults (AUTO reorder, window 256, threshold 48,
 * lanes 1..64, FP64 only). */
fs_status csr_opts_default(fs_csr_opts *o);

/* Build the layout of an n_rows x n_cols CSR matrix.  rowptr (n_rows+1),
 * colind (nnz) and vals (nnz) are device arrays; columns may be unsorted
 * inside a row but must be unique and in [0, n_cols).  opts may be NULL
 * (defaults).  The call reads the structure on the host, builds the row
 * permutation and row groups, assigns the slots and the slot map (on the
 * device by default, on the host with opts->build = FS_BUILD_HOST), and
 * scatters the values on the device.
 * It synchronises stream s before returning, after which the caller may
 * free or reuse its arrays.  *out receives the handle.
 * Errors: FS_E_ARG, FS_E_BAD_CSR, FS_E_OOM, FS_E_HIP, FS_E_UNSUPPORTED. */
fs_status csr_create(int32_t n_rows, int32_t n_cols, int64_t nnz,
                     const int32_t *rowptr, const int32_t *colind,
                     const double *vals, const fs_csr_opts *opts,
                     hipStream_t s, fs_csr_t *out);

/* New values for the same pattern (vals in the CSR order that csr_create
 * saw), refreshing any low-precision copies: the per-Newton-step value
 * reorder of section "Cost of Reordering Matrix Values".  One device pass
 * in slot order; each slot reads its entry at its row's CSR start plus a
 * byte-wide position within the row (kept from creation, 1 byte per slot
 * and 5 per row, when no row holds more than 255 entries), else through a
 * 4-byte slot-to-CSR map.  vals is a device array of nnz doubles the
 * library only reads.  Asynchronous on s.
 * Errors: FS_E_ARG (NULL handle or values), FS_E_HIP. */
fs_status csr_update_values(fs_csr_t A, const double *vals, hipStream_t s);

/* Materialise a low-precision copy (FS_DT_F32 or FS_DT_BF16) of the values
 * for mixed-precision solves.  Not in the paper, which stores and computes
 * in FP64 throughout (section "Description of the Physical Problem"): this
 * is the storage half of the mixed-precision addition (values rounded to
 * nearest into FP32; BF16 rounded nearest-even from that FP32 value).
 * Synchronises s. */
fs_status csr_add_dtype(fs_csr_t A, int32_t dtype, hipStream_t s);

typedef struct fs_csr_stats {
    int32_t n_rows, n_cols;
    int64_t nnz;
    int64_t slots;            /* padded slots, >= nnz                       */
    int32_t n_groups;         /* row groups (one wavefront each)            */
    int32_t reorder;          /* reordering actually applied (FS_REORDER_*) */
    double padding;           /* (slots - nnz) / slots                      */
    int64_t bytes_algorithmic;/* 12 nnz + 8 n_cols + 8 n_rows: compulsory
                                 traffic of one FP64 product                */
    int64_t bytes_layout;     /* (8 + index bytes) slots + (16 or 20)
                                 n_groups + 8 n_cols + 8 n_rows              */
    int32_t groups_by_lanes[7];/* groups with 1,2,4,...,64 lanes per row    */
    int32_t dtypes;           /* FS_DT_* copies held                        */
    int32_t vec;              /* slots per lane per load (1 or 2)           */
    double mean_band_before;  /* mean |i - j| over non-zeros, input order  */
    double mean_band_after;   /* same, layout order                         */
    double t_build_ms;        /* wall time of csr_create                    */
    int64_t device_bytes;     /* device memory held by the handle          */
    int32_t tuned;            /* 0 no, 1 tuned now, 2 from the tuning cache */
    int32_t tune_candidates;  /* layouts timed                              */
    double tune_best_us;      /* product time of the kept layout            */
    int32_t index_bits;       /* 16 or 32: column index width in the slots  */
    int32_t build;            /* FS_BUILD_DEVICE / FS_BUILD_HOST: the
                                 builder that ran                            */
} fs_csr_stats;

fs_status csr_info(fs_csr_t A, fs_csr_stats *st);

/* Copy the layout's row permutation to a HOST array of n_rows entries:
 * layout row i is row perm[i] of the caller's matrix. */
fs_status csr_get_perm(fs_csr_t A, int32_t *perm_host);

/* Copy the handle's layout (the row-grouped, column-interleaved storage of
 * sections "ELL-WARP", "ELL-WARP v2 (K2)" and "K1rs") to HOST arrays (each
 * may be NULL; sizes from csr_info): groups (4 int32 per group, as csr_layout_host), slot_col
 * (layout column of every slot, -1 = padding), map (slot of every CSR
 * position), and, when index_bits is 16, col16 (column minus the group's
 * base column, 0xffff = padding) and gbase (base column of every group).
 * Synchronous.  FS_E_ARG when col16 / gbase are asked for a 32-bit layout. */
fs_status csr_get_layout(fs_csr_t A, int32_t *groups, int32_t *slot_col,
                         int32_t *map, uint16_t *col16, int32_t *gbase);

/* Host-only dry run of the layout builder on HOST arrays (no device memory
 * is touched, no GPU needed): the same validation, reordering, grouping and
 * slot assignment csr_create performs.  Outputs (each may be NULL):
 * n_groups, slots, vec (slots per lane per load); groups: 4 int32 per
 * group {first element / 64, first layout row, rows, slots per lane |
 * log2(lanes per row) << 24}; slot_col:
 * layout column of every slot (-1 = padding); map: slot of every CSR
 * position; perm: layout row i is caller row perm[i].  Call once with NULL
 * arrays to learn the sizes. */
fs_status csr_layout_host(int32_t n_rows, int32_t n_cols, int64_t nnz,
                          const int32_t *rowptr, const int32_t *colind,
                          const fs_csr_opts *opts, int32_t *n_groups,
                          int64_t *slots, int32_t *vec, int32_t *groups,
                          int32_t *slot_col, int32_t *map, int32_t *perm);

/* Free everything the handle owns (after synchronising the device).  NULL
 * is a no-op. */
fs_status csr_destroy(fs_csr_t A);

/* --------------------------------------------------------------- products */
/* y = A x in the caller's numbering (x has n_cols, y n_rows entries).  x and
 * y must not alias.  Asynchronous on s. */
fs_status spmv(fs_csr_t A, const double *x, double *y, hipStream_t s);

/* y' = A' x' in the layout numbering, A' = P A P^T (square matrices only):
 * x'(i) = x(perm[i]) and y'(i) = y(perm[i]) (paper: section "ELL-WARP with
 * row reordering (K1r)" -- an iterative solver keeps its vectors in this
 * numbering and never pays the final re-mapping).  Asynchronous on s. */
fs_status spmv_perm(fs_csr_t A, const double *xp, double *yp, hipStream_t s);

/* y = A x straight from CSR device arrays (rowptr n_rows + 1, colind and
 * vals nnz entries), without building a layout: T lanes per row stride over
 * the row's entries (T = the largest power of two not above half the mean
 * row length, at most 64) and are reduced by shuffles.  The product for a
 * matrix used once, and the reference for the layout build's break-even
 * count (section "Cost of Reordering Matrix Values": reordering pays off
 * after enough products).  No validation pass: a malformed CSR gives wrong
 * values but no out-of-bounds access (row bounds and columns are clamped).
 * x and y must not alias.  Asynchronous on s. */
fs_status spmv_csr(int32_t n_rows, int32_t n_cols, int64_t nnz,
                   const int32_t *rowptr, const int32_t *colind,
                   const double *vals, const double *x, double *y,
                   hipStream_t s);

/* Measurement aid, not part of the method: stream n doubles of buf (device,
 * 16-byte aligned; an odd last element is skipped) with `blocks`
 * workgroups of 256 threads, writing one partial sum per block to
 * sink[0 .. blocks-1] (device).  Timing it gives the achievable streaming
 * read rate of the device, the practical ceiling for the products above.
 * Asynchronous on s; FS_E_ARG on bad sizes or alignment. */
fs_status probe_read_bandwidth(const double *buf, int64_t n, double *sink,
                               int32_t blocks, hipStream_t s);

/* m independent products y_i = A_i x_i in the caller's numbering, the
 * batch form of spmv (same statement of the problem; each result is bitwise
 * the spmv result).  Not in the paper: the batching addition, for many
 * small systems whose products alone are launch-latency bound.  A, x and y are HOST arrays of m entries holding handles
 * and DEVICE vector pointers; all handles live on one device.  The y_i are
 * distinct and no x_i is any y_j; a handle may appear more than once.  The products of
 * up to 56 matrices share each launch (per-matrix descriptors are passed as
 * kernel arguments: nothing is allocated or copied to the device), so many
 * small matrices cost one launch latency instead of m.  m = 0 is a no-op.
 * Asynchronous on s; errors: FS_E_ARG (NULL entries, aliasing, mixed
 * devices), FS_E_HIP. */
fs_status spmv_batch(int32_t m, const fs_csr_t *A, const double *const *x,
                     double *const *y, hipStream_t s);

enum { FS_TO_LAYOUT = 0, FS_FROM_LAYOUT = 1 };
/* out(i) = in(perm[i]) (FS_TO_LAYOUT) or out(perm[i]) = in(i)
 * (FS_FROM_LAYOUT); n_rows entries; in and out must not alias. */
fs_status csr_permute(fs_csr_t A, int32_t dir, const double *in, double *out,
                      hipStream_t s);

/* Y = A X for k right-hand sides, 1 <= k <= 16.  X is n_cols x k and Y is
 * n_rows x k, row-major with row strides ldx >= k and ldy >= k (elements).
 * Not in the paper: the multi-right-hand-side part of the batching
 * addition; each column is the product of section "Description of Current
 * GPU Methods", and the matrix stream is read once for all k columns.
 * Asynchronous on s. */
fs_status spmm(fs_csr_t A, int32_t k, const double *X, int64_t ldx,
               double *Y, int64_t ldy, hipStream_t s);

/* Low-precision product in the layout numbering: y' = A'_lo x' with the FP32
 * or BF16 copy of the values (csr_add_dtype first), float x' and y', float
 * accumulation.  Not in the paper (FP64 only, section "Description of the
 * Physical Problem"): the inner operation of the mixed-precision refinement
 * addition; BF16 values are widened to float exactly.  Square matrices
 * only.  Asynchronous on s. */
fs_status spmv_lowp(fs_csr_t A, int32_t dtype, const float *xp, float *yp,
                    hipStream_t s);

/* --------------------------------------------------------------- solvers */
enum { FS_PC_NONE = 0, FS_PC_JACOBI = 1 };
enum { FS_PREC_F64 = 0, FS_PREC_IR_F32 = 1, FS_PREC_IR_BF16 = 2 };

typedef struct fs_cg_opts {
    double rtol;          /* stop when |b - A x|_2 <= rtol |b|_2 (true
                             residual, checked in FP64); default 1e-8      */
    int32_t maxit;        /* iteration limit (inner iterations for IR);
                             0 = default 20000                              */
    int32_t precond;      /* FS_PC_*; default JACOBI                         */
    int32_t precision;    /* FS_PREC_*; default F64                          */
    double inner_rtol;    /* IR: inner solve tolerance; 0 = default 1e-2    */
    int32_t check_every;  /* iterations between host convergence checks
                             (one captured graph); 0 = default 32           */
    int32_t x0_zero;      /* 1: start from x = 0 and ignore x on input      */
    int32_t use_graph;    /* 1: replay chunks as HIP graphs (default 1)    */
    int32_t max_outer;    /* IR: refinement steps; 0 = default 50           */
    int32_t ir_restart;   /* IR: 0 (default) keeps the inner search
                             direction from step to step (the FP64
                             residual replaces the inner one); 1 restarts
                             the inner CG from zero at every step           */
    int32_t ir_scaled;    /* IR: 1 stores the low-precision copy after
                             Jacobi scaling, round(D^-1/2 A D^-1/2) with
                             D = diag(A) (all diagonal entries must be
                             positive); the inner CG then solves the
                             scaled system with M = I, on the right-hand
                             side D^-1/2 r, and the FP64 update is
                             x += D^-1/2 d.  0 (default): round(A)         */
    int32_t estimate_cond;/* FP64, one right-hand side: 1 records the CG
                             coefficients alpha_j, beta_j and returns in
                             info->cond_est the ratio of the extreme
                             eigenvalues of their Lanczos tridiagonal, an
                             estimate of the condition number of M^-1 A   */
    int32_t wg_threads;   /* cg_solve_batch_wg: threads per workgroup, 256,
                             512 or 1024; 0 = the fastest of the three, each
                             with the Krylov vectors in LDS where they fit
                             and with z = D^-1 r alone there (more
                             workgroups per compute unit), timed on the
                             first call for a batch shape and remembered
                             for the process (the results do not depend on
                             the choice)                                    */
    int32_t reserved[2];  /* must be zero                                    */
} fs_cg_opts;

fs_status cg_opts_default(fs_cg_opts *o);

typedef struct fs_cg_info {
    int32_t status;       /* same value the call returned                   */
    int32_t iters;        /* CG iterations (F64) / inner iterations (IR)    */
    int32_t outer;        /* IR refinement steps (0 for F64)                */
    int32_t replacements; /* residual replacements performed               */
    double relres;        /* true relative residual |b - A x| / |b| (FP64) */
    double ms;            /* wall time of the call                          */
    double bytes;         /* algorithmic HBM bytes moved by the solve       */
    double cond_est;      /* with opts->estimate_cond (FP64, one column):
                             lambda_max / lambda_min of the Lanczos
                             tridiagonal T of the CG coefficients,
                             T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
                             T_j,j+1 = sqrt(beta_j)/alpha_j (Saad, Iterative
                             Methods for Sparse Linear Systems, sec. 6.7.3);
                             0 when not asked for                           */
} fs_cg_info;

/* Solve A x = b (A square, symmetric positive definite).  b and x are
 * device vectors in the caller's numbering; x holds the initial guess on
 * entry (unless opts->x0_zero) and the solution on return.  Blocking: the
 * call synchronises stream s.  opts NULL = defaults; info may be NULL.
 * Returns FS_OK when the true residual meets rtol, FS_E_NOT_CONVERGED
 * (x = last iterate), FS_E_BREAKDOWN, or an argument/runtime error.
 * Mixed precision (opts->precision IR_F32 / IR_BF16): a refinement step
 * that does not reduce the FP64 residual is undone and the solve stops,
 * with FS_E_BREAKDOWN if the inner solve on the low-precision copy broke
 * down (that copy need not be positive definite when rounding error times
 * the condition number exceeds 1), else FS_E_NOT_CONVERGED. */
fs_status cg_solve(fs_csr_t A, const double *b, double *x,
                   const fs_cg_opts *opts, fs_cg_info *info, hipStream_t s);

/* Stream-ordered form of cg_solve (FP64, one right-hand side): the call
 * only enqueues work on s and returns.  The solver is the Jacobi-PCG of
 * sections "Computational Cost of the Finite Element Method" and
 * "Description of Current GPU Methods"; the stream form is an addition (the
 * paper drives its solver from the host).  The whole solve -- Jacobi scaling,
 * start residual, every iteration, true-residual confirmation with residual
 * replacement -- is one cooperative launch that holds its scalars on the
 * device (no host round trip per chunk), between the permutation of b in
 * and of x out.  The iteration and the stopping rule are those of cg_solve;
 * sums are ordered differently, so x and the iteration count agree with
 * cg_solve up to rounding.  Work that follows on s sees the solution in x.
 * info is HOST memory that receives the result (status, iters,
 * replacements, relres, ms = device time of the solve kernel, bytes) by an
 * asynchronous copy when s reaches the end of the solve; with pinned memory
 * (hipHostMalloc) the call returns at once, pageable memory makes that copy
 * synchronous.  opts->precision must be FP64 (else FS_E_UNSUPPORTED);
 * use_graph and check_every are ignored.  Uses per-handle workspace (7 n
 * doubles, allocated on the first call): calls on one handle must be
 * ordered on one stream.  Returns FS_OK once enqueued, or FS_E_ARG,
 * FS_E_NOT_SQUARE, FS_E_UNSUPPORTED (no cooperative launch), FS_E_OOM,
 * FS_E_HIP; the solve's own status arrives in info->status. */
fs_status cg_solve_async(fs_csr_t A, const double *b, double *x,
                         const fs_cg_opts *opts, fs_cg_info *info,
                         hipStream_t s);

/* cg_solve_async for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same stream-ordered solve, same kernels and results
 * (bitwise those of cg_solve_async on the same arguments), but its
 * workspace -- 7 n doubles of Krylov vectors, the block partials and the
 * device result record -- is a fixed device array of the library, sized
 * for systems of up to 262,144 rows (14.7 MB, held by every GPU the
 * library runs on until the process ends).  The call allocates nothing:
 * no hipMalloc, no host or device allocation by the library.  Systems
 * above 262,144 rows return FS_E_ARG.  All calls on one GPU share that
 * array (the last call's contents stay in it): calls whose solves overlap
 * on one GPU -- on different streams, or from different threads without
 * ordering -- race and must not be made; calls ordered on one stream are
 * safe.  Arguments, info and errors as cg_solve_async. */
fs_status cg_solve_async_noalloc(fs_csr_t A, const double *b, double *x,
                                 const fs_cg_opts *opts, fs_cg_info *info,
                                 hipStream_t s);

/* k independent solves A X[:, c] = B[:, c], 1 <= k <= 16, advanced
 * together (not in the paper: the multi-right-hand-side part of the
 * batching addition; each column runs the Jacobi-PCG of section
 * "Computational Cost of the Finite Element Method"): one multi-column
 * product per iteration (the k columns of a row
 * of X are contiguous, so one gathered row serves all k).  B and X are
 * n x k row-major device blocks with row strides ldb, ldx >= k.  Columns
 * stop independently.  The order of every sum is fixed by the column-count
 * class (k rounded up to 1, 2, 4, 8 or 16): a column's iterates are bitwise
 * the same for any k of one class, and equal those of a cg_solve of the
 * column alone up to rounding.  info (may be NULL) receives k entries.
 * Blocking; returns the worst column status. */
fs_status cg_solve_multi(fs_csr_t A, int32_t k, const double *B, int64_t ldb,
                         double *X, int64_t ldx, const fs_cg_opts *opts,
                         fs_cg_info *info, hipStream_t s);

/* m independent systems A[i] X[i] = B[i] with k[i] right-hand sides each
 * (1 <= k[i] <= 16), advanced by the same launches (not in the paper: the
 * batching addition, for many small systems -- such as the small heart
 * meshes of section "Finite Element Comparison Between GPU and Multi-core"
 * -- whose solves are launch-latency bound): every iteration is one
 * batched product kernel and a fixed number of vector / reduction kernels
 * for all systems together, so many small systems cost what one does.
 * B[i] and X[i] are n_i x k[i] row-major device blocks (row stride k[i]).
 * Each system's iterates, reductions included, are bitwise those of solving
 * it alone with cg_solve_multi (systems are launched with others of the
 * same slot width and column-count class only).  FP64 only (FS_E_UNSUPPORTED otherwise).  info (may be NULL)
 * receives sum(k) entries, systems in order.  Blocking; returns the worst
 * status over all right-hand sides. */
fs_status cg_solve_batch(int32_t m, const fs_csr_t *A, const int32_t *k,
                         const double *const *B, double *const *X,
                         const fs_cg_opts *opts, fs_cg_info *info,
                         hipStream_t s);

/* m independent small systems A[i] x[i] = b[i], one right-hand side each,
 * each solved to the end by one workgroup (not in the paper: the batching
 * addition, for systems so small that cg_solve_batch is bound by its
 * per-iteration launches and host checks; the solver is the Jacobi-PCG of
 * sections "Computational Cost of the Finite Element Method" and
 * "Description of Current GPU Methods").  One launch holds every system:
 * the workgroup of system i runs its Jacobi scaling, start residual,
 * iterations and true-residual confirmation with residual replacement,
 * synchronising only within itself; the matrix stays in the L2 between
 * iterations, and the Krylov vectors stay in LDS where they fit (z, x, r, p
 * and q up to about 4,000 rows, z = D^-1 r alone up to about 19,000).  The stopping rule is cg_solve's;
 * the sums are ordered per row group and per 64-row chunk, so x and the
 * iteration counts agree with cg_solve up to rounding, and are bitwise the
 * same alone or in any batch and for every opts->wg_threads.  A handle may
 * appear several times (several right-hand sides of one matrix).  b[i] and
 * x[i] are device vectors of n_i entries in the caller's numbering; x[i]
 * holds the initial guess unless opts->x0_zero; the x[i] must not overlap
 * each other or any b[j].  Limits: each system square, at most 65,536 rows
 * and 1,024 row groups (FS_E_ARG above), FP64 only (FS_E_UNSUPPORTED
 * otherwise), all handles on one device.  Work space (7 n doubles per
 * system, plus descriptors) is kept per device between calls, grown to the
 * largest batch and held until the process ends; calls on one device run
 * one at a time (a lock is held for the call).  info (may be NULL) receives
 * m entries; ms = device time of that system's workgroup.  Blocking;
 * returns the worst status. */
fs_status cg_solve_batch_wg(int32_t m, const fs_csr_t *A,
                            const double *const *b, double *const *x,
                            const fs_cg_opts *opts, fs_cg_info *info,
                            hipStream_t s);

/* ------------------------------------------------------------- serving */
/* Not in the paper: the serving addition (continuous batching of solves
 * with admission by device memory), built on cg_solve_batch.
 * A solve server: requests (a matrix handle and k right-hand sides) are
 * admitted in arrival order while a device-memory budget and a slot count
 * allow, and every admitted request is advanced by the same batched
 * launches as the others (continuous batching: requests join and leave at
 * chunk boundaries of check_every iterations).  Each result is bitwise the
 * result of solving that request alone with cg_solve_multi and the same
 * options.  One worker thread per server does all device work on its own
 * stream; submit / poll / stats may be called from any thread. */
typedef struct fs_server *fs_server_t;

typedef struct fs_server_opts {
    int64_t hbm_budget_bytes; /* device bytes for admitted requests: their
                                 Krylov state plus the handle of every
                                 matrix in use; 0 = 16 GiB                  */
    int32_t max_slots;        /* requests in flight; 0 = 64                 */
    int32_t check_every;      /* iterations per chunk; 0 = 16               */
    int32_t precond;          /* FS_PC_*; default JACOBI                     */
    int32_t maxit;            /* 0 = 20000                                  */
    double rtol;              /* true relative residual; 0 = 1e-8          */
    int32_t use_graph;        /* replay chunks as HIP graphs (default 1)    */
    int32_t reserved[7];
} fs_server_opts;

typedef struct fs_server_done {
    uint64_t req_id;
    int32_t k;
    int32_t pad;
    fs_cg_info info;          /* worst status, max iterations and max true
                                 relative residual over the k columns;
                                 info.ms = submit-to-done latency           */
    double t_submit_ms, t_admit_ms, t_done_ms;   /* server clock (ms)       */
} fs_server_done;

typedef struct fs_server_stats {
    int32_t queued, active, peak_active, pad;
    uint64_t submitted, completed;
    int64_t bytes_in_use, peak_bytes;
} fs_server_stats;

fs_status server_opts_default(fs_server_opts *o);
fs_status server_create(const fs_server_opts *opts, fs_server_t *out);

/* Queue a request: solve A X = B for the k columns (1..16) of the n x k
 * row-major device block B (row stride k) into X (same shape).  B and X
 * stay owned by the caller and must stay valid, and A must not be
 * destroyed, until the request is returned by server_poll.  Returns at
 * once with *req_id.  FS_E_BUDGET if the request alone exceeds the budget
 * (it could never be admitted). */
fs_status server_submit(fs_server_t S, fs_csr_t A, int32_t k, const double *B,
                        double *X, uint64_t *req_id);

/* Move up to cap finished requests into done[]; *n receives the count.
 * Non-blocking. */
fs_status server_poll(fs_server_t S, fs_server_done *done, int32_t cap,
                      int32_t *n);
fs_status server_stats(fs_server_t S, fs_server_stats *st);

/* Finish every queued and running request, then free the server. */
fs_status server_destroy(fs_server_t S);

/* ------------------------------------------------------------- assembly
 * Finite-element assembly as a sum-only SpMV (paper: section "Description of
 * Current GPU Methods", the assembly of the global tangent matrix and
 * residual: one row per global non-zero whose entries are the element
 * contributions to it, multiplied by a vector of ones, so the product is a
 * plain race-free sum; section "Cost of Reordering Matrix Values" and the
 * conclusion: when assembly writes its result straight into the solver's
 * layout, the value reorder disappears).
 *
 * The element data use this layout (row-major, device memory):
 *   edof[e * nde + a]            row/column of A of local DOF a of element e,
 *                                or -1 for a DOF that is not in A (e.g.
 *                                removed by a Dirichlet condition);
 *   ke[(e * nde + a) * nde + b]  element matrix entry (a, b), FP64;
 *   re[e * nde + a]              element vector entry a, FP64.
 * Assembled entry (I, J) of K is the sum over e = 0, 1, ..., n_elem - 1 and,
 * inside an element, over (a, b) in row-major order, of ke[e][a][b] for every
 * (a, b) with edof[e][a] = I and edof[e][b] = J, added left to right from
 * 0.0 in exactly that order (so the result is bitwise reproducible and
 * equals a sequential element-by-element assembly); entries of A that no
 * element touches become 0.  R_I is the same sum of re[e][a] over
 * edof[e][a] = I. */
typedef struct fs_asm *fs_asm_t;

enum {  /* asm_create(plan): how asm_matrix finds the element values */
    FS_ASM_AUTO = 0,      /* ROWGROUP when it applies, else GATHER         */
    FS_ASM_GATHER = 1,    /* one lane per value slot, gathering its element
                             values through a stored 4-byte position list */
    FS_ASM_ROWGROUP = 2   /* one workgroup per row group of the layout,
                             summing in LDS; the nde lanes of a row read an
                             element row's nde consecutive values; needs
                             nde <= 64, no kept DOF twice in one element,
                             every row group within 6144 slots            */
};

/* Build an assembly plan for square A from the element-to-DOF map edof
 * (n_elem x nde int32, device).  Every pair of kept DOFs of an element must
 * be a structural non-zero of A (FS_E_BAD_CSR names the first element that
 * is not); entries of edof must be -1 or in [0, n_rows).  plan: FS_ASM_*;
 * both kinds give bitwise the same values.  The plan keeps a reference to
 * A: A must outlive it.  Synchronises s; the caller may free edof when the
 * call returns.  The work runs on the host (multi-threaded), once per mesh.
 * Errors: FS_E_ARG, FS_E_NOT_SQUARE, FS_E_BAD_CSR, FS_E_UNSUPPORTED
 * (n_elem * nde * nde >= 2^31, or FS_ASM_ROWGROUP where it does not apply),
 * FS_E_OOM, FS_E_HIP. */
fs_status asm_create(fs_csr_t A, int32_t n_elem, int32_t nde,
                     const int32_t *edof, int32_t plan, hipStream_t s,
                     fs_asm_t *out);

/* Host-only dry run of asm_create on HOST arrays (no device memory is
 * touched, no GPU needed): builds the layout csr_layout_host would build
 * for the square CSR pattern (rowptr, colind) and opts, then the plan for
 * the matrix (which = 0) or the vector (which = 1).  Outputs: *ntasks
 * tasks, *nwaves waves of 64 tasks, *stored index entries; waves (2 int32
 * per wave: first index row, number of index rows), tpos (ntasks: output
 * position of each task -- a layout value slot for the matrix, a row for
 * the vector -- or -1 for a filler task that completes a wave) and aidx (stored: at (waves[2w] + j) * 64 + t % 64,
 * entry j of task t's list of flat element-array indices, ascending, -1
 * after the last).  Pass NULL arrays to learn the sizes first. */
fs_status asm_plan_host(int32_t n_rows, int64_t nnz, const int32_t *rowptr,
                        const int32_t *colind, const fs_csr_opts *opts,
                        int32_t n_elem, int32_t nde, const int32_t *edof,
                        int32_t which, int64_t *ntasks, int32_t *nwaves,
                        int64_t *stored, int32_t *waves, int32_t *tpos,
                        int32_t *aidx);

/* Host-only dry run of the FS_ASM_ROWGROUP matrix plan on HOST arrays
 * (same inputs as asm_plan_host).  *built = 0 when that plan does not
 * apply.  Outputs: *ngroups row groups, *nbatch batches, *nrec records,
 * *rows rows per batch (64 / nde); gdesc (4 int32 per group: first slot /
 * 64, slots per lane, first batch, batches), bdesc (2 int32 per batch:
 * first record, steps), ea (rows int32 per record: element row e*nde + a
 * that batch row adds at that step, -1 none) and off (64 uint16 per record:
 * for lane q*nde + b, the offset from the group's first slot of the slot
 * that receives element value (ea[q]*nde + b), 0xffff none).  Pass NULL
 * arrays to learn the sizes first. */
fs_status asm_plan_host_groups(int32_t n_rows, int64_t nnz,
                               const int32_t *rowptr, const int32_t *colind,
                               const fs_csr_opts *opts, int32_t n_elem,
                               int32_t nde, const int32_t *edof,
                               int32_t *built, int32_t *ngroups,
                               int64_t *nbatch, int64_t *nrec, int32_t *rows,
                               int32_t *gdesc, int32_t *bdesc, int32_t *ea,
                               uint16_t *off);

/* Assemble the element matrices ke (n_elem x nde x nde FP64, device)
 * straight into A's layout values, replacing them, and refresh A's FP32 /
 * BF16 copies if it holds any (rounded as csr_update_values rounds).  Same
 * effect as assembling K in CSR order and calling csr_update_values, without
 * the CSR intermediate.  Asynchronous on s; ke must stay valid until the
 * stream reaches the call. */
fs_status asm_matrix(fs_asm_t P, const double *ke, hipStream_t s);

/* Assemble the element vectors re (n_elem x nde FP64, device) into r
 * (n_rows FP64, device, the caller's row numbering of A): every entry of r
 * is written.  r must not overlap re.  Asynchronous on s. */
fs_status asm_vector(fs_asm_t P, const double *re, double *r, hipStream_t s);

/* Element storage in the assembler's order (paper: conclusion -- element
 * routines can store their contributions where the assembly kernel reads
 * them in order, which removes the reorder from the hot path).  Row-group
 * plan only (FS_E_UNSUPPORTED otherwise).  asm_element_rows fills the HOST
 * array pos (n_elem * nde int32, may be NULL to learn *rows) with, for each
 * element row (e, a), the row of a plan-ordered buffer of *rows x nde
 * doubles where that row belongs (-1 if DOF a of element e is not in A).
 * asm_matrix_ordered then assembles from such a buffer (device memory,
 * ke_ordered[pos[e*nde+a]*nde + b] = ke[e][a][b]; rows no element row maps
 * to are never read): the element values stream in order instead of being
 * gathered.  Same values, bitwise, as asm_matrix.  Asynchronous on s. */
fs_status asm_element_rows(fs_asm_t P, int32_t *pos, int64_t *rows);
fs_status asm_matrix_ordered(fs_asm_t P, const double *ke_ordered,
                             hipStream_t s);

/* asm_matrix and asm_vector together.  With the row-group plan one launch
 * does both: the lane that starts each row's element rows also sums the
 * matching element vector entries (the paper notes that tangent and
 * residual assembly can be one operation).  Same results, bitwise, as the
 * two calls.  Asynchronous on s; same argument rules as the two calls. */
fs_status asm_system(fs_asm_t P, const double *ke, const double *re,
                     double *r, hipStream_t s);

typedef struct fs_asm_stats {
    int32_t n_elem, nde;
    int64_t contrib_matrix;   /* element entries that land in K             */
    int64_t contrib_vector;   /* element entries that land in R             */
    int64_t stored_matrix;    /* index entries stored for K, with padding
                                 (4-byte positions, or 2-byte LDS offsets
                                 for the row-group plan)                   */
    int64_t stored_vector;    /* same for R                                 */
    int64_t bytes_algorithmic_matrix; /* 12 contrib_matrix + 8 nnz: element
                                 values and their 4-byte positions read,
                                 the FP64 result written                    */
    int64_t bytes_algorithmic_vector; /* 12 contrib_vector + 8 n_rows        */
    int64_t device_bytes;     /* device memory held by the plan             */
    double t_build_ms;        /* wall time of asm_create                    */
    int32_t plan;             /* FS_ASM_GATHER or FS_ASM_ROWGROUP in use    */
    int32_t reserved[7];
} fs_asm_stats;

fs_status asm_info(fs_asm_t P, fs_asm_stats *st);

/* Free the plan (after synchronising the device).  NULL is a no-op. */
fs_status asm_destroy(fs_asm_t P);

/* Copy A's FP64 values back in the CSR order csr_create saw: vals[k] is the
 * value at CSR position k (device array of nnz doubles).  The inverse of
 * csr_update_values; use it to read what asm_matrix assembled.
 * Asynchronous on s. */
fs_status csr_get_values(fs_csr_t A, double *vals, hipStream_t s);

#ifdef __cplusplus
}
#endif
#endif /* FESPMV_H */
