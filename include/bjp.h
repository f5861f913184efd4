/*
 * bjp.h - block-Jacobi preconditioned conjugate gradient and Lanczos
 * condition-number estimation for sparse SPD systems on AMD Instinct MI355X
 * (gfx950).
 *
 * Method (arXiv 2410.02408, "Optimised Hybrid Classical-Quantum Algorithm
 * for Accelerated Solution of Sparse Linear Systems"):
 *   - Section 3.1: solve A x = b for sparse symmetric positive-definite A;
 *     the quality measure is kappa(A) = ||A|| ||A^-1|| (2-norm: the ratio of
 *     extreme eigenvalues).
 *   - Section 3.2: A and b are split into contiguous diagonal blocks A_i of
 *     n_b rows (the partition code of Section 4.2 leaves a shorter last
 *     block when n_b does not divide N).
 *   - Section 3.3: each block gets a preconditioner M_i and the system
 *     M_i A_i x_i = M_i b_i.  The paper uses M_i = diag(A_i)^-1; this
 *     library uses the inverse of the whole block A_ii (block Jacobi), which
 *     equals the paper's choice at n_b = 1.
 *   - Section 3.6: the solution is the concatenation of block solutions;
 *     conjugate gradient generalises that aggregate to coupled blocks.
 *   - Section 3.7: accuracy is ||A x - b|| / ||b||.
 * kappa of the preconditioned operator is the quantity that sets the cost
 * of the paper's quantum stage (Sections 2.2 and 3.4); it is estimated here
 * with Lanczos.
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless the comment says "host".
 *   - Work is enqueued on the caller's stream `stream` (0 = null stream).
 *   - The library never allocates device memory: the caller queries the
 *     workspace size with the matching *_workspace() call and passes a
 *     buffer of at least that many bytes, 256-byte aligned.
 *   - Entry points that fill a host info struct synchronise `stream` before
 *     returning; bjp_apply is fully asynchronous.
 *   - Return value: BJP_OK (0) or a negative bjp_status; nothing throws or
 *     aborts across this interface.  Calls on one workspace must not
 *     overlap.
 */
#ifndef BJP_H
#define BJP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BJP_OK = 0,
    BJP_EINVAL = -1,      /* bad sizes, pointers, CSR structure or block spec */
    BJP_ENOTSPD = -2,     /* a diagonal block is not positive definite        */
    BJP_ENOCONV = -3,     /* max_iter (or the replacement budget) exhausted   */
    BJP_EBREAKDOWN = -4,  /* p^T A p <= 0 or r^T M^-1 r <= 0 (A not SPD)      */
    BJP_ENONFINITE = -5,  /* NaN/Inf in the input or produced by the solve    */
    BJP_EWORKSPACE = -6,  /* workspace missing, too small or misaligned       */
    BJP_EHIP = -7         /* a HIP runtime call failed                         */
} bjp_status;

/* Sparse matrix in CSR form (device arrays).  Full symmetric storage (both
 * triangles), int32 indices, FP64 values; duplicate (i, j) entries are
 * summed, columns inside a row may be unsorted.  n >= 0; nnz = row_ptr[n].
 * n and nnz are at most BJP_MAX_DIM (a margin below INT32_MAX keeps every
 * index the kernels form, such as one grid stride past the last row, inside
 * int32); larger sizes are rejected with BJP_EINVAL. */
#define BJP_MAX_DIM (2147483647 - (1 << 24))
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *row_ptr;   /* [n+1] */
    const int32_t *col_idx;   /* [nnz] */
    const double *val;        /* [nnz] */
} bjp_csr_t;

/* Block partition (Section 3.2).  block_size > 0: contiguous blocks of
 * block_size rows, block t = rows [t*block_size, min((t+1)*block_size, n)).
 * block_size == 0: explicit partition given by `offsets` (host array of
 * num_blocks+1 strictly increasing entries, offsets[0] = 0,
 * offsets[num_blocks] = n).  Every block has at most BJP_MAX_BLOCK rows. */
typedef struct {
    int32_t block_size;
    int32_t num_blocks;       /* used only when block_size == 0 */
    const int32_t *offsets;   /* host; used only when block_size == 0 */
} bjp_block_spec_t;

#define BJP_MAX_BLOCK 64

/* Storage precision of the block inverses. */
typedef enum {
    BJP_FP64 = 0,        /* FP64 inverses, FP64 application */
    BJP_FP32_STORE = 1   /* FP32 inverses applied in FP32 inside the FP64 solve */
} bjp_precision;

/* Preconditioner handle: plain data pointing into the workspace given to
 * bjp_precondition.  It stays valid while that workspace is alive and
 * unmodified.  Layout (for readers of the library's kernels): blocks are
 * grouped into "packets" of 64/group consecutive blocks, group = the
 * smallest power of two >= the largest block; every packet stores the
 * symmetric block inverses diagonal by diagonal (see the kernels). */
typedef struct {
    int32_t n;
    int32_t block_size;       /* uniform block size (a requested size above n is
                                 stored as n: one block), or 0 for an explicit
                                 partition */
    int32_t num_blocks;
    int32_t precision;        /* bjp_precision */
    int32_t group;            /* lanes per block, power of two <= 64 */
    int32_t num_packets;
    int32_t packet_elems;     /* scalars per packet */
    int32_t pad;
    const int32_t *offsets;   /* device [num_blocks+1] */
    const void *tiles;        /* device, num_packets * packet_elems scalars */
} bjp_precond_t;

/* Bytes of workspace bjp_precondition needs for this matrix and partition. */
int bjp_precondition_workspace(const bjp_csr_t *A, const bjp_block_spec_t *spec,
                               int precision, size_t *bytes /* host out */);

/* Build M = blockdiag(A_11, ..., A_kk)^-1 (Sections 3.2-3.3): extract every
 * diagonal block of A, factor it A_tt = L L^T (Cholesky, no pivoting) and
 * store M_t^-1 = L^-T L^-1 in `ws`.  Validates the CSR structure first.
 * On BJP_ENOTSPD, *failed_block (host, may be NULL) receives the index of
 * the first block whose Cholesky pivot was <= 0 or not finite; otherwise -1.
 * Synchronises `stream`. */
int bjp_precondition(const bjp_csr_t *A, const bjp_block_spec_t *spec, int precision,
                     void *ws, size_t ws_bytes, bjp_precond_t *M_out /* host out */,
                     int32_t *failed_block /* host out */, hipStream_t stream);

/* z = M^-1 r, block by block: z_t = A_tt^-1 r_t for every diagonal block t
 * (the preconditioner of Section 3.3 with the whole block inverted; at
 * n_b = 1 it is the paper's point Jacobi, r_i / A_ii).  r and z are device
 * [n]; they must not overlap.  Asynchronous; returns BJP_EINVAL for a NULL
 * pointer or a handle that does not describe a partition of n rows. */
int bjp_apply(const bjp_precond_t *M, const double *r, double *z, hipStream_t stream);

/* Optional kernel timing.  When a solver is given one, every stride-th
 * launch of the selected kernel inside its iteration loop (launches 0,
 * stride, 2*stride, ...) is bracketed by a pair of events recorded on the
 * solver's stream: events[2i] before, events[2i+1] after the i-th timed
 * launch, for the first `capacity` timed launches.  Each event pair adds a
 * few microseconds between the launches it brackets, so a stride above 1
 * keeps the timing from slowing the solve it measures.  The events are
 * created and destroyed by the caller (host array of 2*capacity handles). */
typedef enum {
    BJP_KERNEL_APPLY = 0,   /* the block-inverse application (x, r update + z = M^-1 r) */
    BJP_KERNEL_SPMV = 1     /* the sparse product q = A p                           */
} bjp_kernel_id;

typedef struct {
    int32_t kernel;         /* bjp_kernel_id */
    int32_t capacity;       /* event pairs available */
    int32_t recorded;       /* out: pairs recorded */
    int32_t stride;         /* time every stride-th launch (0 or 1: every launch) */
    hipEvent_t *events;     /* host array [2*capacity] */
} bjp_timing_t;

/* Solver options.  Zero-initialised fields take the defaults noted. */
typedef struct {
    double tol;               /* relative residual target (default 1e-10)          */
    int32_t max_iter;         /* iteration cap (default n)                          */
    int32_t x0_given;         /* 1: x holds the starting guess; 0: start from 0     */
    int32_t max_replacements; /* true-residual restarts (default 3; <0 means none)  */
    int32_t check_every;      /* iterations between convergence polls (default 16) */
    int32_t spmv_lanes;       /* CSR product schedule: 0 = auto, 1,2,..,64 = lanes
                                 per row, -2 = column panels for the iteration's
                                 product (rows of >= 12 entries on average, n >=
                                 512; BJP_EINVAL otherwise; auto picks them from
                                 n >= 2^20 on), other < 0 = row blocks streamed
                                 through LDS                                      */
    int32_t pad;
    double *history;          /* device, optional, >= max_iter+1 entries: recursive
                                 relative residual after each iteration             */
    bjp_timing_t *timing;     /* host, optional kernel timing (see bjp_timing_t)    */
} bjp_pcg_opts_t;

typedef struct {
    int32_t status;            /* bjp_status of the solve                         */
    int32_t iterations;        /* PCG iterations performed                         */
    int32_t replacements;      /* true-residual restarts used                      */
    int32_t polls;             /* host convergence polls                           */
    double rel_res_recursive;  /* ||r_k|| / ||b|| of the recurrence                */
    double rel_res_true;       /* ||b - A x|| / ||b|| recomputed at the end        */
} bjp_pcg_info_t;

/* Bytes of workspace bjp_pcg_solve needs for this matrix (with rows of >= 12
 * entries on average this includes the column-panel copy of A: 12 bytes per
 * entry and 100 bytes per row). */
int bjp_pcg_workspace(const bjp_csr_t *A, size_t *bytes /* host out */);

/* Solve A x = b by preconditioned CG (Hestenes-Stiefel with a symmetric
 * preconditioner; M == NULL gives plain CG).  Stops when the recursive
 * residual satisfies ||r|| <= tol ||b||, then recomputes ||b - A x|| / ||b||
 * (Section 3.7); if that is above tol the residual is replaced by the true
 * one and iteration continues (up to max_replacements times).
 *   b: device [n], x: device [n] (in: x0 when opts->x0_given; out: solution,
 *   or the last iterate on BJP_ENOCONV / BJP_EBREAKDOWN).  b = 0 gives x = 0.
 * Systems of at most 2048 rows (at most 32 entries per row on average) with
 * spmv_lanes = 0 and no timing are solved in a single workgroup, the whole
 * solve in one launch (the same steps and decisions; info->polls = 1 and
 * check_every is not used).
 * Synchronises `stream`; `info` (host) is always filled. */
int bjp_pcg_solve(const bjp_csr_t *A, const bjp_precond_t *M, const double *b, double *x,
                  const bjp_pcg_opts_t *opts, void *ws, size_t ws_bytes,
                  bjp_pcg_info_t *info /* host out */, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Allocation-free solve, for callers that cannot allocate device memory or
 * pass a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).
 * ------------------------------------------------------------------------ */

/* Size of the library's static scratch: one copy per GPU, held from the
 * library's first use on that GPU until the process ends. */
#define BJP_NOALLOC_SCRATCH_BYTES (128u << 20)

/* bjp_pcg_solve with the library's static scratch as its workspace: same
 * arguments minus the workspace, same algorithm, kernels and results for the
 * same options.  Differences:
 *   - The scratch must hold the solver's vectors: about 40 n + 2 nnz bytes
 *     plus 67 KB (the bjp_pcg_workspace size without the column-panel copy);
 *     a larger system returns BJP_EWORKSPACE before any HIP call.  That
 *     admits up to ~2.48M rows of 7 entries (the 128^3 stencil fits).
 *   - The iteration's product never uses column panels (spmv_lanes = -2 is
 *     BJP_EINVAL; the automatic choice takes the CSR schedule).
 *   - Host polls copy the solver state into ordinary host memory and
 *     synchronise `stream` (no pinned host memory, no events).
 * Nothing is allocated: no device memory, no pinned host memory.  The
 * scratch of the current device is used, so `stream` must belong to the
 * current device.  Every call on one GPU shares that GPU's scratch, which
 * keeps the last call's contents (the solver initialises everything it
 * reads): calls that overlap on one GPU, from several host threads or on
 * several streams, race and give wrong results.  Synchronises `stream`;
 * `info` (host) is always filled. */
int bjp_pcg_solve_noalloc(const bjp_csr_t *A, const bjp_precond_t *M, const double *b, double *x,
                          const bjp_pcg_opts_t *opts, bjp_pcg_info_t *info /* host out */,
                          hipStream_t stream);

typedef struct {
    int32_t status;       /* bjp_status                                          */
    int32_t steps_done;   /* Lanczos steps taken (< steps after an invariant-
                             subspace breakdown, which is success)              */
    double theta_min;     /* smallest Ritz value                                  */
    double theta_max;     /* largest Ritz value                                   */
    double kappa;         /* theta_max / theta_min, a lower bound on kappa         */
} bjp_kappa_info_t;

/* Bytes of workspace bjp_kappa_estimate needs for `steps` Lanczos steps. */
int bjp_kappa_workspace(const bjp_csr_t *A, int steps, size_t *bytes /* host out */);

/* Estimate kappa(M^-1 A) = lambda_max / lambda_min (kappa(A) when M == NULL),
 * the condition number of Section 3.1 (2-norm) of the preconditioned system of
 * Section 3.3, which sets the cost of the quantum stage (Sections 2.2, 3.4),
 * with `steps` Lanczos steps in the M inner product, started from v0
 * (device [n], nonzero), with full reorthogonalisation (classical
 * Gram-Schmidt applied twice), then the extreme eigenvalues of the
 * tridiagonal by Sturm-count multisection.  A step whose new off-diagonal is
 * below 1e-12 of the largest coefficient ends the run early (success).
 * alpha/beta (device [steps], optional) receive the tridiagonal.  Systems of
 * at most 2048 rows (at most 32 entries per row on average) with steps <=
 * 2048 run the estimate in a single workgroup (the same steps).
 * Synchronises `stream`; `info` (host) is always filled. */
int bjp_kappa_estimate(const bjp_csr_t *A, const bjp_precond_t *M, const double *v0,
                       int steps, double *alpha, double *beta, void *ws, size_t ws_bytes,
                       bjp_kappa_info_t *info /* host out */, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batches of independent systems (every system advances in the same kernel
 * launches; the iterations between polls are replayed from a captured graph).
 * The batch is a single block-diagonal CSR matrix: system s owns rows
 * [sys_rows[s], sys_rows[s+1]) and every column of those rows must lie in
 * the same range (checked).  Each system has its own uniform block size.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t num_systems;
    const int32_t *sys_rows;     /* host [num_systems+1], sys_rows[0] = 0, last = n */
    const int32_t *block_size;   /* host [num_systems], each 1..BJP_MAX_BLOCK */
} bjp_batch_t;

/* Batched preconditioner handle (points into the bjp_batch_precondition
 * workspace). */
typedef struct {
    int32_t num_systems;
    int32_t precision;           /* bjp_precision */
    const void *systems;         /* device table, one record per system */
    const void *tiles;           /* device, diagonal packets of every system */
} bjp_batch_precond_t;

typedef struct {
    double tol;                  /* default 1e-10 */
    int32_t max_iter;            /* per system, default its size */
    int32_t max_replacements;    /* default 3; < 0 means none */
    int32_t lanes;               /* CSR product schedule: 0 = auto, a power of two <= 64
                                    = lanes per row, < 0 = row blocks streamed
                                    through LDS                                      */
    int32_t tile_rows;           /* rows per SpMV tile: 0 = auto (2048), else >= 256 */
    int32_t check_every;         /* iterations between convergence polls (default 16) */
    int32_t eager;               /* 0: the check_every iterations between polls are
                                    captured once into a hipGraph and replayed;
                                    1: every kernel is launched from the host       */
    const int32_t *sys_lanes;    /* host [num_systems] or NULL: per-system product
                                    schedule (as `lanes`; 0 = the batch's `lanes`).
                                    Systems sharing a schedule share a launch.     */
    const int32_t *sys_tile_rows;/* host [num_systems] or NULL: per-system rows per
                                    product tile (as `tile_rows`; 0 = the batch's)  */
} bjp_batch_opts_t;

/* Per-system result (same layout as the device record the solver writes). */
typedef struct {
    int32_t status, iterations, replacements, pad;
    double rel_res_recursive, rel_res_true;
} bjp_system_info_t;

typedef struct {
    int32_t status;              /* BJP_OK if every system converged, else the first failure */
    int32_t systems_ok;
    int32_t max_iterations;
    int32_t pad;
    int64_t total_iterations;    /* sum over systems */
    double max_rel_res_true;
} bjp_batch_info_t;

int bjp_batch_precondition_workspace(const bjp_csr_t *A, const bjp_batch_t *B, int precision,
                                     size_t *bytes /* host out */);

/* Per-system block-Jacobi setup (the same extraction, Cholesky and inverse as
 * bjp_precondition) for every system of the batch.  *failed_block receives the
 * global index (counting blocks system by system) of the first non-SPD block.
 * Synchronises `stream`. */
int bjp_batch_precondition(const bjp_csr_t *A, const bjp_batch_t *B, int precision, void *ws,
                           size_t ws_bytes, bjp_batch_precond_t *M_out /* host out */,
                           int32_t *failed_block /* host out */, hipStream_t stream);

int bjp_batch_pcg_workspace(const bjp_csr_t *A, const bjp_batch_t *B, size_t *bytes /* host out */);

/* Solve every system of the batch with PCG (the algorithm, stopping rule and
 * true-residual check of bjp_pcg_solve, x0 = 0).  All systems advance
 * together: each kernel launch covers every system (row and packet tiles that
 * never straddle two systems), each system keeps its own scalars, and a
 * converged system drops out.  b, x: device [n].  per_system (host
 * [num_systems], optional) receives each system's result.  Synchronises
 * `stream`. */
int bjp_batch_pcg_solve(const bjp_csr_t *A, const bjp_batch_t *B, const bjp_batch_precond_t *M,
                        const double *b, double *x, const bjp_batch_opts_t *opts, void *ws,
                        size_t ws_bytes, bjp_batch_info_t *info /* host out */,
                        bjp_system_info_t *per_system /* host out, optional */, hipStream_t stream);

/* Gradient with respect to the stored values of A of a loss L(x), x = A^-1 b,
 * given the adjoint lambda = A^-1 dL/dx (a second bjp_pcg_solve with rhs
 * dL/dx, which is also dL/db): grad[k] = -lambda[i] * x[col_idx[k]] for every
 * stored entry k of row i (the outer product -lambda x^T on A's pattern).
 * lambda, x: device [n]; grad: device [nnz].  The CSR structure is trusted
 * (validate it with bjp_precondition or bjp_pcg_solve first).  Asynchronous.
 * (Differentiation through the solve; the paper's method has no gradient.) */
int bjp_value_grad(const bjp_csr_t *A, const double *lambda, const double *x, double *grad,
                   hipStream_t stream);

/* Human-readable name of a status code (static storage). */
const char *bjp_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* BJP_H */
