/*
 * bta.h -- C ABI of the MI355X (gfx950) block Cholesky factorization and
 * selected inversion of symmetric positive-definite block-tridiagonal-
 * arrowhead (BTA) matrices.
 *
 * Paper notation (Section 2.1, Table 2): a BTA matrix A has n diagonal blocks
 * of size b, the lower blocks A_{i+1,i} (b x b), the arrowhead blocks A_{n,i}
 * (a x b, the last block row) and the arrow tip A_{n,n} (a x a); N = n*b + a.
 * a = 0 is the block-tridiagonal case.
 *
 * Block storage used by every entry point: row-major, contiguous, FP64,
 *   D[n][b][b]   = A_{i,i}    (only the lower triangle is read)
 *   B[n-1][b][b] = A_{i+1,i}
 *   R[n][a][b]   = A_{n,i}
 *   T[a][a]      = A_{n,n}    (only the lower triangle is read)
 * The factor L and the selected inverse X = Sigma = A^{-1} (restricted to
 * the nonzero block positions of A) use the same four arrays.
 *
 * Common conventions:
 *  - Every pointer argument is a device pointer (HIP device memory of the
 *    current device) owned by the caller; the library never allocates or
 *    frees memory.  Scratch memory is the caller's `work` buffer of at least
 *    bta_workspace_bytes(op, ...) bytes, 256-byte aligned.
 *  - Every call only validates its arguments and enqueues work on `stream`
 *    (0 = the null stream); it returns before the work runs (one exception:
 *    the first bta_selinv_batched call with a descriptor set).  The return
 *    value reports argument errors (BTA_EINVAL) and launch errors (BTA_EHIP)
 *    only; numerical outcomes are reported on the device (d_info).
 *  - Outputs may alias the corresponding inputs exactly (in place: LD == D,
 *    and so on); any other overlap between arrays is rejected with
 *    BTA_EINVAL.  Arrays must be 8-byte aligned.
 *  - n >= 1, b >= 1, a >= 0.  With a == 0, R/T (and LR/LT, XR/XT) may be
 *    NULL; with n == 1, B (and LB, XB) may be NULL.
 *  - The library is reentrant per stream: calls enqueued on different
 *    streams, from one or several host threads, may run concurrently as long
 *    as they use different workspaces and outputs.  The library's own helper
 *    streams and events (used by bta_selinv and bta_selinv_batched) are leased
 *    per call, so concurrent calls never share them.
 *  - No C++ exception and no abort crosses this interface.
 */
#ifndef BTA_H
#define BTA_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define BTA_API __attribute__((visibility("default")))
#else
#define BTA_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* bta_stream_t; /* a hipStream_t */

/* Status of a call.  A matrix that is not positive definite is a numerical
 * outcome, known only once the work has run: it is reported on the device
 * through d_info (bta_factor), never as a status (value 2 is unused). */
typedef enum {
  BTA_OK = 0,
  BTA_EINVAL = 1,   /* invalid argument (dims, NULL, overlap, alignment, workspace) */
  BTA_EHIP = 3,     /* a HIP runtime call failed; bta_last_error() has its text */
  BTA_ENOTSUP = 4   /* no supported HIP device (not gfx950) */
} bta_status;

typedef enum {
  BTA_OP_FACTOR = 0,
  BTA_OP_SELINV = 1,
  BTA_OP_SOLVE = 2,
  BTA_OP_LOGDET = 3
} bta_op;

/* Bytes of caller workspace that `op` needs for these sizes (nrhs is used by
 * BTA_OP_SOLVE only).  Returns 0 for invalid sizes. */
BTA_API size_t bta_workspace_bytes(int op, int64_t n, int64_t b, int64_t a, int64_t nrhs);

/*
 * POBTAF (Algorithm 1): block Cholesky factorization A = L L^T.
 *  in : D, B, R, T   blocks of A (lower triangles of D[i] and T are read)
 *  out: LD, LB, LR, LT   blocks of L: L_{i,i} (lower, exact zeros above the
 *       diagonal), L_{i+1,i}, L_{n,i}, L_{n,n} (lower, zeros above).
 *  d_info: device int64; set to 0 on success, to the 1-based global row of
 *       the first pivot that is not positive or not finite (LAPACK POTRF
 *       convention; tip rows are n*b+1 .. n*b+a), or to -1 if an internal
 *       progress watchdog fired.  On a nonzero d_info the outputs are
 *       unspecified and must not be passed to bta_selinv or bta_solve.
 */
BTA_API bta_status bta_factor(int64_t n, int64_t b, int64_t a,
               const double* D, const double* B, const double* R, const double* T,
               double* LD, double* LB, double* LR, double* LT,
               void* work, size_t work_bytes, int64_t* d_info, bta_stream_t stream);

/*
 * bta_factor without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the factorization's scratch (the progress flags,
 * the diagonal-tile inverses and the tip partial sums) lives in a fixed,
 * library-owned device array of BTA_NOALLOC_SCRATCH_BYTES (64 MiB) per
 * device, held from the library's load on that device until the process ends.
 * The call allocates nothing (no hipMalloc, no allocating library routine).
 *  - Problems whose scratch (bta_workspace_bytes(BTA_OP_FACTOR, n, b, a, 0))
 *    exceeds the limit are rejected with BTA_EINVAL before any HIP work;
 *    they need bta_factor and a workspace.
 *  - Arguments, outputs, d_info and the results are exactly those of
 *    bta_factor (the same kernels run).
 *  - Every call on a device shares that device's array, and each call resets
 *    the parts that must start cleared: calls that may overlap on one device
 *    (different streams, or different host threads) race on it and must be
 *    serialized by the caller.
 */
#define BTA_NOALLOC_SCRATCH_BYTES (64u << 20)
BTA_API bta_status bta_factor_noalloc(int64_t n, int64_t b, int64_t a,
               const double* D, const double* B, const double* R, const double* T,
               double* LD, double* LB, double* LR, double* LT, int64_t* d_info, bta_stream_t stream);

/*
 * POBTASI (Algorithm 2): selected inversion from the factor of bta_factor.
 *  in : LD, LB, LR, LT   blocks of L
 *  out: XD, XB, XR, XT   blocks of Sigma = A^{-1} at the BTA pattern:
 *       Sigma_{i,i} and Sigma_{n,n} full symmetric, Sigma_{i+1,i},
 *       Sigma_{n,i}.
 */
BTA_API bta_status bta_selinv(int64_t n, int64_t b, int64_t a,
               const double* LD, const double* LB, const double* LR, const double* LT,
               double* XD, double* XB, double* XR, double* XT,
               void* work, size_t work_bytes, bta_stream_t stream);

/*
 * Solve A x = rhs with the factor (block forward then back substitution; not
 * in the paper, which stops at the selected inverse: the textbook triangular
 * solves with L and L^T, needed for the objective of Gaussian models below).
 * rhs is [N][nrhs] row-major and is overwritten by x.
 * Workspace: bta_workspace_bytes(BTA_OP_SOLVE, n, b, a, nrhs).
 */
BTA_API bta_status bta_solve(int64_t n, int64_t b, int64_t a,
              const double* LD, const double* LB, const double* LR, const double* LT,
              double* rhs, int64_t nrhs, void* work, size_t work_bytes, bta_stream_t stream);

/*
 * log det A = 2 * sum log diag(L) over the diagonal blocks and the tip (not
 * in the paper: the determinant of A = L L^T read off the factor's diagonal).
 * d_out: device double receiving the result; the sum runs in a fixed order
 * (deterministic).  Workspace: bta_workspace_bytes(BTA_OP_LOGDET, n, b, a, 0).
 */
BTA_API bta_status bta_logdet(int64_t n, int64_t b, int64_t a, const double* LD, const double* LT,
               double* d_out, void* work, size_t work_bytes, bta_stream_t stream);

/*
 * f = log det A + sum_j y_j^T x_j, where x = A^{-1} y comes from bta_solve
 * (the objective log det Q + y^T Q^{-1} y of Gaussian models).  y and x are
 * [N][nrhs] row-major device arrays (they may be the same array); d_out is a
 * device double.  Workspace: bta_workspace_bytes(BTA_OP_LOGDET, ...).
 */
BTA_API bta_status bta_logdet_quad(int64_t n, int64_t b, int64_t a, const double* LD, const double* LT,
                    const double* y, const double* x, int64_t nrhs, double* d_out,
                    void* work, size_t work_bytes, bta_stream_t stream);

/*
 * Gradient of f = log det Q + sum_j y_j^T Q^{-1} y_j with respect to the block
 * arrays, from the selected inverse X (bta_selinv) and x = Q^{-1} y:
 * G = Sigma - sum_j x_j x_j^T on the BTA pattern, returned as
 *   GD = s*G_D, GB = 2s*G_B, GR = 2s*G_R, GT = s*G_T
 * (the lower and arrow blocks also stand at their mirrored positions of Q),
 * and gy = 2s*x when gy is not NULL.  s = *d_scale (device double), or 1 when
 * d_scale is NULL.  Elementwise: G* may alias X* exactly (in place).
 */
BTA_API bta_status bta_grad_logdet_quad(int64_t n, int64_t b, int64_t a,
                    const double* XD, const double* XB, const double* XR, const double* XT,
                    const double* x, int64_t nrhs, const double* d_scale,
                    double* GD, double* GB, double* GR, double* GT, double* gy, bta_stream_t stream);

/*
 * Batched interface: many independent BTA matrices of different n, b, a.
 * The descriptor array lives in host memory; every pointer in it is a device
 * pointer with the same conventions as the single-matrix calls (exact
 * in-place aliasing allowed within a matrix; arrays of different matrices
 * must not overlap).  d_info is that matrix's device int64 info.
 */
typedef struct {
  int64_t n, b, a;
  const double *D, *B, *R, *T;   /* A blocks (bta_factor_batched input) */
  double *LD, *LB, *LR, *LT;     /* L blocks (factor output, selinv input) */
  double *XD, *XB, *XR, *XT;     /* selected-inverse blocks (selinv output) */
  int64_t* d_info;
} bta_desc;

/* Workspace bytes for a batched op (BTA_OP_FACTOR or BTA_OP_SELINV); 0 on invalid input. */
BTA_API size_t bta_batched_workspace_bytes(int op, int count, const bta_desc* descs);

/* POBTAF for every matrix of the batch, all in one persistent kernel launch. */
BTA_API bta_status bta_factor_batched(int count, const bta_desc* descs, void* work, size_t work_bytes,
                               bta_stream_t stream);

/* POBTASI for every matrix of the batch: the launches of all matrices are
 * merged stage by stage (one grouped launch per stage across the batch), the
 * tile shape of every merged GEMM launch is chosen by the autotuner (measured
 * on first use of a shape class), and the whole launch sequence is captured
 * once in a HIP graph per descriptor set and replayed (the graphs of the eight
 * most recently used descriptor sets are kept).  In the graph the per-block
 * preprocessing and the arrow rows form one branch and the backward sweep
 * another; each sweep step depends only on the stage that completes its
 * blocks (the backward recurrence of Algorithm 2).
 * Exception to the enqueue-only convention: the first call with a descriptor
 * set runs the stages eagerly and, for shape classes not yet in the tuning
 * table, times both tilings on `stream` and waits for those timings on the
 * host.  Later calls with the same descriptor set, workspace and device only
 * enqueue: an upload of the stage table from a pinned host buffer the library
 * owns, then the graph.  No call may be made while `stream` is being captured
 * (the library replays its own graph). */
BTA_API bta_status bta_selinv_batched(int count, const bta_desc* descs, void* work, size_t work_bytes,
                               bta_stream_t stream);

/* Static text for a status code. */
BTA_API const char* bta_status_string(int status);

/* Text of the last BTA_EHIP / BTA_EINVAL error raised on this thread. */
BTA_API const char* bta_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BTA_H */
