/*
 * submat.h -- C ABI of the MI355X (gfx950) submatrix-method library.
 *
 * The library computes the submatrix-method approximation X ~ f(A) of a
 * sparse symmetric positive-definite matrix A, with X restricted to A's
 * sparsity pattern (Lass et al., arXiv:1710.10899). The paper's main case is
 * the inverse p-th root f(lambda) = lambda^(-1/p); its subsection
 * "Applicability to other matrix operations" (Section 4) extends the method
 * to positive p-th roots, and the same per-submatrix spectral route serves
 * any real power lambda^alpha:
 *
 *   Section 3.1 (Algorithm "Construction of submatrices"): for column j,
 *     R_j = rows holding a stored entry of column j, S_j = A[R_j, R_j].
 *   Section 3.2: the operation is applied to every S_j; here a symmetric
 *     eigendecomposition S_j = Q diag(lambda) Q^T with f(lambda) = lambda^(-1/p).
 *   Section 3.3 (Algorithm "Assembly of result matrix"): column j of X on
 *     rows R_j is column R_j.indexof(j) of f(S_j).
 *   Section 3.4: X has exactly A's pattern; its value array is the
 *     concatenation of those columns and A's index arrays are reused.
 *
 * Matrix format: CSR with int32 row pointers and column indices. The pattern
 * must be structurally symmetric, each row strictly increasing, and every
 * diagonal entry stored. Because the pattern is symmetric, CSR row segment j
 * equals column j, and segment j of the output value array holds column j
 * of X (the row-based reading of Section 3 gives the same array).
 * Each S_j is used in its symmetric part (S_j + S_j^T)/2.
 *
 * Pointers: every array argument is a DEVICE pointer owned by the caller
 * (for example a torch tensor's data_ptr()), on the current HIP device.
 * Inputs are never written. Outputs are fully overwritten, never accumulated.
 * `stream` is a hipStream_t (NULL = the legacy default stream); all work is
 * enqueued on it and the call returns without waiting, except that the first
 * call for a new sparsity pattern builds a plan (pattern validation on the
 * device, one device-to-host copy) and allocates the library's workspace.
 *
 * Plans are cached by (rowptr, colind, n, nnz, device). The caller must not
 * change a pattern's contents while its plan is cached, nor free the index
 * arrays and hand their addresses to another pattern of the same n and nnz:
 * call submat_release_pattern() (or submat_release()) first. A column whose
 * order no longer fits the cached plan is not computed: its output segment
 * is NaN and it is counted (submat_query_counters slot 4); no memory
 * outside the plan's slots is touched.
 *
 * Workspaces: each stream gets its own workspace (slabs, per-item flags,
 * work counters, captured graphs) and its own status counters, allocated at
 * its first call on a plan; calls on different streams may run concurrently.
 * A plan keeps at most 4 stream workspaces (the least recently used is
 * dropped). The workspace is sized from the free device memory when the
 * plan is built, after the device's other cached plans have been trimmed,
 * least recently used first, to a quarter of the device; if a workspace
 * cannot be allocated, the other plans (then this plan's other workspaces)
 * are dropped and the allocation retried, else SUBMAT_ENOMEM.
 *
 * Errors: every int-returning call returns SUBMAT_OK (0) or a negative code;
 * submat_strerror() names it. Invalid input is reported synchronously and
 * nothing is written. Numerical failures are asynchronous: a submatrix with
 * an eigenvalue <= 0 (outside the domain of the functions above) or whose eigensolver did not
 * converge yields NaN in its output segment and is counted in device
 * counters that submat_query_status() reads. The library never aborts and
 * never prints.
 */
#ifndef SUBMAT_H
#define SUBMAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* value type of vals / x_vals / grad arrays */
#define SUBMAT_F64 0
#define SUBMAT_F32 1

/* compute precision */
#define SUBMAT_PREC_F64 0       /* batched FP64 eigensolves */
#define SUBMAT_PREC_F32_MIXED 1 /* batched FP32 eigensolves (FP64 Jacobi rotation
                                   angles); a submatrix whose FP32 eigenvalues give
                                   lambda_min <= 0 or lambda_max/lambda_min above
                                   the kappa threshold is redone in FP64 */
#define SUBMAT_PREC_F64_PLAIN 2 /* FP64, one column per launch, no batching and
                                   no graph: the per-column comparison path */

/* status codes */
#define SUBMAT_OK 0
#define SUBMAT_EINVAL -1   /* n < 1, nnz < n, p < 1, null pointer, bad dtype/precision */
#define SUBMAT_EPATTERN -2 /* rowptr not 0..nnz non-decreasing, column index out of range,
                              row not strictly increasing, or pattern not symmetric */
#define SUBMAT_ENODIAG -3  /* a diagonal entry is not stored: R_j.indexof(j) is undefined
                              (Section 3.3) */
#define SUBMAT_ENOMEM -4   /* device allocation failed */
#define SUBMAT_EHIP -5     /* a HIP runtime call failed */
#define SUBMAT_ETOOBIG -6  /* a submatrix order exceeds SUBMAT_MAX_ORDER */
#define SUBMAT_ESAVED -7   /* `saved` buffer does not belong to this pattern/dtype */
#define SUBMAT_EBREAKDOWN -8  /* CG breakdown: p^T B p <= 0 or a non-finite residual (operator not SPD) */
#define SUBMAT_ENOCONV -9     /* refinement stopped without reaching its tolerance (outputs written) */

/* largest supported submatrix order m_j = nnz of row j */
#define SUBMAT_MAX_ORDER 2048

/* option keys for submat_set_option / submat_get_option */
#define SUBMAT_OPT_KAPPA_MAX 1   /* FP64-fallback threshold on lambda_max/lambda_min (1e5) */
#define SUBMAT_OPT_USE_GRAPH 2   /* 1: capture each call sequence once in a hipGraph and
                                    replay it (default 1); 0: direct launches */
#define SUBMAT_OPT_SMALL_MAX 3   /* largest order on the one-wavefront Jacobi path, 1..64;
                                    0 (the initial state): the tuning table's (64 built in);
                                    setting it, or a table change that moves it, drops
                                    cached plans */
#define SUBMAT_OPT_WS_BYTES 4    /* workspace budget per plan in bytes (0: automatic) */
#define SUBMAT_OPT_CLUSTER_TOL 5 /* relative eigenvalue gap (times ||T||) below which the
                                    tridiagonal eigensolver computes eigenvectors by inverse
                                    iteration with reorthogonalisation (1e-7), in [0, 1) */
#define SUBMAT_OPT_TUNE_FILE 6   /* tuning table (workgroups per compute unit, the reduction's
                                    panel width, the one-wavefront bucket edge): set 1 to
                                    (re)read the file named by the environment variable
                                    SUBMAT_TUNE_FILE (lines "kind m_hi value", as written
                                    by the package's autotune module), 0 for the built-in
                                    table; get returns 1 when a file is in use. The table is
                                    first read at the first call. */
#define SUBMAT_OPT_DETERMINISTIC 7 /* 1: the adjoint is assembled without atomic adds: each
                                    phase (the one-wavefront launch, each chunk of the
                                    large-order path) leaves every D_j in memory, then every
                                    stored entry adds the terms of the columns that share it
                                    in ascending column order, so grad_a is bit-identical
                                    from run to run and exactly symmetric (one extra pass
                                    over the pattern per phase). 0 (default): atomic adds,
                                    equal up to rounding order. */
#define SUBMAT_OPT_PLAIN_STRIDE 8 /* measurement aid for SUBMAT_PREC_F64_PLAIN: the per-column
                                    path computes only every k-th column of each size bucket
                                    (buckets ordered by decreasing order, so the sample spans
                                    the order distribution) and leaves the other columns'
                                    outputs unwritten; k >= 1, default 1 (every column).
                                    No other precision looks at it. */
#define SUBMAT_OPT_XCD_QUEUES 9 /* 1 (default): the launches over (submatrix, column block)
                                    units of the back-transformation and of the adjoint's
                                    products take their units from eight queues, one per
                                    XCD, each holding every eighth submatrix, so that the
                                    units of one submatrix run together on one XCD and
                                    share its L2; 0: one queue in submatrix order. Results
                                    are bit-identical either way. */

/* spectral function f applied to every submatrix, and the meaning of `param` */
#define SUBMAT_FN_INV_ROOT 0  /* f(lambda) = lambda^(-1/p), param = p, integer >= 1 (Sections 3-4) */
#define SUBMAT_FN_ROOT     1  /* f(lambda) = lambda^(1/p),  param = p, integer >= 1 (Section 4,
                                 "Applicability to other matrix operations") */
#define SUBMAT_FN_POWER    2  /* f(lambda) = lambda^alpha,  param = alpha, finite real (the same
                                 spectral route for any real power) */

/*
 * Forward: x_vals[rowptr[j] + i] = (f(S_j))[i][c_j] for every column j and
 * i < m_j, where c_j = R_j.indexof(j) (Sections 3.1-3.4).
 *   rowptr  int32[n+1], colind int32[nnz]: CSR pattern (see above).
 *   vals    nnz values of A, type `dtype`.
 *   fn      SUBMAT_FN_*; param its parameter (an invalid pair is SUBMAT_EINVAL).
 *   x_vals  nnz values of X (same type), fully written.
 *   saved   NULL, or a device buffer of submat_saved_bytes() bytes; when given, the
 *           eigenvectors and eigenvalues of every submatrix on the large-order path
 *           are kept there so that the adjoint need not recompute them. They do
 *           not depend on fn, so one saved buffer serves every function.
 * f(lambda) is evaluated in FP64 from the eigenvalues in every precision mode.
 */
int submat_matfun_fwd(const int32_t* rowptr, const int32_t* colind, const void* vals,
                      int32_t n, int64_t nnz, int32_t fn, double param, int32_t dtype,
                      int32_t precision, void* x_vals, void* saved, void* stream);

/*
 * Adjoint (Daleckii-Krein; the paper has no gradient): for the loss
 * L = sum_q grad_x[q] * x_vals[q], grad_a[q] = dL/d vals[q] for every stored
 * entry q. Per column j, with S_j = Q diag(lambda) Q^T, w = grad_x segment j,
 * a = Q^T w, b = Q[c_j, :]^T, G[k][l] = (f(lambda_k) - f(lambda_l)) /
 * (lambda_k - lambda_l) (f'(lambda_k) when equal) and M = G o (a b^T):
 * D_j = Q (M + M^T)/2 Q^T, and every stored pair (R_j[k], R_j[l]) at
 * position q receives D_j[k][l]. grad_a is fully written (zeroed first).
 * G is evaluated without cancellation: through alpha = lambda^(1/p) for the
 * roots, through expm1/log1p of the eigenvalue ratio for a real power.
 *   saved   NULL (recompute), or the buffer filled by a forward call with the
 *           same pattern, vals, dtype and precision. The library records which
 *           pattern, dtype and precision each saved buffer was last filled for;
 *           a buffer not recorded for this call's is rejected synchronously
 *           with SUBMAT_ESAVED and nothing is written. (It cannot tell whether
 *           vals changed in between: that remains the caller's contract.)
 */
int submat_matfun_bwd(const int32_t* rowptr, const int32_t* colind, const void* vals,
                      int32_t n, int64_t nnz, int32_t fn, double param, int32_t dtype,
                      int32_t precision, const void* grad_x, void* grad_a, const void* saved,
                      void* stream);

/* The inverse p-th root (the paper's main case): submat_matfun_fwd / _bwd with
   fn = SUBMAT_FN_INV_ROOT and param = p (integer p >= 1). */
int submat_invroot_fwd(const int32_t* rowptr, const int32_t* colind, const void* vals,
                       int32_t n, int64_t nnz, int32_t p, int32_t dtype, int32_t precision,
                       void* x_vals, void* saved, void* stream);
int submat_invroot_bwd(const int32_t* rowptr, const int32_t* colind, const void* vals,
                       int32_t n, int64_t nnz, int32_t p, int32_t dtype, int32_t precision,
                       const void* grad_x, void* grad_a, const void* saved, void* stream);

/*
 * The forward of submat_invroot_fwd for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): it calls no hipMalloc/hipFree and no allocating
 * library routine, builds no cached plan and synchronises nothing. Its only
 * device memory besides the caller's arrays is a fixed scratch array of
 * 8 MiB + 1 KiB per device, held until the process ends (status slots,
 * validation bits, a work counter, m_j and c_j).
 *   Limits: n <= 1048576 (else SUBMAT_ETOOBIG, synchronously); every column
 *   is taken by the one-wavefront Jacobi path, so orders m_j <= 64 (a longer
 *   column's segment is NaN and counted in status slot 4, as for a changed
 *   pattern); precision SUBMAT_PREC_F64 or SUBMAT_PREC_F32_MIXED (else
 *   SUBMAT_EINVAL). Arguments as for submat_invroot_fwd, without `saved`.
 *   The pattern is validated on the device within the call: an invalid one
 *   writes nothing and is counted in status slot 5 (submat_query_counters),
 *   not reported synchronously.
 *   Calls on one device share the scratch array: calls that overlap in time
 *   on the same device (different streams, or threads) race and must be
 *   serialised; each call clears the counters it uses. submat_query_status /
 *   submat_query_counters on the call's stream report its counters until the
 *   next call on that stream.
 */
int submat_invroot_fwd_noalloc(const int32_t* rowptr, const int32_t* colind, const void* vals, int32_t n,
                               int64_t nnz, int32_t p, int32_t dtype, int32_t precision, void* x_vals,
                               void* stream);

/* Bytes of the optional `saved` buffer for this pattern and dtype; < 0 on error.
   Builds (and caches) the plan if needed (synchronous). */
int64_t submat_saved_bytes(const int32_t* rowptr, const int32_t* colind, int32_t n,
                           int64_t nnz, int32_t dtype, int32_t precision);

/*
 * Synchronises `stream` and reports the device counters of the last completed
 * fwd/bwd call on that stream (current device): submatrices with an eigenvalue <= 0,
 * submatrices redone in FP64 by the mixed-precision path, and submatrices whose
 * eigensolver did not converge. Any pointer may be NULL.
 */
int submat_query_status(void* stream, int64_t* n_nonpositive, int64_t* n_fallback,
                        int64_t* n_unconverged);

/*
 * Synchronises `stream` and copies the first n (n <= 8) device counters of the
 * last completed call on that stream (current device): [0] non-positive
 * submatrices, [1] FP64 redos, [2] unconverged, [3] eigenvectors of the
 * tridiagonal eigensolver (large-order path) computed by inverse iteration
 * because their eigenvalue lies in a cluster, [4] columns not computed because
 * their order does not fit the cached plan (the pattern changed under it) or
 * exceeds 64 in submat_invroot_fwd_noalloc, [5] calls of
 * submat_invroot_fwd_noalloc whose pattern failed validation, [6] columns whose
 * output was written (n after a complete call: every column exactly once,
 * whichever size bucket, chunk or precision pass took it).
 * Returns SUBMAT_EINVAL for n outside 1..8 or out NULL.
 */
int submat_query_counters(void* stream, int64_t* out, int32_t n);

/* Options (process-wide). Unknown keys return SUBMAT_EINVAL. */
int submat_set_option(int32_t key, double value);
double submat_get_option(int32_t key);

/* Name of a status code (static string). */
const char* submat_strerror(int32_t code);

/*
 * ---- Consumers of the result: sparse products, the residual metric and
 * ---- preconditioned CG. FP64 values only; every array is a device pointer
 * ---- on the current device; the pattern rules above apply (validated once
 * ---- per pattern and cached like plans). These calls are synchronous: they
 * ---- return after the result (and the host outputs) are ready.
 */

/*
 * y = M x (trans = 0) or y = M^T x (trans = 1) for the CSR matrix M with
 * M[i][colind[q]] = vals[q], q in row i. For the column-based X that
 * submat_matfun_fwd writes (segment j = column j of X), X^T x is trans = 0
 * and X x is trans = 1. x and y hold n doubles and must not overlap.
 */
int submat_spmv(const int32_t* rowptr, const int32_t* colind, const double* vals, int32_t n,
                int64_t nnz, int32_t trans, const double* x, double* y, void* stream);

/*
 * Section 4.1 ("Error for random input matrices"): the spectral norm of the
 * residual R = X^p A - I of an approximate inverse p-th root X (column-based
 * values on A's pattern), ||R||_2 = sqrt(lambda_max(R^T R)). Lanczos on
 * R^T R applied matrix-free (R v = X^p (A v) - v, R^T u = A (X^T)^p u - u),
 * with full reorthogonalisation, from a seeded start vector; stops when the
 * largest Ritz value changes by at most tol (relative) over 4 steps, or
 * after max_iter (1..4096) steps. *norm receives ||R||_2, *iters (may be
 * NULL) the number of Lanczos steps. Workspace: (max_iter + 5) n doubles,
 * kept per pattern.
 */
int submat_residual_norm(const int32_t* rowptr, const int32_t* colind, const double* a_vals,
                         const double* x_vals, int32_t n, int64_t nnz, int32_t p, int32_t max_iter,
                         double tol, double* norm, int32_t* iters, void* stream);

/*
 * Section 4.4 ("Application as preconditioner"): solve A x = b by conjugate
 * gradients on K^T A K y = K^T b, x = K y, with K the column-based values of
 * an approximate A^(-1/2) on A's pattern (k_vals; NULL: plain CG on A x = b).
 * Starts from y = 0; stops when ||r|| <= tol ||K^T b|| for the recursively
 * updated residual r of the system being solved, or after max_iter
 * iterations. Outputs: x (n doubles), *iters, *relres = ||r|| / ||K^T b||,
 * *true_relres = ||b - A x|| / ||b|| (each may be NULL). Returns
 * SUBMAT_EBREAKDOWN (outputs still written) when the operator is found not
 * positive definite. Workspace: 6 n doubles (+ nnz with K), kept per pattern.
 */
int submat_pcg(const int32_t* rowptr, const int32_t* colind, const double* a_vals,
               const double* k_vals, int32_t n, int64_t nnz, const double* b, double* x,
               double tol, int32_t max_iter, int32_t* iters, double* relres, double* true_relres,
               void* stream);

/*
 * Section 4.5 ("Controlling the approximation error"): refine the
 * submatrix-method inverse (p = 1) with the Newton-Schulz iteration
 * X_{k+1} = 2 X_k - X_k A X_k seeded with X_0 = X (x_vals, column-based on
 * A's pattern). I - A X_{k+1} = (I - A X_k)^2, so it converges quadratically
 * to A^{-1} whenever the spectral radius of I - A X_0 is below 1. The result
 * leaves A's pattern: x_dense receives the dense row-major n x n iterate
 * (n^2 doubles, caller-owned, n <= 65536). Stops when ||I - A X_k||_F /
 * sqrt(n) <= tol (*residual, may be NULL, receives that value for the
 * returned X; *iters the number of Newton-Schulz steps), after max_iter
 * steps, or when the residual grows beyond 1e3 times its start (or 1e3),
 * the last two returning SUBMAT_ENOCONV with the outputs written. Dense
 * products by rocBLAS DGEMM; workspace 3 n^2 doubles, kept per pattern.
 * (For p >= 2 the Newton-Schulz step is not stable from a seed that does
 * not commute with A, so no refinement is offered there.)
 */
int submat_refine_inverse(const int32_t* rowptr, const int32_t* colind, const double* a_vals,
                          const double* x_vals, int32_t n, int64_t nnz, double* x_dense,
                          int32_t max_iter, double tol, int32_t* iters, double* residual,
                          void* stream);

/* Drop every cached plan, graph and workspace (synchronises the device). */
void submat_release(void);

/* Drop the cached plan, workspaces, graphs and Krylov data of one pattern
   (key rowptr, colind, n, nnz on the current device; synchronises the device
   when something is freed). Call it before the pattern's index arrays are
   freed or changed. Unknown keys are not an error. SUBMAT_EINVAL for NULL. */
int submat_release_pattern(const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz);

/* ABI version: 100*major + minor. */
int32_t submat_version(void);

/*
 * Measurement helper: runs the forward (and, when grad_x != NULL, the adjoint)
 * with direct launches on `stream`, times each phase with HIP events recorded on
 * that stream, and writes per-phase totals in milliseconds to phase_ms[] and the
 * number of launches to phase_launches[] (arrays of SUBMAT_NUM_PHASES entries).
 * Phase order: plan-reset, small-jacobi, gather, tridiagonalise, tridiagonal-eig,
 * reorthogonalise, back-transform, apply-column, adjoint, fallback.
 */
#define SUBMAT_NUM_PHASES 10
int submat_time_phases(const int32_t* rowptr, const int32_t* colind, const void* vals,
                       int32_t n, int64_t nnz, int32_t fn, double param, int32_t dtype,
                       int32_t precision, void* x_vals, const void* grad_x, void* grad_a,
                       void* stream, double* phase_ms, int32_t* phase_launches);

#ifdef __cplusplus
}
#endif

#endif /* SUBMAT_H */
