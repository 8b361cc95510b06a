"""FP64 CPU oracle of the consumers of the submatrix method's result -- TEST
INFRASTRUCTURE ONLY (tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg). Shares nothing with the GPU library.

* Section 4.1, error metric: ||R||_2 with R = X^p A - I, the spectral norm
  being sqrt(lambda_max(R^H R)). ``residual_norm_sparse`` forms no dense
  matrix: R is applied as an operator (X^p (A v) - v, and its transpose)
  and its largest singular value is taken from ARPACK (scipy's svds), so
  sizes where the dense definition in ``submat_oracle.residual_norm`` is
  out of reach can still be checked.
* Section 4.4, application as preconditioner: with K ~ A^(-1/2) from the
  submatrix method, solve K^T A K y = K^T b by the conjugate gradient
  method and return x = K y; without K, plain CG on A x = b. ``cg`` is the
  Hestenes-Stiefel recurrence written out, starting from y = 0 and stopping
  when the recursively updated residual satisfies ||r|| <= tol ||K^T b||
  (the paper's residual threshold, read as relative to the right-hand side
  of the system being solved), or after maxit iterations.

X and K are column-based value arrays on A's pattern: CSR value segment j
holds column j (Section 3.3).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def column_based_matrix(rowptr, colind, vals, n: int) -> sp.csr_matrix:
    """The matrix whose column j is value segment j (rows colind[segment])."""
    rows = np.asarray(colind, dtype=np.int64)
    cols = np.repeat(np.arange(n), np.diff(np.asarray(rowptr, dtype=np.int64)))
    return sp.csr_matrix((np.asarray(vals, dtype=np.float64), (rows, cols)), shape=(n, n))


def row_based_matrix(rowptr, colind, vals, n: int) -> sp.csr_matrix:
    return sp.csr_matrix((np.asarray(vals, dtype=np.float64), np.asarray(colind), np.asarray(rowptr)),
                         shape=(n, n))


def residual_operator(xvals, rowptr, colind, avals, n: int, p: int) -> spla.LinearOperator:
    """R = X^p A - I as an operator (and R^T = A (X^T)^p - I)."""
    X = column_based_matrix(rowptr, colind, xvals, n)
    A = row_based_matrix(rowptr, colind, avals, n)
    XT = X.T.tocsr()

    def mv(v):
        v = np.asarray(v, dtype=np.float64).ravel()
        t = A @ v
        for _ in range(p):
            t = X @ t
        return t - v

    def rmv(u):
        u = np.asarray(u, dtype=np.float64).ravel()
        t = u
        for _ in range(p):
            t = XT @ t
        return A @ t - u

    return spla.LinearOperator((n, n), matvec=mv, rmatvec=rmv, dtype=np.float64)


def residual_norm_sparse(xvals, rowptr, colind, avals, n: int, p: int, seed: int = 0) -> float:
    """||X^p A - I||_2 = largest singular value of R (ARPACK, full
    precision)."""
    R = residual_operator(xvals, rowptr, colind, avals, n, p)
    v0 = np.random.default_rng(seed).standard_normal(n)
    s = spla.svds(R, k=1, which="LM", v0=v0, tol=0, return_singular_vectors=False, maxiter=20 * n)
    return float(s[0])


def cg(rowptr, colind, avals, b, tol: float = 1e-6, maxit: int | None = None, kvals=None):
    """Conjugate gradients on K^T A K y = K^T b (K = I when kvals is None),
    x = K y. Returns (x, iterations, ||r|| / ||K^T b||)."""
    n = len(rowptr) - 1
    A = row_based_matrix(rowptr, colind, avals, n)
    b = np.asarray(b, dtype=np.float64)
    if kvals is not None:
        K = column_based_matrix(rowptr, colind, kvals, n)
        KT = K.T.tocsr()

        def op(v):
            return KT @ (A @ (K @ v))

        rhs = KT @ b
    else:
        K = None

        def op(v):
            return A @ v

        rhs = b.copy()
    maxit = 2 * n if maxit is None else maxit
    y = np.zeros(n)
    r = rhs.copy()
    d = r.copy()                      # search direction
    rr = float(r @ r)
    bnorm = np.sqrt(rr)
    it = 0
    if bnorm == 0.0:
        return (np.zeros(n), 0, 0.0)
    while it < maxit:
        q = op(d)
        dq = float(d @ q)
        if not dq > 0.0:
            break                     # the operator is not positive definite
        alpha = rr / dq
        y = y + alpha * d
        r = r - alpha * q
        rr_new = float(r @ r)
        it += 1
        if np.sqrt(rr_new) <= tol * bnorm:
            rr = rr_new
            break
        d = r + (rr_new / rr) * d
        rr = rr_new
    x = K @ y if K is not None else y
    return x, it, float(np.sqrt(rr) / bnorm)


def refine_inverse(rowptr, colind, avals, xvals, tol: float = 1e-14, maxit: int = 20):
    """Section 4.5: refinement of the submatrix-method inverse (p = 1),
    used as the initial guess of the Newton-Schulz iteration
    X_{k+1} = 2 X_k - X_k A X_k (so that I - A X_{k+1} = (I - A X_k)^2).
    Stops when ||I - A X_k||_F / sqrt(n) <= tol, after maxit steps, or when
    that residual exceeds 1e3 times its start (or 1e3). Returns (dense X,
    steps, residual of the returned X, converged)."""
    n = len(rowptr) - 1
    A = row_based_matrix(rowptr, colind, avals, n).toarray()
    X = column_based_matrix(rowptr, colind, xvals, n).toarray()
    I = np.eye(n)
    k = 0
    res0 = None
    while True:
        T = A @ X
        res = float(np.linalg.norm(T - I) / np.sqrt(n))
        if res0 is None:
            res0 = res
        if res <= tol:
            return X, k, res, True
        if not np.isfinite(res) or res > 1e3 * max(res0, 1.0) or k >= maxit:
            return X, k, res, False
        X = 2.0 * X - X @ T
        k += 1
