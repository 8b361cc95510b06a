"""Plain FP64 CPU oracle of the submatrix method -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run this module. It shares no code with the GPU
library (``paper_1710_10899_amd``) and imports nothing from it; the product
path never calls it.

What it computes (Lass et al., "A Massively Parallel Algorithm for the
Approximate Calculation of Inverse p-th Roots of Large Sparse Matrices"):

* Section 3.1, Algorithm "Construction of submatrices": for column j, R_j is
  the set of rows i holding an entry A[i][j]; the dense submatrix is
  S_j[k][l] = A[R_j[k]][R_j[l]].
* Section 3.2: the operation of interest (the inverse p-th root) is
  applied to every S_j; the paper leaves the method free. This oracle takes
  the spectral route named in Section 2 for symmetric matrices: a symmetric
  eigendecomposition S = Q diag(lambda) Q^T (LAPACK through numpy) and
  f(lambda) = lambda^(-1/p).
* Section 4, "Applicability to other matrix operations": the same method
  applies to positive p-th roots, f(lambda) = lambda^(1/p); the spectral
  route takes any real power f(lambda) = lambda^alpha the same way
  (functions "inv_root", "root", "power"; the parameter is p for the roots
  and alpha for the power).
* Section 3.3, Algorithm "Assembly of result matrix": column j of X on rows
  R_j is the column of f(S_j) that belongs to j, i.e. column R_j.indexof(j).
* Section 3.4: X has exactly A's pattern; in CSR/CSC its value array is the
  concatenation of those columns and the index arrays are A's.

Readings taken where the paper is silent:

1. R_j is the *stored* pattern of column j (explicit zeros are kept), so X's
   pattern is A's pattern bit for bit (Section 3.4).
2. A column whose diagonal entry is not stored has no R_j.indexof(j): this is
   an input error (ENODIAG).
3. Rows are used for columns: for a symmetric pattern the CSR row segment j
   equals column j, and the CSR value segment j of X is the column-based
   result read row-wise (Section 3, row/column equivalence).
4. S_j is symmetrised as (S_j + S_j^T)/2; this is exact for exactly
   symmetric storage.
5. A submatrix with an eigenvalue <= 0 is outside the domain of the
   functions (no real inverse p-th root; for the others, kept to the same
   SPD domain): its segment is NaN and it is counted.
6. p is an integer >= 1; alpha is any finite real.
7. The adjoint (not in the paper) is the Daleckii-Krein formula with the
   divided differences of f in closed form; gradients are per stored entry.
"""
from __future__ import annotations

import numpy as np


class PatternError(ValueError):
    def __init__(self, code: str, msg: str):
        super().__init__(f"{code}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# Input checks (the conditions under which Algorithms 1 and 2 are defined)


def validate(rowptr, colind, n: int) -> None:
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    if n <= 0 or rowptr.shape[0] != n + 1:
        raise PatternError("EINVAL", "rowptr must have n+1 entries, n >= 1")
    if rowptr[0] != 0 or rowptr[-1] != colind.shape[0] or np.any(np.diff(rowptr) < 0):
        raise PatternError("EPATTERN", "rowptr must start at 0, end at nnz and not decrease")
    if colind.size and (colind.min() < 0 or colind.max() >= n):
        raise PatternError("EPATTERN", "column index out of range")
    present = set()
    for j in range(n):
        seg = colind[rowptr[j]:rowptr[j + 1]]
        if np.any(np.diff(seg) <= 0):
            raise PatternError("EPATTERN", f"row {j}: indices not strictly increasing")
        if j not in set(seg.tolist()):
            raise PatternError("ENODIAG", f"row {j}: diagonal entry not stored")
        present.update((j, int(i)) for i in seg)
    for (j, i) in present:
        if (i, j) not in present:
            raise PatternError("EPATTERN", f"pattern not symmetric at ({j},{i})")


# ---------------------------------------------------------------------------
# Section 3.1 (Algorithm "Construction of submatrices")


def submatrix_rows(rowptr, colind, j: int) -> np.ndarray:
    """R_j: the rows holding a stored entry in column j (sorted)."""
    return np.asarray(colind[rowptr[j]:rowptr[j + 1]], dtype=np.int64)


def gather_submatrix(rowptr, colind, vals, R: np.ndarray):
    """S[k][l] = A[R[k]][R[l]] (0 where not stored), and the position in the
    value array of every stored pair (-1 where not stored)."""
    m = R.shape[0]
    S = np.zeros((m, m), dtype=np.float64)
    pos = np.full((m, m), -1, dtype=np.int64)
    for k in range(m):
        a, b = rowptr[R[k]], rowptr[R[k] + 1]
        seg = np.asarray(colind[a:b], dtype=np.int64)
        idx = np.searchsorted(seg, R)
        idx_c = np.minimum(idx, max(seg.shape[0] - 1, 0))
        found = (idx < seg.shape[0]) & (seg[idx_c] == R)
        pos[k, found] = a + idx[found]
        S[k, found] = np.asarray(vals, dtype=np.float64)[a + idx[found]]
    return S, pos


def symmetrise(S: np.ndarray) -> np.ndarray:
    return 0.5 * (S + S.T)


# ---------------------------------------------------------------------------
# Section 3.2: the submatrix operation, spectral route (Section 2)


def inv_root(lam: np.ndarray, p: int) -> np.ndarray:
    """f(lambda) = lambda^(-1/p), rounded as one division of a root."""
    if p == 1:
        return 1.0 / lam
    if p == 2:
        return 1.0 / np.sqrt(lam)
    if p == 3:
        return 1.0 / np.cbrt(lam)
    return 1.0 / np.power(lam, 1.0 / p)


def root(lam: np.ndarray, p: int) -> np.ndarray:
    """alpha = lambda^(1/p)."""
    if p == 1:
        return lam.copy()
    if p == 2:
        return np.sqrt(lam)
    if p == 3:
        return np.cbrt(lam)
    return np.power(lam, 1.0 / p)


FUNCTIONS = ("inv_root", "root", "power")


def check_function(fn: str, param) -> None:
    if fn not in FUNCTIONS:
        raise PatternError("EINVAL", f"function must be one of {FUNCTIONS}")
    if fn in ("inv_root", "root"):
        if not (param >= 1 and float(param) == int(param)):
            raise PatternError("EINVAL", "p must be an integer >= 1")
    elif not np.isfinite(param):
        raise PatternError("EINVAL", "alpha must be finite")


def spectral_function(lam: np.ndarray, fn: str, param) -> np.ndarray:
    """f(lambda) for the selected function."""
    if fn == "inv_root":
        return inv_root(lam, int(param))
    if fn == "root":
        return root(lam, int(param))
    return np.power(lam, float(param))


def eig(S: np.ndarray):
    lam, Q = np.linalg.eigh(S)
    return lam, Q


def column_of_function(S: np.ndarray, c: int, fn: str, param):
    """Column c of f(S) = Q (f(lambda) * Q[c, :]); (x, ok)."""
    lam, Q = eig(S)
    if lam.min() <= 0.0:
        return np.full(S.shape[0], np.nan), False
    return Q @ (spectral_function(lam, fn, param) * Q[c, :]), True


def column_of_inverse_root(S: np.ndarray, c: int, p: int):
    """Column c of S^(-1/p); (x, ok)."""
    return column_of_function(S, c, "inv_root", p)


# ---------------------------------------------------------------------------
# Sections 3.3/3.4: assembly into A's pattern


def forward_columns(rowptr, colind, vals, p, cols, fn: str = "inv_root"):
    """Segments of X = f(A) for the given columns: {j: x_j}; and the count
    of submatrices that were not positive definite. `p` is the function's
    parameter (p for the roots, alpha for the power)."""
    check_function(fn, p)
    out = {}
    bad = 0
    for j in cols:
        R = submatrix_rows(rowptr, colind, int(j))
        c = int(np.nonzero(R == j)[0][0])
        S, _ = gather_submatrix(rowptr, colind, vals, R)
        x, ok = column_of_function(symmetrise(S), c, fn, p)
        bad += 0 if ok else 1
        out[int(j)] = x
    return out, bad


def forward(rowptr, colind, vals, n: int, p, check: bool = True, fn: str = "inv_root"):
    """X.vals on A's pattern (X.rowptr, X.colind are A's), and the number of
    non-positive-definite submatrices."""
    check_function(fn, p)
    if check:
        validate(rowptr, colind, n)
    x = np.empty(len(colind), dtype=np.float64)
    segs, bad = forward_columns(rowptr, colind, vals, p, range(n), fn)
    for j, xj in segs.items():
        x[rowptr[j]:rowptr[j + 1]] = xj
    return x, bad


# ---------------------------------------------------------------------------
# Adjoint (Daleckii-Krein); the paper has no gradient


def divided_differences(lam: np.ndarray, p, fn: str = "inv_root") -> np.ndarray:
    """G[k,l] = (f(l_k) - f(l_l)) / (l_k - l_l), f'(l_k) where l_k == l_l.

    Written so that no digits cancel:
    * inv_root, f = x^(-1/p): with a = lambda^(1/p),
      f(l_k) - f(l_l) = (a_l - a_k) / (a_k a_l) and
      l_k - l_l = a_k^p - a_l^p = (a_k - a_l) s, s = sum_{i<p} a_k^i a_l^(p-1-i),
      so G = -1 / (a_k a_l s) (also the derivative when a_k == a_l);
    * root, f = x^(1/p): G = (a_k - a_l) / (a_k^p - a_l^p) = 1 / s;
    * power, f = x^alpha: with t = log(l_k / l_l), l_k^alpha =
      l_l^alpha exp(alpha t), so f(l_k) - f(l_l) = l_l^alpha expm1(alpha t),
      and on the diagonal G = alpha l^(alpha - 1). t is formed as log1p(d),
      d = (l_k - l_l) / l_l, when |d| < 1/2 (the difference is exact there,
      and log1p keeps a small t to full relative accuracy), else as the log
      of the ratio (a rounding of the ratio then moves t by about one ulp of
      1, small against |t| > 0.4, where log1p of a d near -1 would not be)."""
    if fn == "power":
        alpha = float(p)
        lk = lam[:, None] + np.zeros((1, lam.shape[0]))
        ll = lam[None, :] + np.zeros((lam.shape[0], 1))
        diff = lk - ll
        G = np.empty_like(diff)
        same = diff == 0.0
        G[same] = alpha * np.power(ll[same], alpha - 1.0)
        o = ~same
        d = diff[o] / ll[o]
        t = np.where(np.abs(d) < 0.5, np.log1p(d), np.log(lk[o] / ll[o]))
        G[o] = np.power(ll[o], alpha) * np.expm1(alpha * t) / diff[o]
        return G
    p = int(p)
    a = root(lam, p)
    ak = a[:, None]
    al = a[None, :]
    s = np.zeros((a.shape[0], a.shape[0]))
    for i in range(p):
        s += ak ** i * al ** (p - 1 - i)
    if fn == "root":
        return 1.0 / s
    return -1.0 / (ak * al * s)


def adjoint_column(S: np.ndarray, c: int, w: np.ndarray, p, fn: str = "inv_root"):
    """dL/dS for L = w . (column c of f(S)), on the symmetric part of S."""
    lam, Q = eig(S)
    if lam.min() <= 0.0:
        return np.full(S.shape, np.nan)
    a = Q.T @ w
    b = Q[c, :]
    M = divided_differences(lam, p, fn) * np.outer(a, b)
    return Q @ (0.5 * (M + M.T)) @ Q.T


def adjoint(rowptr, colind, vals, n: int, p, wvals, cols=None, check: bool = True, fn: str = "inv_root"):
    """dL/dA.vals for L = sum(W.vals * X.vals), X = forward(A): every stored
    pair (R_j[k], R_j[l]) of every submatrix receives D_j[k, l]."""
    check_function(fn, p)
    if check:
        validate(rowptr, colind, n)
    dA = np.zeros(len(colind), dtype=np.float64)
    wvals = np.asarray(wvals, dtype=np.float64)
    for j in (range(n) if cols is None else cols):
        j = int(j)
        R = submatrix_rows(rowptr, colind, j)
        c = int(np.nonzero(R == j)[0][0])
        S, pos = gather_submatrix(rowptr, colind, vals, R)
        D = adjoint_column(symmetrise(S), c, wvals[rowptr[j]:rowptr[j + 1]], p, fn)
        mask = pos >= 0
        np.add.at(dA, pos[mask], D[mask])
    return dA


# ---------------------------------------------------------------------------
# Section 4.1 error metric (dense; small n only)


def residual_norm(xvals, rowptr, colind, avals, n: int, p: int) -> float:
    """Spectral norm of X^p A - I with X the column-based result (the CSR
    value segment j holds column j of X)."""
    X = np.zeros((n, n))
    A = np.zeros((n, n))
    for j in range(n):
        seg = slice(rowptr[j], rowptr[j + 1])
        X[np.asarray(colind[seg]), j] = xvals[seg]
        A[j, np.asarray(colind[seg])] = avals[seg]
    R = np.linalg.matrix_power(X, p) @ A - np.eye(n)
    return float(np.linalg.norm(R, 2))
