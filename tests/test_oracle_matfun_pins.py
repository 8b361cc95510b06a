"""Pins of the oracle's other spectral functions: positive p-th roots
lambda^(1/p) (Section 4, "Applicability to other matrix operations") and
real powers lambda^alpha.

Each expected value comes from a route independent of the oracle's
eigendecomposition formula: a structural identity of the method (alpha = 1
returns A; alpha = 2 returns A^2 on A's pattern), a different
matrix-function algorithm (Schur-based square root, Schur-Pade fractional
power), an invariant (X^p = A where the method is exact), 50-digit
evaluation of the plain definition of a divided difference, a closed form or
a Sylvester equation for the gradient, and finite differences.
"""
import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from workloads import generators as G


def rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def dense_X_from_vals(csr, xvals):
    """Column-based X: CSR value segment j is column j (Section 3.3)."""
    X = np.zeros((csr.n, csr.n))
    for j in range(csr.n):
        seg = slice(csr.rowptr[j], csr.rowptr[j + 1])
        X[csr.colind[seg], j] = xvals[seg]
    return X


def fwd(csr, fn, param):
    x, bad = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, param, fn=fn)
    assert bad == 0
    return x


# ---------------------------------------------------------------------------
# Forward


def test_power_one_reproduces_A():
    """f(S) = S, so column c of f(S_j) is A's column j on R_j: X = A."""
    for csr in (G.random_sparse_spd(80, 0.08, kappa=20.0), G.banded_spd(60, 4),
                G.block_diagonal_spd((1, 5, 17), permute=True)):
        x = fwd(csr, "power", 1.0)
        assert rel_fro(x, csr.vals) <= 1e-13


def test_power_two_is_A_squared_on_the_pattern():
    """Column c of S_j^2 at row k is sum_{l in R_j} A[R_k][l] A[l][j]; since
    A[l][j] is zero for every l outside R_j, that is (A^2)[R_k][j] exactly:
    the method returns A^2 sampled on A's pattern (a sparse product, no
    eigendecomposition)."""
    csr = G.random_sparse_spd(90, 0.07, kappa=30.0)
    A = csr.to_scipy()
    A2 = (A @ A).tocsr()
    rows = np.repeat(np.arange(csr.n), csr.row_sizes())
    ref = np.asarray(A2[csr.colind, rows]).ravel()  # column-based: segment j = column j
    x = fwd(csr, "power", 2.0)
    assert rel_fro(x, ref) <= 1e-13


def test_root2_of_dense_matrix_is_sqrtm():
    """Full pattern: every S_j is A itself, so X = A^(1/2) exactly; compared
    with the Schur-based square root."""
    csr = G.dense_spd(40, kappa=50.0)
    X = dense_X_from_vals(csr, fwd(csr, "root", 2))
    ref = np.real(sla.sqrtm(csr.dense()))
    assert rel_fro(X, ref) <= 1e-12


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("permute", [False, True])
def test_block_diagonal_root_powers_back_to_A(p, permute):
    """Block-diagonal pattern: the method is exact, so X^p = A and X is
    symmetric."""
    csr = G.block_diagonal_spd((1, 6, 14, 30), kappa=40.0, permute=permute)
    X = dense_X_from_vals(csr, fwd(csr, "root", p))
    assert rel_fro(X, X.T) <= 1e-14
    assert rel_fro(np.linalg.matrix_power(X, p), csr.dense()) <= 1e-12


@pytest.mark.parametrize("alpha", [0.3, -1.7, 2.5])
def test_dense_real_power_matches_schur_pade(alpha):
    """Full pattern: X = A^alpha, compared with the Schur-Pade fractional
    matrix power."""
    csr = G.dense_spd(36, kappa=20.0)
    X = dense_X_from_vals(csr, fwd(csr, "power", alpha))
    ref = np.real(sla.fractional_matrix_power(csr.dense(), alpha))
    assert rel_fro(X, ref) <= 1e-11


@pytest.mark.parametrize("alpha", [-2.0, -0.5, 0.25, 3.0])
def test_diagonal_power_is_elementwise(alpha):
    csr = G.diagonal_spd(40)
    x = fwd(csr, "power", alpha)
    ref = np.array([float(mpmath.mpf(v) ** mpmath.mpf(alpha)) for v in csr.vals])
    assert np.max(np.abs(x - ref) / np.abs(ref)) <= 4e-16


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_power_family_agrees_with_roots(p):
    """lambda^(1/p) and lambda^(-1/p) through the power branch (np.power)
    and through the root branches (sqrt/cbrt/reciprocal)."""
    csr = G.random_sparse_spd(60, 0.1, kappa=25.0)
    assert rel_fro(fwd(csr, "power", 1.0 / p), fwd(csr, "root", p)) <= 1e-14
    assert rel_fro(fwd(csr, "power", -1.0 / p), fwd(csr, "inv_root", p)) <= 1e-14


def test_power_zero_gives_identity_columns():
    csr = G.random_sparse_spd(40, 0.1, kappa=10.0)
    x = fwd(csr, "power", 0.0)
    rows = np.repeat(np.arange(csr.n), csr.row_sizes())
    ref = (rows == csr.colind).astype(float)
    assert np.max(np.abs(x - ref)) <= 1e-14


def test_rejects_bad_function_parameters():
    csr = G.diagonal_spd(4)
    for fn, param in (("root", 0), ("root", 2.5), ("inv_root", -1), ("power", np.inf), ("power", np.nan),
                      ("sqrt", 2)):
        with pytest.raises(oracle.PatternError) as e:
            oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, param, fn=fn)
        assert e.value.code == "EINVAL"


# ---------------------------------------------------------------------------
# Divided differences and adjoint


def _dd_exact(lk, ll, fn, param):
    """(f(l_k) - f(l_l)) / (l_k - l_l), f'(l) when equal, at 50 digits."""
    with mpmath.workdps(50):
        if fn == "power":
            e = mpmath.mpf(param)
        else:
            e = (1 if fn == "root" else -1) / mpmath.mpf(int(param))
        a, b = mpmath.mpf(lk), mpmath.mpf(ll)
        if a == b:
            return float(e * a ** (e - 1))
        return float((a ** e - b ** e) / (a - b))


@pytest.mark.parametrize("fn,param", [("root", 1), ("root", 2), ("root", 3), ("root", 5),
                                      ("power", 0.7), ("power", -1.3), ("power", 2.0), ("power", 1.0 / 3.0),
                                      ("power", -0.5)])
def test_divided_differences_high_precision(fn, param):
    """The oracle's cancellation-free forms against the plain definition in
    50-digit arithmetic, on eigenvalues that include equal, nearly equal
    (relative gaps 1e-14 and 1e-9) and widely spread (ratio 1e6) pairs."""
    lam = np.array([1e-3, 0.37, 1.0, 1.0 + 1e-14, 1.0 + 1e-9, 2.5, 2.5, 40.0, 1e3])
    Gm = oracle.divided_differences(lam, param, fn)
    for k in range(lam.size):
        for l in range(lam.size):
            ref = _dd_exact(lam[k], lam[l], fn, param)
            assert abs(Gm[k, l] - ref) <= 2e-14 * abs(ref), (k, l, Gm[k, l], ref)


def test_adjoint_power_one_is_symmetrised_upstream():
    """For alpha = 1, X = A (as a function of the symmetric part of each
    S_j): D_j = (w e_c^T + e_c w^T) / 2, so the stored entry (r, s) receives
    half of the upstream value at (r, s) and half of the one at (s, r)."""
    csr = G.random_sparse_spd(60, 0.1, kappa=20.0)
    w = G.upstream_gradient(csr, 21)
    dA = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 1.0, w, fn="power")
    W = csr.to_scipy().copy()
    W.data = w.copy()
    Wt = W.T.tocsr()
    Wt.sort_indices()
    ref = 0.5 * (w + Wt.data)
    assert rel_fro(dA, ref) <= 1e-13


def _sym(M):
    return 0.5 * (M + M.T)


def test_adjoint_root2_sylvester():
    """L = w^T Y e_c with Y = S^(1/2): dL/dY = w e_c^T, and dL/dS (symmetric
    part) solves Y Z + Z Y = dL/dY."""
    csr = G.random_sparse_spd(50, 0.12, kappa=15.0)
    w = G.upstream_gradient(csr, 22)
    A = csr.dense()
    for j in range(0, csr.n, 5):
        R = csr.colind[csr.rowptr[j]:csr.rowptr[j + 1]]
        S = A[np.ix_(R, R)]
        Y = np.real(sla.sqrtm(S))
        e = (R == j).astype(float)
        wj = w[csr.rowptr[j]:csr.rowptr[j + 1]]
        Z = _sym(sla.solve_sylvester(Y, Y, np.outer(wj, e)))
        Dj = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, w, cols=[j], check=False, fn="root")
        _, pos = oracle.gather_submatrix(csr.rowptr, csr.colind, csr.vals, R)
        mask = pos >= 0
        got = np.zeros_like(Z)
        got[mask] = Dj[pos[mask]]
        assert rel_fro(got[mask], Z[mask]) <= 1e-11


def _affected_columns(csr, q):
    rows = np.repeat(np.arange(csr.n), csr.row_sizes())
    i, k = rows[q], csr.colind[q]
    ri = csr.colind[csr.rowptr[i]:csr.rowptr[i + 1]]
    rk = csr.colind[csr.rowptr[k]:csr.rowptr[k + 1]]
    return np.intersect1d(ri, rk)


def _loss_on(csr, vals, w, fn, param, cols):
    segs, _ = oracle.forward_columns(csr.rowptr, csr.colind, vals, param, cols, fn)
    return sum(float(np.dot(w[csr.rowptr[j]:csr.rowptr[j + 1]], segs[j])) for j in cols)


@pytest.mark.parametrize("fn,param", [("root", 2), ("root", 3), ("power", 0.7), ("power", -1.3)])
def test_matfun_adjoint_central_finite_differences(fn, param):
    csr = G.random_sparse_spd(60, 0.09, kappa=20.0)
    w = G.upstream_gradient(csr, 23)
    dA = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, param, w, fn=fn)
    rng = np.random.default_rng(G.BASE_SEED + 210)
    h = 1e-6
    for q in rng.choice(csr.nnz, size=30, replace=False):
        cols = _affected_columns(csr, q)
        vp = csr.vals.copy()
        vm = csr.vals.copy()
        vp[q] += h
        vm[q] -= h
        fd = (_loss_on(csr, vp, w, fn, param, cols) - _loss_on(csr, vm, w, fn, param, cols)) / (2 * h)
        assert abs(fd - dA[q]) <= 1e-6 * max(1.0, abs(dA[q])), (q, fd, dA[q])
