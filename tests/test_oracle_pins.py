"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each expected value comes
from an independent route (closed forms, exact rational arithmetic, a
different matrix-function algorithm, the dense transcription of Algorithms
1 and 2, finite differences, invariants).
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from workloads import generators as G


def rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def dense_of(csr):
    return csr.dense()


def dense_X_from_vals(csr, xvals):
    """Column-based X: CSR value segment j is column j (Section 3.3)."""
    X = np.zeros((csr.n, csr.n))
    for j in range(csr.n):
        seg = slice(csr.rowptr[j], csr.rowptr[j + 1])
        X[csr.colind[seg], j] = xvals[seg]
    return X


def run(csr, p):
    x, bad = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, p)
    return x, bad


def literal_dense_method(A, p, fn):
    """Algorithms 1 and 2 transcribed on a dense matrix: R = nonzero rows of
    column j, S = A[R][R], X[R[i]][j] = fn(S)[i][R.indexof(j)]."""
    n = A.shape[0]
    X = np.zeros_like(A)
    for j in range(n):
        R = [i for i in range(n) if A[i][j] != 0]
        S = np.array([[A[r][s] for s in R] for r in R])
        F = fn(S, p)
        c = R.index(j)
        for i, r in enumerate(R):
            X[r][j] = F[i][c]
    return X


def frac_power_schur(S, p):
    """S^(-1/p) by the Schur-Pade algorithm (Higham-Lin), not eigh."""
    return np.real(sla.fractional_matrix_power(S, -1.0 / p))


# ---------------------------------------------------------------------------
# Whole forward on the cases the method gets exactly


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_diagonal_is_elementwise_root_within_ulps(p):
    csr = G.diagonal_spd(200)
    x, bad = run(csr, p)
    assert bad == 0
    mpmath.mp.prec = 200
    ref = np.array([float(mpmath.mpf(float(a)) ** (-mpmath.mpf(1) / p)) for a in csr.vals])
    ulps = np.abs(x - ref) / np.spacing(ref)
    assert ulps.max() <= (1.0 if p <= 2 else 2.0), ulps.max()


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("permute", [False, True])
def test_block_diagonal_is_exact_inverse_root(p, permute):
    csr = G.block_diagonal_spd((1, 7, 13, 64, 100), permute=permute)
    x, bad = run(csr, p)
    assert bad == 0
    X = dense_X_from_vals(csr, x)
    A = dense_of(csr)
    # every S_j is its whole block, so X = A^(-1/p) exactly (block by block)
    ref = frac_power_schur(A, p)
    ref[A == 0] = 0.0
    assert rel_fro(X, ref) <= 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_dense_matrix_gives_exact_inverse_root(p):
    csr = G.dense_spd(48)
    x, _ = run(csr, p)
    X = dense_X_from_vals(csr, x)
    A = dense_of(csr)
    if p == 1:
        ref = np.linalg.inv(A)
    elif p == 2:
        ref = np.linalg.inv(np.real(sla.sqrtm(A)))
    else:
        ref = frac_power_schur(A, p)
    assert rel_fro(X, ref) <= 1e-12
    assert rel_fro(X, X.T) <= 1e-12


def test_p1_columns_are_cholesky_solves():
    csr = G.random_sparse_spd(150, 0.06, kappa=30.0)
    x, _ = run(csr, 1)
    A = dense_of(csr)
    for j in range(csr.n):
        R = np.nonzero(A[:, j])[0]
        R = csr.colind[csr.rowptr[j]:csr.rowptr[j + 1]]  # stored pattern
        S = A[np.ix_(R, R)]
        e = (R == j).astype(float)
        ref = sla.cho_solve(sla.cho_factor(S), e)
        seg = x[csr.rowptr[j]:csr.rowptr[j + 1]]
        assert rel_fro(seg, ref) <= 1e-12


def test_p2_columns_are_sqrtm_solves():
    csr = G.random_sparse_spd(120, 0.08, kappa=30.0)
    x, _ = run(csr, 2)
    A = dense_of(csr)
    for j in range(csr.n):
        R = csr.colind[csr.rowptr[j]:csr.rowptr[j + 1]]
        S = A[np.ix_(R, R)]
        e = (R == j).astype(float)
        ref = np.linalg.solve(np.real(sla.sqrtm(S)), e)
        seg = x[csr.rowptr[j]:csr.rowptr[j + 1]]
        assert rel_fro(seg, ref) <= 1e-11


@pytest.mark.parametrize("p", [1, 2, 3])
def test_literal_dense_algorithms_match(p):
    """The dense, loop-by-loop reading of Algorithms 1 and 2 with a
    Schur-Pade matrix function gives the same X."""
    csr = G.banded_spd(40, 3)
    x, _ = run(csr, p)
    X = dense_X_from_vals(csr, x)
    ref = literal_dense_method(dense_of(csr), p, frac_power_schur)
    assert rel_fro(X, ref) <= 1e-12


def test_arrowhead_two_by_two_closed_form():
    """Submatrices j >= 1 of an arrowhead are 2x2: [[a00, a0j], [a0j, ajj]].
    S^(-1/2) of a 2x2 SPD matrix: S^(1/2) = (S + sqrt(det) I)/sqrt(tr + 2 sqrt(det))."""
    csr = G.arrowhead_spd(40)
    x, bad = run(csr, 2)
    assert bad == 0
    A = dense_of(csr)
    for j in range(1, csr.n):
        S = np.array([[A[0, 0], A[0, j]], [A[j, 0], A[j, j]]])
        sd = np.sqrt(np.linalg.det(S))
        half = (S + sd * np.eye(2)) / np.sqrt(np.trace(S) + 2 * sd)
        ref = np.linalg.inv(half)[:, 1]
        seg = x[csr.rowptr[j]:csr.rowptr[j + 1]]  # rows (0, j)
        assert rel_fro(seg, ref) <= 1e-14


def _exact_solve(S, e):
    n = len(S)
    M = [[Fraction(S[i][k]) for k in range(n)] + [Fraction(e[i])] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def test_p1_exact_rational_brute_force():
    """Integer matrix, p = 1: every column of the submatrix inverse in exact
    rational arithmetic (Algorithms 1 and 2 on the dense matrix)."""
    n = 8
    A = np.zeros((n, n), dtype=np.int64)
    rng = np.random.default_rng(3)
    for i in range(n):
        for d in (1, 2):
            if i + d < n and rng.random() < 0.8:
                A[i, i + d] = A[i + d, i] = int(rng.integers(-3, 4)) or 1
    for i in range(n):
        A[i, i] = 1 + np.abs(A[i]).sum()
    r, c = np.nonzero(A)
    from workloads.generators import _from_coo
    csr = _from_coo(r, c, A[r, c].astype(float), n)
    x, _ = run(csr, 1)
    for j in range(n):
        R = [i for i in range(n) if A[i][j] != 0]
        S = [[int(A[a][b]) for b in R] for a in R]
        ex = _exact_solve(S, [1 if i == j else 0 for i in R])
        seg = x[csr.rowptr[j]:csr.rowptr[j + 1]]
        for got, want in zip(seg, ex):
            assert abs(got - float(want)) <= 4e-16 * max(1.0, abs(float(want)))


def test_pattern_and_inputs_unchanged():
    csr = G.banded_spd(64, 4)
    rp, ci, va = csr.rowptr.copy(), csr.colind.copy(), csr.vals.copy()
    x, _ = run(csr, 2)
    assert x.shape == csr.vals.shape
    assert np.array_equal(rp, csr.rowptr) and np.array_equal(ci, csr.colind)
    assert np.array_equal(va, csr.vals)
    assert np.all(np.isfinite(x))


def test_explicit_zeros_stay_in_pattern():
    csr = G.explicit_zero_pattern()
    assert np.any(csr.vals == 0.0)
    x, _ = run(csr, 2)
    # the stored-pattern submatrix differs from the numeric-nonzero one
    A = dense_of(csr)
    ref = literal_dense_method(A, 2, frac_power_schur)
    X = dense_X_from_vals(csr, x)
    assert np.all(np.isfinite(x))
    assert rel_fro(X, ref) > 1e-8  # numeric-pattern reading differs
    # and agrees with a stored-pattern dense transcription
    Xs = np.zeros_like(A)
    for j in range(csr.n):
        R = list(csr.colind[csr.rowptr[j]:csr.rowptr[j + 1]])
        S = A[np.ix_(R, R)]
        F = frac_power_schur(S, 2)
        for i, r in enumerate(R):
            Xs[r, j] = F[i, R.index(j)]
    assert rel_fro(X, Xs) <= 1e-12


# ---------------------------------------------------------------------------
# Invariants


def test_permutation_equivariance():
    csr = G.random_sparse_spd(90, 0.08, kappa=20.0)
    x, _ = run(csr, 2)
    X = dense_X_from_vals(csr, x)
    A = dense_of(csr)
    perm = np.random.default_rng(5).permutation(csr.n)
    P = np.eye(csr.n)[perm]
    Ap = P @ A @ P.T
    r, c = np.nonzero(Ap)
    from workloads.generators import _from_coo
    cp = _from_coo(r, c, Ap[r, c], csr.n)
    xp, _ = run(cp, 2)
    Xp = dense_X_from_vals(cp, xp)
    assert rel_fro(Xp, P @ X @ P.T) <= 1e-13


@pytest.mark.parametrize("p,k", [(1, 3), (2, 2), (3, 1)])
def test_scaling_law(p, k):
    csr = G.banded_spd(50, 4)
    x, _ = run(csr, p)
    scaled = G.CSR(csr.rowptr, csr.colind, csr.vals * 2.0 ** (p * k), csr.n)
    xs, _ = run(scaled, p)
    assert np.max(np.abs(xs - x * 2.0 ** (-k))) <= 1e-14 * np.max(np.abs(x))


def test_atoms_share_submatrix():
    csr = G.overlap_matrix(n_atoms=24, density=0.1, nbf=4, rcut=3.0, kappa=20.0)
    x, _ = run(csr, 2)
    A = dense_of(csr)
    atom = 5
    cols = list(range(atom * 4, atom * 4 + 4))
    R = csr.colind[csr.rowptr[cols[0]]:csr.rowptr[cols[0] + 1]]
    F = np.real(sla.fractional_matrix_power(A[np.ix_(R, R)], -0.5))
    for j in cols:
        assert np.array_equal(csr.colind[csr.rowptr[j]:csr.rowptr[j + 1]], R)
        seg = x[csr.rowptr[j]:csr.rowptr[j + 1]]
        assert rel_fro(seg, F[:, list(R).index(j)]) <= 1e-12


def test_submatrix_spectra_interlace():
    csr = G.random_sparse_spd(100, 0.06, kappa=40.0)
    lmin, lmax = csr.meta["lmin"], csr.meta["lmax"]
    for j in range(0, csr.n, 7):
        R = oracle.submatrix_rows(csr.rowptr, csr.colind, j)
        S, _ = oracle.gather_submatrix(csr.rowptr, csr.colind, csr.vals, R)
        w = np.linalg.eigvalsh(S)
        assert w[0] >= lmin * (1 - 1e-10) and w[-1] <= lmax * (1 + 1e-10)


def test_residual_metric_block_diagonal_is_rounding():
    csr = G.block_diagonal_spd((3, 5, 8, 20))
    for p in (1, 2, 3):
        x, _ = run(csr, p)
        assert oracle.residual_norm(x, csr.rowptr, csr.colind, csr.vals, csr.n, p) < 1e-12


def test_residual_metric_small_for_well_conditioned():
    csr = G.banded_spd(60, 3)
    x, _ = run(csr, 1)
    r = oracle.residual_norm(x, csr.rowptr, csr.colind, csr.vals, csr.n, 1)
    assert 1e-6 < r < 0.5  # an approximation, and a useful one (Section 4.1)


# ---------------------------------------------------------------------------
# Error behaviour


def test_rejects_missing_diagonal():
    rowptr = np.array([0, 1, 2, 3], dtype=np.int32)
    colind = np.array([0, 2, 1], dtype=np.int32)
    with pytest.raises(oracle.PatternError) as e:
        oracle.forward(rowptr, colind, np.ones(3), 3, 2)
    assert e.value.code in ("ENODIAG", "EPATTERN")


def test_rejects_unsorted_and_asymmetric():
    rowptr = np.array([0, 2, 3], dtype=np.int32)
    with pytest.raises(oracle.PatternError):
        oracle.validate(rowptr, np.array([1, 0, 1], dtype=np.int32), 2)
    with pytest.raises(oracle.PatternError) as e:
        oracle.validate(rowptr, np.array([0, 1, 1], dtype=np.int32), 2)
    assert e.value.code == "EPATTERN"
    with pytest.raises(oracle.PatternError) as e:
        oracle.forward(np.array([0, 1, 2]), np.array([0, 1]), np.ones(2), 2, 0)
    assert e.value.code == "EINVAL"


def test_non_spd_submatrix_gives_nan_and_count():
    csr = G.banded_spd(30, 2)
    vals = csr.vals.copy()
    d5 = csr.rowptr[5] + np.searchsorted(csr.colind[csr.rowptr[5]:csr.rowptr[6]], 5)
    vals[d5] = -3.0
    x, bad = oracle.forward(csr.rowptr, csr.colind, vals, csr.n, 2)
    assert bad >= 1
    assert np.all(np.isnan(x[csr.rowptr[5]:csr.rowptr[6]]))
    assert np.isfinite(x[csr.rowptr[20]:csr.rowptr[21]]).all()


# ---------------------------------------------------------------------------
# Adjoint


@pytest.mark.parametrize("p", [1, 2, 3])
def test_divided_differences_match_definition(p):
    lam = np.array([0.5, 1.3, 2.0, 7.5, 11.0])
    Gm = oracle.divided_differences(lam, p)
    f = lam ** (-1.0 / p)
    for k in range(5):
        for l in range(5):
            if k != l:
                ref = (f[k] - f[l]) / (lam[k] - lam[l])
            else:
                ref = -(1.0 / p) * lam[k] ** (-1.0 / p - 1.0)
            assert abs(Gm[k, l] - ref) <= 1e-13 * abs(ref)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_adjoint_diagonal_closed_form(p):
    csr = G.diagonal_spd(50)
    w = G.upstream_gradient(csr, 7)
    dA = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, p, w)
    ref = w * (-(1.0 / p)) * csr.vals ** (-1.0 / p - 1.0)
    assert np.max(np.abs(dA - ref) / np.abs(ref)) <= 1e-13


def _sym(M):
    return 0.5 * (M + M.T)


def test_adjoint_p1_closed_form():
    csr = G.random_sparse_spd(60, 0.1, kappa=20.0)
    w = G.upstream_gradient(csr, 8)
    A = dense_of(csr)
    ref = np.zeros(csr.nnz)
    for j in range(csr.n):
        R = csr.colind[csr.rowptr[j]:csr.rowptr[j + 1]]
        S = A[np.ix_(R, R)]
        cf = sla.cho_factor(S)
        u = sla.cho_solve(cf, w[csr.rowptr[j]:csr.rowptr[j + 1]])
        v = sla.cho_solve(cf, (R == j).astype(float))
        D = -_sym(np.outer(u, v))
        for k, r in enumerate(R):
            for l, s in enumerate(R):
                a, b = csr.rowptr[r], csr.rowptr[r + 1]
                q = a + np.searchsorted(csr.colind[a:b], s)
                if q < b and csr.colind[q] == s:
                    ref[q] += D[k, l]
    dA = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 1, w)
    assert rel_fro(dA, ref) <= 1e-12


def test_adjoint_p2_sylvester():
    """L = w^T S^(-1/2) e_c; with Y = S^(1/2), X = Y^(-1):
    dL/dY = -X w e_c^T X and dL/dS solves Y Z + Z Y = dL/dY."""
    csr = G.random_sparse_spd(50, 0.12, kappa=15.0)
    w = G.upstream_gradient(csr, 9)
    A = dense_of(csr)
    dA = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, w)
    for j in range(0, csr.n, 5):
        R = csr.colind[csr.rowptr[j]:csr.rowptr[j + 1]]
        S = A[np.ix_(R, R)]
        Y = np.real(sla.sqrtm(S))
        X = np.linalg.inv(Y)
        e = (R == j).astype(float)
        wj = w[csr.rowptr[j]:csr.rowptr[j + 1]]
        Ybar = -X @ np.outer(wj, e) @ X
        Z = _sym(sla.solve_sylvester(Y, Y, Ybar))
        Dj = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, w, cols=[j], check=False)
        S_, pos = oracle.gather_submatrix(csr.rowptr, csr.colind, csr.vals, R)
        got = np.zeros_like(Z)
        mask = pos >= 0
        got[mask] = Dj[pos[mask]]
        # on the stored pairs of this submatrix
        assert rel_fro(got[mask], Z[mask]) <= 1e-11


def _affected_columns(csr, q):
    rows = np.repeat(np.arange(csr.n), csr.row_sizes())
    i, k = rows[q], csr.colind[q]
    ri = csr.colind[csr.rowptr[i]:csr.rowptr[i + 1]]
    rk = csr.colind[csr.rowptr[k]:csr.rowptr[k + 1]]
    return np.intersect1d(ri, rk)


def _loss_on(csr, vals, w, p, cols):
    segs, _ = oracle.forward_columns(csr.rowptr, csr.colind, vals, p, cols)
    return sum(float(np.dot(w[csr.rowptr[j]:csr.rowptr[j + 1]], segs[j])) for j in cols)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_adjoint_central_finite_differences(p):
    csr = G.random_sparse_spd(70, 0.08, kappa=20.0)
    w = G.upstream_gradient(csr, 10)
    dA = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, p, w)
    rng = np.random.default_rng(G.BASE_SEED + 200)
    h = 1e-6
    for q in rng.choice(csr.nnz, size=40, replace=False):
        cols = _affected_columns(csr, q)
        vp = csr.vals.copy()
        vm = csr.vals.copy()
        vp[q] += h
        vm[q] -= h
        fd = (_loss_on(csr, vp, w, p, cols) - _loss_on(csr, vm, w, p, cols)) / (2 * h)
        assert abs(fd - dA[q]) <= 1e-6 * max(1.0, abs(dA[q])), (q, fd, dA[q])


def test_adjoint_random_symmetric_directions():
    csr = G.banded_spd(40, 3)
    w = G.upstream_gradient(csr, 11)
    p = 2
    dA = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, p, w)
    rng = np.random.default_rng(G.BASE_SEED + 201)
    rows = np.repeat(np.arange(csr.n), csr.row_sizes())
    h = 1e-6
    for _ in range(8):
        dirn = rng.standard_normal(csr.nnz)
        # symmetric direction: equal value at (i,k) and (k,i)
        A = csr.to_scipy().copy()
        A.data = dirn
        Asym = (A + A.T) * 0.5
        Asym = Asym.tocsr()
        Asym.sort_indices()
        dsym = np.asarray(Asym[rows, csr.colind]).ravel()
        allc = range(csr.n)
        fd = (_loss_on(csr, csr.vals + h * dsym, w, p, allc)
              - _loss_on(csr, csr.vals - h * dsym, w, p, allc)) / (2 * h)
        assert abs(fd - np.dot(dA, dsym)) <= 1e-6 * max(1.0, abs(fd))


def test_adjoint_symmetry_and_linearity():
    csr = G.random_sparse_spd(60, 0.1, kappa=20.0)
    w1 = G.upstream_gradient(csr, 12)
    w2 = G.upstream_gradient(csr, 13)
    d1 = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, w1)
    d2 = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, w2)
    d12 = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, 2.0 * w1 - w2)
    assert rel_fro(d12, 2.0 * d1 - d2) <= 1e-12
    M = csr.to_scipy().copy()
    M.data = d1
    assert abs(M - M.T).max() <= 1e-12 * np.abs(d1).max()


def test_adjoint_block_diagonal_equals_full_block_frechet():
    """Each S_j is its whole block B, so dA restricted to B is the adjoint of
    B -> B^(-1/2) applied to the block of W read column-wise; checked by
    finite differences on the whole block function."""
    csr = G.block_diagonal_spd((4, 9))
    w = G.upstream_gradient(csr, 14)
    dA = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, w)
    A = dense_of(csr)
    Wd = dense_X_from_vals(csr, w)
    B = A[4:13, 4:13]
    WB = Wd[4:13, 4:13]
    h = 1e-6
    got = dense_X_from_vals(csr, dA)[4:13, 4:13].T  # stored (row, col) entries
    for (k, l) in [(0, 0), (2, 5), (8, 1), (4, 4)]:
        E = np.zeros_like(B)
        E[k, l] = 1.0
        E = _sym(E)  # the method sees the symmetric part
        fp = np.sum(WB * frac_power_schur(B + h * E, 2))
        fm = np.sum(WB * frac_power_schur(B - h * E, 2))
        fd = (fp - fm) / (2 * h)
        assert abs(fd - got[k, l]) <= 1e-7 * max(1.0, abs(fd))
