"""Pins of the oracle's residual metric (Section 4.1) and conjugate
gradients (Section 4.4) against routes independent of their code: the
dense definition of the spectral norm (SVD), diagonal closed forms, scipy's
own CG, CG's finite termination on k distinct eigenvalues, and exact
preconditioners."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle import krylov_oracle as ko
from workloads import generators as G


# ---------------------------------------------------------------------------
# Residual metric


@pytest.mark.parametrize("p", [1, 2, 3])
def test_sparse_residual_norm_equals_dense_definition(p):
    """ARPACK on the operator R against the SVD of the dense X^p A - I."""
    csr = G.random_sparse_spd(160, 0.05, kappa=20.0)
    x, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, p)
    dense = oracle.residual_norm(x, csr.rowptr, csr.colind, csr.vals, csr.n, p)
    sparse = ko.residual_norm_sparse(x, csr.rowptr, csr.colind, csr.vals, csr.n, p)
    assert dense > 1e-6
    assert abs(sparse - dense) <= 1e-10 * dense


@pytest.mark.parametrize("p", [1, 2, 3])
def test_residual_norm_diagonal_closed_form(p):
    """A = diag(a), X = diag(x): R = diag(x_i^p a_i - 1), so ||R||_2 =
    max_i |x_i^p a_i - 1|; X is a perturbed inverse root."""
    csr = G.diagonal_spd(60)
    rng = np.random.default_rng(5)
    x = csr.vals ** (-1.0 / p) * (1.0 + 1e-3 * rng.standard_normal(csr.n))
    ref = np.max(np.abs(x ** p * csr.vals - 1.0))
    got = ko.residual_norm_sparse(x, csr.rowptr, csr.colind, csr.vals, csr.n, p)
    assert abs(got - ref) <= 1e-12 * ref


def test_residual_norm_of_exact_result_is_rounding():
    csr = G.block_diagonal_spd((3, 9, 20), kappa=10.0)
    x, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, 2)
    assert ko.residual_norm_sparse(x, csr.rowptr, csr.colind, csr.vals, csr.n, 2) <= 1e-12


def test_residual_operator_transpose_is_adjoint():
    """<R u, v> = <u, R^T v> for random u, v (the rmatvec ARPACK needs)."""
    csr = G.random_sparse_spd(80, 0.08, kappa=15.0)
    x, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, 3)
    R = ko.residual_operator(x, csr.rowptr, csr.colind, csr.vals, csr.n, 3)
    rng = np.random.default_rng(6)
    u, v = rng.standard_normal(csr.n), rng.standard_normal(csr.n)
    lhs, rhs = float((R @ u) @ v), float(u @ R.rmatvec(v))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_column_based_matrix_reads_segments_as_columns():
    csr = G.random_sparse_spd(30, 0.2, kappa=5.0)
    vals = np.arange(csr.nnz, dtype=float)
    M = ko.column_based_matrix(csr.rowptr, csr.colind, vals, csr.n).toarray()
    for j in range(csr.n):
        seg = slice(csr.rowptr[j], csr.rowptr[j + 1])
        assert np.array_equal(M[csr.colind[seg], j], vals[seg])


# ---------------------------------------------------------------------------
# Conjugate gradients


def _scipy_cg_iterations(A, b, tol, maxit):
    count = [0]

    def cb(_):
        count[0] += 1

    x, info = spla.cg(A, b, rtol=tol, atol=0.0, maxiter=maxit, callback=cb)
    return x, count[0], info


@pytest.mark.parametrize("kappa", [1e2, 1e4])
def test_cg_matches_scipy_iterations_and_solution(kappa):
    """Same recurrence, same stopping rule as scipy's CG (relative to
    ||b||): the iteration counts agree and both solve the system."""
    csr = G.random_sparse_spd(400, 0.03, kappa=kappa)
    A = csr.to_scipy()
    b = np.ones(csr.n)
    x, it, rel = ko.cg(csr.rowptr, csr.colind, csr.vals, b, tol=1e-6)
    xs, its, info = _scipy_cg_iterations(A, b, 1e-6, 2 * csr.n)
    assert info == 0 and rel <= 1e-6
    assert abs(it - its) <= 1, (it, its)
    xe = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(x - xe) <= 10 * kappa * 1e-6 * np.linalg.norm(xe)


def test_cg_terminates_in_k_steps_for_k_distinct_eigenvalues():
    """In exact arithmetic CG ends after as many steps as the operator has
    distinct eigenvalues (4 here); in FP64 the residual is at rounding
    level by then."""
    n = 60
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat([1.0, 2.0, 5.0, 9.0], n // 4)
    A = sp.csr_matrix((Q * lam) @ Q.T)
    A.sort_indices()
    b = rng.standard_normal(n)
    x, it, rel = ko.cg(A.indptr, A.indices, A.data, b, tol=1e-10)
    assert it <= 4 + 1 and rel <= 1e-10
    assert np.linalg.norm(A @ x - b) <= 1e-8 * np.linalg.norm(b)


def test_exact_preconditioner_converges_in_one_step():
    """Full pattern: the submatrix method returns A^(-1/2) exactly, so
    K^T A K = I and CG ends after one step."""
    csr = G.dense_spd(40, kappa=1e3)
    k, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, 2)
    b = np.ones(csr.n)
    x, it, rel = ko.cg(csr.rowptr, csr.colind, csr.vals, b, tol=1e-6, kvals=k)
    assert it == 1 and rel <= 1e-10
    xe = sla.solve(csr.dense(), b, assume_a="pos")
    assert np.linalg.norm(x - xe) <= 1e-9 * np.linalg.norm(xe)


def test_preconditioned_cg_solves_original_system():
    csr = G.overlap_matrix(n_atoms=30, nbf=13, rcut=4.14, kappa=1e4, seed=90)
    k, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, 2)
    b = np.ones(csr.n)
    x, it, rel = ko.cg(csr.rowptr, csr.colind, csr.vals, b, tol=1e-10, kvals=k)
    xe = sla.solve(csr.dense(), b, assume_a="pos")
    assert rel <= 1e-10
    assert np.linalg.norm(x - xe) <= 1e-5 * np.linalg.norm(xe)
    _, it0, _ = ko.cg(csr.rowptr, csr.colind, csr.vals, b, tol=1e-10)
    assert it < it0   # the submatrix preconditioner reduces the iteration count


def test_cg_zero_rhs_and_iteration_cap():
    csr = G.banded_spd(50, 3)
    x, it, rel = ko.cg(csr.rowptr, csr.colind, csr.vals, np.zeros(csr.n))
    assert it == 0 and rel == 0.0 and not np.any(x)
    x, it, rel = ko.cg(csr.rowptr, csr.colind, csr.vals, np.ones(csr.n), tol=1e-14, maxit=3)
    assert it == 3 and rel > 1e-14


def test_cg_stops_on_indefinite_operator():
    """p . A p <= 0 ends the iteration without counting it."""
    n = 10
    A = sp.diags(np.r_[np.ones(5), -np.ones(5)]).tocsr()
    A.sort_indices()
    x, it, rel = ko.cg(A.indptr, A.indices, A.data, np.r_[np.zeros(5), np.ones(5)])
    assert it == 0 and rel == 1.0


# ---------------------------------------------------------------------------
# Refinement of the inverse (Section 4.5)


def test_refinement_squares_the_residual():
    """One Newton-Schulz step maps I - A X to (I - A X)^2 exactly."""
    csr = G.overlap_matrix(n_atoms=20, nbf=13, rcut=4.14, kappa=100.0, seed=92)
    x, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, 1)
    A = csr.dense()
    X0 = ko.column_based_matrix(csr.rowptr, csr.colind, x, csr.n).toarray()
    X1, k, _, _ = ko.refine_inverse(csr.rowptr, csr.colind, csr.vals, x, tol=0.0, maxit=1)
    E0 = np.eye(csr.n) - A @ X0
    assert k == 1
    assert np.linalg.norm((np.eye(csr.n) - A @ X1) - E0 @ E0) <= 1e-12 * max(1.0, np.linalg.norm(E0 @ E0))


@pytest.mark.parametrize("kappa", [1e2, 1e4])
def test_refinement_converges_to_the_inverse(kappa):
    csr = G.overlap_matrix(n_atoms=24, nbf=13, rcut=4.14, kappa=kappa, seed=93)
    x, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, 1)
    X, k, res, ok = ko.refine_inverse(csr.rowptr, csr.colind, csr.vals, x, tol=1e-13)
    Ai = np.linalg.inv(csr.dense())
    assert ok and res <= 1e-13 and 1 <= k <= 12
    assert np.linalg.norm(X - Ai) <= 1e-12 * kappa * np.linalg.norm(Ai)


def test_refinement_of_exact_seed_takes_no_step():
    csr = G.block_diagonal_spd((4, 9, 30), kappa=10.0)
    x, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, 1)
    _, k, res, ok = ko.refine_inverse(csr.rowptr, csr.colind, csr.vals, x, tol=1e-13)
    assert ok and k == 0 and res <= 1e-13


def test_refinement_detects_divergence():
    """Diagonal A with X = 3 A^{-1}: I - A X = -2 I, spectral radius 2."""
    csr = G.diagonal_spd(30)
    X, k, res, ok = ko.refine_inverse(csr.rowptr, csr.colind, csr.vals, 3.0 / csr.vals, tol=1e-13)
    assert not ok and res > 2.0
