"""Refinement of the p = 2 result (Section 4.5 names iterative refinement
seeded by the submatrix-method result without giving one): a measured
demonstration, on the oracle's result for an overlap-type matrix, that the
cheap candidate iterations for A^(-1/2) are not usable from that seed.
CPU only.

X0 is the column-based submatrix-method result (not symmetric, and it does
not commute with A). The candidates are:
  * Newton-Schulz for the inverse square root: X <- X (3I - X^2 A) / 2;
  * its symmetric form: X <- (X (3I - X A X) + (3I - X A X) X) / 4, from
    the symmetric part of X0;
  * the coupled (Denman-Beavers type) Newton-Schulz iteration
    Y <- Y T, Z <- T Z, T = (3I - Z Y) / 2, seeded with Z0 = X0, Y0 = A X0
    (from Z0 = c I, Y0 = c A it returns Z -> A^(-1/2) and is stable).
From X0 the first blows up, the second decreases for a few steps and then
grows (both amplify any part of the iterate that does not commute with A
by up to lambda_i / lambda_j per step; from c I they also lose to rounding
after converging), and the coupled form stalls at a fixed point that is not
A^(-1/2). Hence the library offers refinement only for p = 1, where
X <- 2X - X A X maps I - A X to (I - A X)^2 for any seed."""
import numpy as np
import pytest

import oracle
from workloads import generators as G


def _dense_from_columns(csr, xvals):
    X = np.zeros((csr.n, csr.n))
    for j in range(csr.n):
        seg = slice(csr.rowptr[j], csr.rowptr[j + 1])
        X[csr.colind[seg], j] = xvals[seg]
    return X


def _true_inv_sqrt(A):
    lam, Q = np.linalg.eigh(A)
    return (Q / np.sqrt(lam)) @ Q.T


def _ns(X, A, steps):
    out = []
    for _ in range(steps):
        X = 0.5 * X @ (3.0 * np.eye(len(A)) - X @ X @ A)
        out.append(X)
    return out


def _ns_sym(X, A, steps):
    out = []
    I = np.eye(len(A))
    for _ in range(steps):
        T = 3.0 * I - X @ A @ X
        X = 0.25 * (X @ T + T @ X)
        out.append(X)
    return out


def _coupled(Z, A, steps):
    out = []
    I = np.eye(len(A))
    Y = A @ Z
    for _ in range(steps):
        T = 0.5 * (3.0 * I - Z @ Y)
        Y, Z = Y @ T, T @ Z
        out.append(Z)
    return out


@pytest.fixture(scope="module")
def case():
    csr = G.overlap_matrix(n_atoms=24, nbf=13, rcut=4.14, kappa=100.0, seed=G.BASE_SEED + 90)
    A = csr.dense()
    x, bad = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, 2)
    assert bad == 0
    X0 = _dense_from_columns(csr, x)
    return A, X0, _true_inv_sqrt(A)


def _res(X, A):
    with np.errstate(all="ignore"):
        r = np.linalg.norm(X @ A @ X - np.eye(len(A)))
    return r if np.isfinite(r) else np.inf


def test_coupled_iteration_converges_from_a_commuting_seed(case):
    """The reference: the coupled form from Z0 = c I reaches A^(-1/2)."""
    A, _, R = case
    c = 1.0 / np.sqrt(np.linalg.eigvalsh(A)[-1])
    Z = _coupled(c * np.eye(len(A)), A, 40)[-1]
    assert np.linalg.norm(Z - R) / np.linalg.norm(R) <= 1e-12


def test_candidates_fail_from_the_submatrix_seed(case):
    """Measured on this case (n = 312, kappa = 100; seed residual
    ||X0 A X0 - I||_F = 0.157, distance to A^(-1/2) 3.0e-3):
    Newton-Schulz 0.49, 8.3, 256, ... (overflow); the symmetric form first
    drops to 0.017, then grows back (0.24 after 8 steps, and on); the
    coupled form stalls at residual 4.4e-2, 7.4e-4 away from A^(-1/2)."""
    A, X0, R = case
    r0 = _res(X0, A)
    ns = [_res(X, A) for X in _ns(X0, A, 8)]
    sym = [_res(X, A) for X in _ns_sym(0.5 * (X0 + X0.T), A, 40)]
    Z = _coupled(X0, A, 40)
    dz = np.linalg.norm(Z[-1] - R) / np.linalg.norm(R)
    print(f"seed residual {r0:.3e}; Newton-Schulz {['%.2e' % v for v in ns]}; symmetric after 8/40 steps "
          f"{sym[7]:.2e}/{sym[-1]:.2e}; coupled after 40 steps {_res(Z[-1], A):.2e}, distance {dz:.2e}")
    assert 0.01 < r0 < 1.0              # a useful seed
    assert ns[-1] > 1e3 * r0            # diverges
    assert sym[-1] > r0                 # grows past its seed after the first steps
    assert _res(Z[-1], A) > 1e-3 and dz > 1e-5                   # stalls away from A^(-1/2)
    assert abs(_res(Z[-1], A) - _res(Z[-10], A)) < 1e-3 * _res(Z[-1], A)   # a fixed point, not slow convergence
