"""Plant plausible mistakes in the oracle (CPU only) and check that the pins
catch each of them: a pin set that cannot fail pins nothing."""
import numpy as np
import pytest

import oracle.submat_oracle as so
import tests.test_oracle_matfun_pins as mpins
import tests.test_oracle_pins as pins


def _wrong_column(S, c, fn, p):
    lam, Q = so.eig(S)
    c2 = (c + 1) % S.shape[0]
    return Q @ (so.spectral_function(lam, fn, p) * Q[c2, :]), True


def _transposed_q(S, c, fn, p):
    lam, Q = so.eig(S)
    return Q.T @ (so.spectral_function(lam, fn, p) * Q[c, :]), True


def _positive_root(S, c, fn, p):
    lam, Q = so.eig(S)
    return Q @ (so.root(lam, p) * Q[c, :]), True


def _dropped_eig_term(S, c, fn, p):
    lam, Q = so.eig(S)
    f = so.spectral_function(lam, fn, p)
    f[0] = 0.0
    return Q @ (f * Q[c, :]), True


def _no_symmetrise_adjoint(S, c, w, p, fn="inv_root"):
    lam, Q = so.eig(S)
    M = so.divided_differences(lam, p, fn) * np.outer(Q.T @ w, Q[c, :])
    return Q @ M @ Q.T


def _wrong_b_adjoint(S, c, w, p, fn="inv_root"):
    lam, Q = so.eig(S)
    M = so.divided_differences(lam, p, fn) * np.outer(Q.T @ w, Q[:, c])
    return Q @ (0.5 * (M + M.T)) @ Q.T


_ORIG_DD = so.divided_differences
_ORIG_F = so.spectral_function


def _sign_flipped_G(lam, p, fn="inv_root"):
    if fn != "inv_root":
        return _ORIG_DD(lam, p, fn)
    a = so.root(lam, p)
    s = sum(a[:, None] ** i * a[None, :] ** (p - 1 - i) for i in range(p))
    return 1.0 / (a[:, None] * a[None, :] * s)


def _dropped_G_term(lam, p, fn="inv_root"):
    if fn != "inv_root":
        return _ORIG_DD(lam, p, fn)
    a = so.root(lam, p)
    s = sum(a[:, None] ** i * a[None, :] ** (p - 1 - i) for i in range(max(p - 1, 1)))
    return -1.0 / (a[:, None] * a[None, :] * s)


# mistakes in the other spectral functions


def _root_G_sign_flipped(lam, p, fn="inv_root"):
    G0 = _ORIG_DD(lam, p, fn)
    return -G0 if fn == "root" else G0


def _root_G_as_inverse_root(lam, p, fn="inv_root"):
    return _ORIG_DD(lam, p, "inv_root" if fn == "root" else fn)


def _power_G_unscaled(lam, p, fn="inv_root"):
    G0 = _ORIG_DD(lam, p, fn)
    if fn != "power":
        return G0
    return G0 / np.power(lam[None, :], float(p))


def _power_G_log_not_log1p(lam, p, fn="inv_root"):
    if fn != "power":
        return _ORIG_DD(lam, p, fn)
    alpha = float(p)
    lk, ll = lam[:, None] * np.ones((1, lam.size)), lam[None, :] * np.ones((lam.size, 1))
    diff = lk - ll
    G = alpha * np.power(ll, alpha - 1.0)
    o = diff != 0
    G[o] = np.power(ll[o], alpha) * np.expm1(alpha * np.log(diff[o] / ll[o] + 2.0)) / diff[o]
    return G


def _root_f_is_inverse_root(lam, fn, param):
    return _ORIG_F(lam, "inv_root" if fn == "root" else fn, param)


def _power_f_reciprocal_exponent(lam, fn, param):
    if fn != "power":
        return _ORIG_F(lam, fn, param)
    return np.power(lam, 1.0 / float(param))


_ORIG_GATHER = so.gather_submatrix


def _gather_ignores_pattern(rowptr, colind, vals, R):
    S, pos = _ORIG_GATHER(rowptr, colind, vals, R)
    # an off-by-one in the merge: the last stored neighbour is dropped
    S2 = S.copy()
    S2[-1, :-1] = 0.0
    S2[:-1, -1] = 0.0
    return S2, pos


FORWARD_PINS = [
    lambda: pins.test_block_diagonal_is_exact_inverse_root(2, False),
    lambda: pins.test_dense_matrix_gives_exact_inverse_root(2),
    lambda: pins.test_p1_columns_are_cholesky_solves(),
    lambda: pins.test_p2_columns_are_sqrtm_solves(),
    lambda: pins.test_literal_dense_algorithms_match(2),
    lambda: pins.test_arrowhead_two_by_two_closed_form(),
    lambda: pins.test_p1_exact_rational_brute_force(),
    lambda: pins.test_diagonal_is_elementwise_root_within_ulps(2),
]

ADJOINT_PINS = [
    lambda: pins.test_adjoint_diagonal_closed_form(2),
    lambda: pins.test_adjoint_p1_closed_form(),
    lambda: pins.test_adjoint_p2_sylvester(),
    lambda: pins.test_adjoint_central_finite_differences(3),
    lambda: pins.test_divided_differences_match_definition(3),
]


MATFUN_FORWARD_PINS = [
    lambda: mpins.test_power_one_reproduces_A(),
    lambda: mpins.test_power_two_is_A_squared_on_the_pattern(),
    lambda: mpins.test_root2_of_dense_matrix_is_sqrtm(),
    lambda: mpins.test_block_diagonal_root_powers_back_to_A(3, True),
    lambda: mpins.test_dense_real_power_matches_schur_pade(2.5),
]

MATFUN_ADJOINT_PINS = [
    lambda: mpins.test_divided_differences_high_precision("root", 2),
    lambda: mpins.test_divided_differences_high_precision("power", 0.7),
    lambda: mpins.test_adjoint_power_one_is_symmetrised_upstream(),
    lambda: mpins.test_adjoint_root2_sylvester(),
    lambda: mpins.test_matfun_adjoint_central_finite_differences("power", -1.3),
]


def _some_pin_fails(pin_list):
    failures = 0
    for pin in pin_list:
        try:
            pin()
        except AssertionError:
            failures += 1
    return failures


@pytest.mark.parametrize("mutant", [_wrong_column, _transposed_q, _positive_root, _dropped_eig_term])
def test_forward_mutants_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(so, "column_of_function", mutant)
    assert _some_pin_fails(FORWARD_PINS) >= 1


@pytest.mark.parametrize("mutant", [_wrong_column, _transposed_q, _dropped_eig_term])
def test_forward_mutants_are_caught_by_other_function_pins(monkeypatch, mutant):
    monkeypatch.setattr(so, "column_of_function", mutant)
    assert _some_pin_fails(MATFUN_FORWARD_PINS) >= 1


@pytest.mark.parametrize("mutant", [_root_f_is_inverse_root, _power_f_reciprocal_exponent])
def test_spectral_function_mutants_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(so, "spectral_function", mutant)
    assert _some_pin_fails(MATFUN_FORWARD_PINS) >= 1


@pytest.mark.parametrize("mutant", [_root_G_sign_flipped, _root_G_as_inverse_root, _power_G_unscaled,
                                    _power_G_log_not_log1p])
def test_other_function_divided_difference_mutants_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(so, "divided_differences", mutant)
    assert _some_pin_fails(MATFUN_ADJOINT_PINS) >= 1


@pytest.mark.parametrize("mutant", [_no_symmetrise_adjoint, _wrong_b_adjoint])
def test_adjoint_mutants_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(so, "adjoint_column", mutant)
    assert _some_pin_fails(ADJOINT_PINS) >= 1


@pytest.mark.parametrize("mutant", [_sign_flipped_G, _dropped_G_term])
def test_divided_difference_mutants_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(so, "divided_differences", mutant)
    assert _some_pin_fails(ADJOINT_PINS) >= 1


def test_gather_mutant_is_caught(monkeypatch):
    monkeypatch.setattr(so, "gather_submatrix", _gather_ignores_pattern)
    assert _some_pin_fails(FORWARD_PINS) >= 1


# ---------------------------------------------------------------------------
# residual metric and conjugate gradients (Sections 4.1 and 4.4)

from oracle import krylov_oracle as ko  # noqa: E402
import tests.test_oracle_krylov_pins as kpins  # noqa: E402

_ORIG_RES_OP = ko.residual_operator
_ORIG_ROW_BASED = ko.row_based_matrix


def _res_op_one_power_short(xvals, rowptr, colind, avals, n, p):
    return _ORIG_RES_OP(xvals, rowptr, colind, avals, n, max(p - 1, 1) if p > 1 else p)


def _column_based_is_row_based(rowptr, colind, vals, n):
    return _ORIG_ROW_BASED(rowptr, colind, vals, n)


def _cg_beta_from_dq(rowptr, colind, avals, b, tol=1e-6, maxit=None, kvals=None):
    """CG with beta = rr_new / (d . B d) instead of rr_new / rr."""
    n = len(rowptr) - 1
    A = ko.row_based_matrix(rowptr, colind, avals, n)
    K = ko.column_based_matrix(rowptr, colind, kvals, n) if kvals is not None else None
    op = (lambda v: K.T @ (A @ (K @ v))) if K is not None else (lambda v: A @ v)
    rhs = K.T @ b if K is not None else np.asarray(b, dtype=float).copy()
    maxit = 2 * n if maxit is None else maxit
    y, r = np.zeros(n), rhs.copy()
    d, rr = r.copy(), float(r @ r)
    bnorm, it = np.sqrt(rr), 0
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0
    while it < maxit:
        q = op(d)
        dq = float(d @ q)
        if not dq > 0.0:
            break
        y, r = y + (rr / dq) * d, r - (rr / dq) * q
        rr_new = float(r @ r)
        it += 1
        if np.sqrt(rr_new) <= tol * bnorm:
            rr = rr_new
            break
        d = r + (rr_new / dq) * d
        rr = rr_new
    return (K @ y if K is not None else y), it, float(np.sqrt(rr) / bnorm)


_ORIG_CG = ko.cg


def _cg_rhs_without_kt(rowptr, colind, avals, b, tol=1e-6, maxit=None, kvals=None):
    """Preconditioned CG with K b instead of K^T b on the right."""
    if kvals is None:
        return _ORIG_CG(rowptr, colind, avals, b, tol, maxit, None)
    n = len(rowptr) - 1
    K = ko.column_based_matrix(rowptr, colind, kvals, n)
    b2 = K.T @ np.linalg.lstsq(K.T.toarray(), K @ b, rcond=None)[0]
    return _ORIG_CG(rowptr, colind, avals, b2, tol, maxit, kvals)


RESIDUAL_PINS = [
    lambda: kpins.test_sparse_residual_norm_equals_dense_definition(2),
    lambda: kpins.test_residual_norm_diagonal_closed_form(2),
    lambda: kpins.test_residual_operator_transpose_is_adjoint(),
    lambda: kpins.test_column_based_matrix_reads_segments_as_columns(),
]

CG_PINS = [
    lambda: kpins.test_cg_matches_scipy_iterations_and_solution(1e2),
    lambda: kpins.test_cg_terminates_in_k_steps_for_k_distinct_eigenvalues(),
    lambda: kpins.test_exact_preconditioner_converges_in_one_step(),
    lambda: kpins.test_preconditioned_cg_solves_original_system(),
]


@pytest.mark.parametrize("name,mutant", [("residual_operator", _res_op_one_power_short),
                                         ("column_based_matrix", _column_based_is_row_based)])
def test_residual_mutants_are_caught(monkeypatch, name, mutant):
    monkeypatch.setattr(ko, name, mutant)
    assert _some_pin_fails(RESIDUAL_PINS) >= 1


@pytest.mark.parametrize("mutant", [_cg_beta_from_dq, _cg_rhs_without_kt])
def test_cg_mutants_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(ko, "cg", mutant)
    assert _some_pin_fails(CG_PINS) >= 1


_ORIG_REFINE = ko.refine_inverse


def _refine_wrong_product_order(rowptr, colind, avals, xvals, tol=1e-14, maxit=20):
    """X_{k+1} = 2 X - (A X) X instead of 2 X - X (A X)."""
    n = len(rowptr) - 1
    A = ko.row_based_matrix(rowptr, colind, avals, n).toarray()
    X = ko.column_based_matrix(rowptr, colind, xvals, n).toarray()
    k, res0 = 0, None
    while True:
        T = A @ X
        res = float(np.linalg.norm(T - np.eye(n)) / np.sqrt(n))
        res0 = res if res0 is None else res0
        if res <= tol:
            return X, k, res, True
        if not np.isfinite(res) or res > 1e3 * max(res0, 1.0) or k >= maxit:
            return X, k, res, False
        X = 2.0 * X - T @ X
        k += 1


REFINE_PINS = [
    lambda: kpins.test_refinement_squares_the_residual(),
    lambda: kpins.test_refinement_converges_to_the_inverse(1e4),
]


def test_refinement_mutant_is_caught(monkeypatch):
    monkeypatch.setattr(ko, "refine_inverse", _refine_wrong_product_order)
    assert _some_pin_fails(REFINE_PINS) >= 1
