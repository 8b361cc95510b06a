"""Plant plausible mistakes in the oracle (CPU only) and check that the pins
catch each of them: a pin set that cannot fail pins nothing."""
import numpy as np
import pytest

import oracle.submat_oracle as so
import tests.test_oracle_pins as pins


def _wrong_column(S, c, p):
    lam, Q = so.eig(S)
    c2 = (c + 1) % S.shape[0]
    return Q @ (so.inv_root(lam, p) * Q[c2, :]), True


def _transposed_q(S, c, p):
    lam, Q = so.eig(S)
    return Q.T @ (so.inv_root(lam, p) * Q[c, :]), True


def _positive_root(S, c, p):
    lam, Q = so.eig(S)
    return Q @ (so.root(lam, p) * Q[c, :]), True


def _dropped_eig_term(S, c, p):
    lam, Q = so.eig(S)
    f = so.inv_root(lam, p)
    f[0] = 0.0
    return Q @ (f * Q[c, :]), True


def _no_symmetrise_adjoint(S, c, w, p):
    lam, Q = so.eig(S)
    M = so.divided_differences(lam, p) * np.outer(Q.T @ w, Q[c, :])
    return Q @ M @ Q.T


def _wrong_b_adjoint(S, c, w, p):
    lam, Q = so.eig(S)
    M = so.divided_differences(lam, p) * np.outer(Q.T @ w, Q[:, c])
    return Q @ (0.5 * (M + M.T)) @ Q.T


def _sign_flipped_G(lam, p):
    a = so.root(lam, p)
    s = sum(a[:, None] ** i * a[None, :] ** (p - 1 - i) for i in range(p))
    return 1.0 / (a[:, None] * a[None, :] * s)


def _dropped_G_term(lam, p):
    a = so.root(lam, p)
    s = sum(a[:, None] ** i * a[None, :] ** (p - 1 - i) for i in range(max(p - 1, 1)))
    return -1.0 / (a[:, None] * a[None, :] * s)


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
    monkeypatch.setattr(so, "column_of_inverse_root", mutant)
    assert _some_pin_fails(FORWARD_PINS) >= 1


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
