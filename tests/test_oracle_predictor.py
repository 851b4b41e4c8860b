"""Pins of the oracle's temporal predictors (Sec. 3 and eq. (2)).

Independent checks: the paper's 0.5/0.5 midpoint rule, a dense solve of the
normal equations assembled from the objective of eq. (2) itself (by a
Hessian of the quadratic, not by the tridiagonal formula), and the closed
forms of the beta -> 0 and beta -> infinity limits.
"""

import numpy as np
import pytest

from oracle import linear_predict, ls_predict, thomas_solve, ls_system, \
    temporal_sets


def test_linear_midpoint_rule():
    n = 17
    K0 = temporal_sets(n, 4)[0]           # {0, 8, 16}
    rng = np.random.default_rng(0)
    Y = rng.standard_normal((n, 2, 3))
    Z = linear_predict(Y, K0)
    np.testing.assert_array_equal(Z[K0], Y[K0])
    np.testing.assert_allclose(Z[4], 0.5 * Y[0] + 0.5 * Y[8], atol=1e-15)
    np.testing.assert_allclose(Z[12], 0.5 * Y[8] + 0.5 * Y[16], atol=1e-15)
    # off-midpoint (n = 8, K_0 = {0,2,4,6,7}): frame 5 halfway 4..6
    Y = rng.standard_normal((8, 4))
    Z = linear_predict(Y, [0, 3, 7])
    np.testing.assert_allclose(Z[5], 0.5 * Y[3] + 0.5 * Y[7], atol=1e-15)
    np.testing.assert_allclose(Z[1], (2 * Y[0] + Y[3]) / 3, atol=1e-15)


def _ls_objective_dense(n, Kq, beta):
    """Hessian/2 and linear term of eq. (2) built entry by entry."""
    A = np.zeros((n, n))
    for k in Kq:
        A[k, k] += 1.0
    for k in range(n - 1):
        e = np.zeros(n)
        e[k + 1] += 1.0
        e[k] -= 1.0
        A += beta * np.outer(e, e)
    return A


@pytest.mark.parametrize("n,nt,beta", [(17, 4, 1e-5), (17, 4, 0.3),
                                       (64, 3, 1e-2), (9, 2, 10.0),
                                       (8, 2, 1.0)])
def test_thomas_equals_dense_solve(n, nt, beta):
    Kq = temporal_sets(n, nt)[0]
    rng = np.random.default_rng(1)
    eta = rng.standard_normal((n, 5))
    omega = rng.standard_normal((n, 5))
    zeta = ls_predict(eta, omega, Kq, beta)
    A = _ls_objective_dense(n, Kq, beta)
    m = np.zeros(n)
    m[Kq] = 1.0
    D = np.diff(np.identity(n), axis=0)       # (n-1) x n forward difference
    rhs = m[:, None] * eta + beta * D.T @ (D @ omega)
    ref = np.linalg.solve(A, rhs)
    np.testing.assert_allclose(zeta, ref, rtol=1e-9, atol=1e-9)
    # gradient of eq. (2) vanishes at zeta
    grad = 2 * m[:, None] * (zeta - eta) + 2 * beta * D.T @ (
        D @ zeta - D @ omega)
    assert np.abs(grad).max() < 1e-9


def test_thomas_generic():
    rng = np.random.default_rng(2)
    n = 12
    sub = rng.uniform(-1, 1, n)
    sup = rng.uniform(-1, 1, n)
    diag = 3 + rng.uniform(0, 1, n)
    sub[0] = 0
    sup[-1] = 0
    A = np.diag(diag) + np.diag(sub[1:], -1) + np.diag(sup[:-1], 1)
    b = rng.standard_normal((n, 3))
    np.testing.assert_allclose(thomas_solve(sub, diag, sup, b),
                               np.linalg.solve(A, b), atol=1e-12)


def test_beta_to_zero_limit():
    """beta -> 0: zeta = omega + linear interpolation of (eta - omega)."""
    n = 17
    Kq = temporal_sets(n, 4)[1]
    rng = np.random.default_rng(3)
    eta = rng.standard_normal((n, 3))
    omega = rng.standard_normal((n, 3))
    zeta = ls_predict(eta, omega, Kq, 1e-9)
    lin = omega + linear_predict(eta - omega, Kq)
    np.testing.assert_allclose(zeta, lin, atol=1e-6)
    # omega = 0 reduces to the coarse-level linear predictor
    np.testing.assert_allclose(ls_predict(eta, 0 * omega, Kq, 1e-9),
                               linear_predict(eta, Kq), atol=1e-6)


def test_beta_to_infinity_limit():
    n = 9
    Kq = temporal_sets(n, 3)[0]
    rng = np.random.default_rng(4)
    eta = rng.standard_normal((n, 2))
    omega = rng.standard_normal((n, 2))
    zeta = ls_predict(eta, omega, Kq, 1e9)
    ref = omega + (eta[Kq] - omega[Kq]).mean(axis=0)
    np.testing.assert_allclose(zeta, ref, atol=1e-6)


def test_eta_equals_omega_fixed_point():
    n = 33
    Kq = temporal_sets(n, 3)[1]
    omega = np.random.default_rng(5).standard_normal((n, 4))
    np.testing.assert_allclose(ls_predict(omega, omega, Kq, 1e-5), omega,
                               atol=1e-12)


def test_ls_system_shape():
    sub, diag, sup = ls_system(5, [0, 2, 4], 0.5)
    np.testing.assert_array_equal(diag, [1.5, 1.0, 2.0, 1.0, 1.5])
    assert sub[0] == 0 and sup[-1] == 0 and np.all(sub[1:] == -0.5)
