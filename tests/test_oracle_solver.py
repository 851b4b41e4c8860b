"""Pins of the oracle's PCG and Gauss-Newton solver.

Independent checks: numpy.linalg.solve on small SPD systems, the monotone
energy error of CG, exact recovery of known integer translations of a
compact phantom (a zero-residual problem whose minimiser is known), exact
invariance under zero motion, and monotone decrease of J.
"""

import numpy as np
import pytest

from oracle import ModelParams, pcg, gauss_newton, objective_value
from paper_2001_06613_amd import synth


def test_pcg_reaches_dense_solve():
    rng = np.random.default_rng(0)
    N = 30
    A = rng.standard_normal((N, N))
    A = A @ A.T / N + np.identity(N)
    b = rng.standard_normal(N)
    diag = np.diag(A).copy()
    x, it, st = pcg(lambda v: A @ v, diag, b, cg_max=N, rtol=0.0, fixed=True)
    assert st == "ok"
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10,
                               atol=1e-10)


def test_pcg_energy_error_decreases():
    rng = np.random.default_rng(1)
    N = 40
    A = rng.standard_normal((N, N))
    A = A @ A.T + np.identity(N)
    b = rng.standard_normal(N)
    xs = np.linalg.solve(A, b)
    errs = []
    for k in range(1, 15):
        x, _, _ = pcg(lambda v: A @ v, np.diag(A).copy(), b, k, 0.0, True)
        e = x - xs
        errs.append(float(e @ A @ e))
    assert all(b_ <= a_ * (1 + 1e-12) for a_, b_ in zip(errs, errs[1:]))


def test_pcg_zero_rhs_and_breakdown():
    A = np.identity(3)
    x, it, st = pcg(lambda v: A @ v, np.ones(3), np.zeros(3), 5)
    assert it == 0 and np.all(x == 0) and st == "ok"
    x, it, st = pcg(lambda v: -v, np.ones(3), np.ones(3), 5)
    assert st == "breakdown" and it == 0


@pytest.mark.parametrize("reg", ["diffusion", "curvature"])
def test_gn_recovers_integer_translations(reg):
    shifts = np.array([[1.0, -1.0], [-1.0, 0.0], [0.0, 1.0]])   # sum 0
    frames = synth.translated_sequence(shifts, (32, 32), seed=1)
    u0 = np.zeros((3, 2, 32, 32))
    par = ModelParams(alpha=1e-2, lam=1e-1, reg=reg)
    res = gauss_newton(frames, u0, [0, 1, 2], 1.0, par, gn_max=40,
                       cg_max=200, cg_rtol=1e-8, tol_J=0.0, tol_u=0.0)
    assert res.J < 1e-6 * res.J0
    for k in range(3):
        for a in range(2):
            assert np.max(np.abs(res.u[k, a] - shifts[k, a])) < 1e-3


def test_gn_zero_motion_stays_zero():
    f = synth.base_image(np.random.default_rng(3), (16, 16))
    frames = np.repeat(f[None].astype(np.float32), 3, axis=0)
    u0 = np.zeros((3, 2, 16, 16))
    res = gauss_newton(frames, u0, [0, 1, 2], 1.0, ModelParams(),
                       gn_max=3, cg_max=5, fixed=True)
    assert np.all(res.u == 0.0) and res.J == 0.0 and res.iterations == 3


def test_gn_monotone_decrease():
    frames, _ = synth.config_small(0)
    frames = frames[:, ::2, ::2]          # 32 x 32, 8 frames
    u0 = np.zeros((8, 2, 32, 32))
    res = gauss_newton(frames, u0, [0, 2, 4, 6, 7], 2.0, ModelParams(),
                       gn_max=5, cg_max=10, fixed=True)
    hist = [res.J0] + res.J_history
    assert all(b < a for a, b in zip(hist, hist[1:]))
    # frames outside K keep their start value
    assert np.all(res.u[[1, 3, 5]] == 0.0)
    J_check = objective_value(frames, res.u, [0, 2, 4, 6, 7], 2.0,
                              ModelParams())[0]
    assert J_check == pytest.approx(res.J, rel=1e-12)


def test_pcg_jacobi_exact_on_diagonal_in_one_step():
    # With M = diag(A) = A the preconditioned system is the identity, so the
    # first Jacobi-PCG step is the exact solution; plain CG (or any other
    # scaling of r) needs one step per distinct eigenvalue.
    d = np.array([1.0, 3.0, 10.0, 0.2, 7.5, 42.0])
    b = np.array([1.0, -2.0, 0.5, 3.0, -1.5, 0.25])
    x, it, st = pcg(lambda v: d * v, d.copy(), b, cg_max=1, rtol=0.0,
                    fixed=True)
    assert it == 1 and st == "ok"
    np.testing.assert_allclose(x, b / d, rtol=1e-14, atol=0)


def _galerkin_krylov(A, Minv, b, k):
    """A-norm minimiser of the error over span{Minv b, (Minv A) Minv b, ...}
    (k vectors), built densely; the classical characterisation of the k-th
    preconditioned CG iterate started at 0."""
    cols = [Minv @ b]
    for _ in range(k - 1):
        cols.append(Minv @ (A @ cols[-1]))
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    return Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ b)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
def test_pcg_iterates_are_preconditioned_krylov_minimisers(k):
    rng = np.random.default_rng(7)
    N = 14
    B = rng.standard_normal((N, N))
    S = np.diag(np.exp(rng.uniform(-2.0, 2.0, N)))   # strongly uneven scale
    A = S @ (B @ B.T / N + np.identity(N)) @ S
    b = rng.standard_normal(N)
    diag = np.diag(A).copy()
    x, it, st = pcg(lambda v: A @ v, diag, b, cg_max=k, rtol=0.0, fixed=True)
    assert it == k and st == "ok"
    ref = _galerkin_krylov(A, np.diag(1.0 / diag), b, k)
    np.testing.assert_allclose(x, ref, rtol=1e-9, atol=1e-12)
    # the test separates Jacobi from no preconditioner and from M = 1/diag
    for wrong in (np.identity(N), np.diag(diag)):
        assert np.max(np.abs(_galerkin_krylov(A, wrong, b, k) - ref)) > \
            1e-3 * np.max(np.abs(ref))


class _UnderestimatedQuadratic:
    """J(x) = (c/2)|x|^2 with a Gauss-Newton Hessian c/rho I (rho > 1).

    The Gauss-Newton direction is delta = -rho x, and
    J(x + t delta) = J(x) (1 - t rho)^2, so Armijo with constant c1 holds
    exactly for t <= 2 (1 - c1) / rho: the unit step fails for rho > 2 and
    the ladder 1, 1/2, 1/4, ... stops at the first power of two below that.
    """

    def __init__(self, c, rho):
        self.c, self.rho = c, rho

    def value(self, x):
        return 0.5 * self.c * float(np.sum(x * x))

    def evaluate(self, x):
        return self.value(x), self.c * x, None

    def hessvec(self, state, v):
        return (self.c / self.rho) * v

    def diag(self, state):
        return np.full(1, self.c / self.rho)


@pytest.mark.parametrize("rho,t_expected", [(3.0, 0.5), (5.0, 0.25),
                                             (10.0, 0.125), (1.5, 1.0)])
def test_gn_armijo_ladder_closed_form(rho, t_expected):
    from oracle.solver import gn_minimise

    model = _UnderestimatedQuadratic(2.0, rho)
    x0 = np.array([0.75])
    res = gn_minimise(model, x0, gn_max=1, cg_max=1, ls_max=10, c1=1e-4,
                      fixed=True)
    assert res.steps == [t_expected]
    # the accepted point in closed form: x0 (1 - t rho)
    np.testing.assert_allclose(res.u, x0 * (1.0 - t_expected * rho),
                               rtol=1e-15)
    assert res.J == pytest.approx(model.value(x0) *
                                  (1.0 - t_expected * rho) ** 2, rel=1e-14)


def test_gn_armijo_ladder_length():
    from oracle.solver import gn_minimise

    # t <= 2 (1 - c1) / 4000 ~ 5.0e-4 < 2^-10: ten halvings are not enough,
    # eleven are (ls_max counts the halvings after t = 1)
    model = _UnderestimatedQuadratic(1.0, 4000.0)
    res = gn_minimise(model, np.array([1.0]), gn_max=1, cg_max=1, ls_max=10,
                      fixed=True)
    assert res.status == "linesearch" and res.steps == []
    assert np.all(res.u == 1.0)
    res = gn_minimise(model, np.array([1.0]), gn_max=1, cg_max=1, ls_max=11,
                      fixed=True)
    assert res.steps == [2.0 ** -11]
