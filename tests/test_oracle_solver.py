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
