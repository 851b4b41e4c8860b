"""Pins of the oracle's bi/trilinear warp and its derivative.

Independent checks: identity at u = 0, exact integer translation, exact
reproduction of affine intensity functions, SciPy's map_coordinates
(order 1, edge clamp) as a library reference, and central finite differences
away from grid lines for the derivative.
"""

import numpy as np
import pytest
from scipy import ndimage

from oracle import interp_with_grad


def _rand(shape, seed):
    return np.random.default_rng(seed).uniform(0.2, 1.0, shape)


@pytest.mark.parametrize("shape", [(7, 9), (5, 6, 4)])
def test_zero_displacement_is_identity(shape):
    img = _rand(shape, 0).astype(np.float32)
    u = np.zeros((len(shape),) + shape)
    for h in (1.0, 4.0):
        W, _ = interp_with_grad(img, u, h)
        np.testing.assert_array_equal(W, img.astype(np.float64))


def test_integer_shift_is_copy():
    img = _rand((10, 12), 1)
    u = np.zeros((2, 10, 12))
    u[0] = 2.0          # 2 finest px = 1 cell at h = 2
    u[1] = -2.0
    W, _ = interp_with_grad(img, u, 2.0)
    np.testing.assert_array_equal(W[:-1, 1:], img[1:, :-1])


@pytest.mark.parametrize("shape", [(8, 9), (6, 5, 7)])
def test_affine_reproduction(shape):
    d = len(shape)
    coef = np.array([0.3, -0.7, 0.45][:d])
    grids = np.meshgrid(*[np.arange(m, dtype=float) for m in shape],
                        indexing="ij")
    img = 1.0 + sum(c * g for c, g in zip(coef, grids))
    rng = np.random.default_rng(3)
    h = 2.0
    u = rng.uniform(-1.0, 1.0, (d,) + shape) * h
    W, dW = interp_with_grad(img, u, h)
    p = [g + u[a] / h for a, g in enumerate(grids)]
    inside = np.all([(pa > 0) & (pa < m - 1) for pa, m in zip(p, shape)],
                    axis=0)
    exact = 1.0 + sum(c * pa for c, pa in zip(coef, p))
    np.testing.assert_allclose(W[inside], exact[inside], atol=1e-12)
    for a in range(d):
        np.testing.assert_allclose(dW[a][inside], coef[a] / h, atol=1e-12)


@pytest.mark.parametrize("shape", [(11, 13), (6, 7, 5)])
def test_matches_map_coordinates(shape):
    d = len(shape)
    img = _rand(shape, 4)
    rng = np.random.default_rng(5)
    u = rng.uniform(-3, 3, (d,) + shape)
    W, _ = interp_with_grad(img, u, 1.0)
    grids = np.meshgrid(*[np.arange(m, dtype=float) for m in shape],
                        indexing="ij")
    coords = np.stack([g + u[a] for a, g in enumerate(grids)])
    ref = ndimage.map_coordinates(img, coords, order=1, mode="nearest")
    np.testing.assert_allclose(W, ref, atol=1e-12)


@pytest.mark.parametrize("shape", [(9, 10), (5, 6, 7)])
def test_derivative_central_fd_off_kink(shape):
    d = len(shape)
    img = _rand(shape, 6)
    rng = np.random.default_rng(7)
    h = 2.0
    # index coordinates with fractional parts in [0.2, 0.8], inside the grid
    grids = np.meshgrid(*[np.arange(m, dtype=float) for m in shape],
                        indexing="ij")
    u = np.empty((d,) + shape)
    for a, m in enumerate(shape):
        target = rng.integers(0, m - 1, shape) + rng.uniform(0.2, 0.8, shape)
        u[a] = (target - grids[a]) * h
    W, dW = interp_with_grad(img, u, h)
    eps = 1e-6
    for a in range(d):
        up = u.copy()
        um = u.copy()
        up[a] += eps
        um[a] -= eps
        fd = (interp_with_grad(img, up, h)[0] -
              interp_with_grad(img, um, h)[0]) / (2 * eps)
        np.testing.assert_allclose(dW[a], fd, atol=1e-8)


def test_derivative_zero_outside_and_one_sided_on_grid():
    img = np.array([[0.0, 1.0, 4.0]])            # 1 x 3
    u = np.zeros((2, 1, 3))
    u[1, 0, 2] = 5.0                               # pushed past the edge
    W, dW = interp_with_grad(img, u, 1.0)
    assert W[0, 2] == 4.0 and dW[1, 0, 2] == 0.0
    # on grid lines: forward difference, backward at the last cell
    assert dW[1, 0, 0] == 1.0 and dW[1, 0, 1] == 3.0
    u[1, 0, 2] = 0.0
    _, dW = interp_with_grad(img, u, 1.0)
    assert dW[1, 0, 2] == 3.0
    # extent 1 along an axis: derivative 0
    assert np.all(dW[0] == 0.0)
