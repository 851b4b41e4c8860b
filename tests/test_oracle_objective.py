"""Pins of the oracle's objective, gradient, Hessian product and diagonal.

Independent checks: the literal pairwise form of eq. (1), the pair SSD,
central finite differences of J, a Jacobian of the residual assembled column
by column by finite differences, SciPy sparse operators built by Kronecker
products, closed-form interior stencils, null spaces, symmetry and positive
definiteness.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import (ModelParams, objective, objective_value, hessvec,
                    jacobi_diag, reg_apply_BtB, reg_value, interp_with_grad)


def _frames(n, shape, seed):
    return np.random.default_rng(seed).uniform(0.2, 1.0, (n,) + shape)


def _offkink_u(n, shape, h, seed, lo=0.1, hi=0.9):
    """Displacements whose index coordinates have fractions in [lo, hi]."""
    rng = np.random.default_rng(seed)
    d = len(shape)
    grids = np.meshgrid(*[np.arange(m, dtype=float) for m in shape],
                        indexing="ij")
    u = np.empty((n, d) + shape)
    for k in range(n):
        for a, m in enumerate(shape):
            tgt = np.clip(grids[a] + rng.integers(-1, 2, shape), 0, m - 2) \
                + rng.uniform(lo, hi, shape)
            u[k, a] = (tgt - grids[a]) * h
    return u


def test_D_matches_literal_pairwise_eq1():
    frames = _frames(4, (6, 7), 0)
    u = _offkink_u(4, (6, 7), 1.0, 1)
    K = [0, 1, 3]
    h = 2.0
    par = ModelParams(alpha=0.0, lam=0.0)
    D = objective_value(frames, u, K, h, par)[1]
    W = [interp_with_grad(frames[k], u[k], h)[0] for k in K]
    pair = 0.0
    for Wi in W:
        for Wj in W:
            # FAIR pair SSD (h^d / 2) ||Wi - Wj||^2, summed over ordered pairs
            pair += 0.5 * h**2 * np.sum((Wi - Wj) ** 2)
    assert D == pytest.approx(pair / len(K), rel=1e-13)


def test_pair_ssd_two_frames():
    frames = _frames(2, (5, 5), 2)
    u = np.zeros((2, 2, 5, 5))
    D = objective_value(frames, u, [0, 1], 1.0, ModelParams(0, 0))[1]
    assert D == pytest.approx(0.5 * np.sum((frames[0] - frames[1]) ** 2),
                              rel=1e-14)


def test_identical_frames_zero_objective_and_gradient():
    f = _frames(1, (6, 8), 3)
    frames = np.repeat(f, 4, axis=0)
    u = np.zeros((4, 2, 6, 8))
    for reg in ("diffusion", "curvature"):
        o = objective(frames, u, [0, 1, 2, 3], 1.0, ModelParams(0.1, 0.1, reg))
        assert o["J"] == 0.0
        assert np.all(o["g"] == 0.0)


@pytest.mark.parametrize("reg", ["diffusion", "curvature"])
@pytest.mark.parametrize("shape,h", [((8, 8), 1.0), ((5, 6, 4), 2.0)])
def test_gradient_central_fd(reg, shape, h):
    n = 3
    frames = _frames(n, shape, 4)
    u = _offkink_u(n, shape, h, 5)
    K = [0, 1, 2]
    par = ModelParams(alpha=0.3, lam=0.2, reg=reg)
    o = objective(frames, u, K, h, par)
    g = o["g"]
    eps = 1e-6
    rng = np.random.default_rng(6)
    flat = [np.unravel_index(i, u.shape) for i in
            rng.choice(u.size, 40, replace=False)]
    for idx in flat:
        up = u.copy()
        um = u.copy()
        up[idx] += eps
        um[idx] -= eps
        fd = (objective_value(frames, up, K, h, par)[0] -
              objective_value(frames, um, K, h, par)[0]) / (2 * eps)
        k = K.index(idx[0])
        assert g[(k,) + idx[1:]] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def _kron_ops(shape):
    """B for diffusion and curvature as scipy.sparse, built by Kronecker
    products of 1-D difference matrices (index order = C order)."""
    d = len(shape)
    Ds = []
    for m in shape:
        Ds.append(sp.diags([-np.ones(m - 1), np.ones(m - 1)], [0, 1],
                           shape=(m - 1, m)).tocsr())
    blocks = []
    for a in range(d):
        mats = [sp.identity(m) for m in shape]
        mats[a] = Ds[a]
        M = mats[0]
        for X in mats[1:]:
            M = sp.kron(M, X)
        blocks.append(M)
    Bd = sp.vstack(blocks).tocsr()
    L = -(Bd.T @ Bd)
    return Bd, L


@pytest.mark.parametrize("shape", [(5, 7), (4, 3, 5)])
@pytest.mark.parametrize("reg", ["diffusion", "curvature"])
def test_BtB_matches_kron_operator(shape, reg):
    h = 2.0
    Bd, L = _kron_ops(shape)
    B = Bd / h if reg == "diffusion" else L / h**2
    rng = np.random.default_rng(7)
    v = rng.standard_normal(shape)
    ref = (B.T @ (B @ v.ravel())).reshape(shape)
    np.testing.assert_allclose(reg_apply_BtB(v, reg, h, len(shape)), ref,
                               atol=1e-12)
    assert reg_value(v, reg, h, len(shape)) == pytest.approx(
        float(np.sum((B @ v.ravel()) ** 2)), rel=1e-12)


def test_curvature_interior_stencils():
    # 2-D: centre 20, face -8, diagonal 2, distance-2 along an axis 1
    e = np.zeros((9, 9))
    e[4, 4] = 1.0
    s = reg_apply_BtB(e, "curvature", 1.0, 2)
    assert s[4, 4] == 20 and s[3, 4] == -8 and s[4, 5] == -8
    assert s[3, 3] == 2 and s[5, 3] == 2 and s[2, 4] == 1 and s[4, 6] == 1
    assert np.count_nonzero(s) == 13
    # 3-D: centre 42, face -12, edge-diagonal 2, distance-2 1; 25 points
    e = np.zeros((9, 9, 9))
    e[4, 4, 4] = 1.0
    s = reg_apply_BtB(e, "curvature", 1.0, 3)
    assert s[4, 4, 4] == 42 and s[3, 4, 4] == -12 and s[4, 3, 5] == 2
    assert s[4, 4, 2] == 1 and np.count_nonzero(s) == 25
    # diffusion: the 5-point Laplacian
    e = np.zeros((5, 5))
    e[2, 2] = 1.0
    s = reg_apply_BtB(e, "diffusion", 1.0, 2)
    assert s[2, 2] == 4 and s[1, 2] == -1 and np.count_nonzero(s) == 5


@pytest.mark.parametrize("reg", ["diffusion", "curvature"])
def test_regulariser_null_space(reg):
    c = np.full((2, 6, 7), 1.7)
    assert reg_value(c, reg, 1.0, 2) == 0.0
    assert np.all(reg_apply_BtB(c, reg, 1.0, 2) == 0.0)


def _dense_H(dW, h, par):
    shape = dW.shape
    N = dW.size
    H = np.zeros((N, N))
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1.0
        H[:, i] = hessvec(dW, e.reshape(shape), h, par).ravel()
    return H


@pytest.mark.parametrize("reg", ["diffusion", "curvature"])
def test_hessvec_against_fd_jacobian(reg):
    """2 h^d J^T J from a finite-difference residual Jacobian, plus the
    quadratic regulariser and penalty Hessians from the sparse operators."""
    shape = (4, 5)
    n, d, h = 3, 2, 2.0
    frames = _frames(n, shape, 8)
    u = _offkink_u(n, shape, h, 9)
    K = [0, 1, 2]
    par = ModelParams(alpha=0.4, lam=0.3, reg=reg)
    o = objective(frames, u, K, h, par)
    N = u.size

    def resid(uu):
        W = np.stack([interp_with_grad(frames[k], uu[k], h)[0] for k in K])
        return (W - W.mean(axis=0)).ravel()

    eps = 1e-6
    Jr = np.zeros((resid(u).size, N))
    for i in range(N):
        up = u.copy().ravel()
        um = u.copy().ravel()
        up[i] += eps
        um[i] -= eps
        Jr[:, i] = (resid(up.reshape(u.shape)) -
                    resid(um.reshape(u.shape))) / (2 * eps)
    Bd, L = _kron_ops(shape)
    B = Bd / h if reg == "diffusion" else L / h**2
    BtB = (B.T @ B).toarray()
    Hreg = sp.kron(sp.identity(n * d), BtB).toarray() * par.alpha * h**d
    # penalty: lambda h^d sum_x |mean_k u_k|^2 -> 2 lambda h^d / n^2 per pair
    Pm = np.kron(np.ones((n, n)), np.identity(d * np.prod(shape)))
    Hpen = 2 * par.lam * h**d / n**2 * Pm
    H_ref = 2 * h**d * Jr.T @ Jr + Hreg + Hpen
    H = _dense_H(o["dW"], h, par)
    np.testing.assert_allclose(H, H_ref, atol=1e-6 * np.abs(H_ref).max())
    # symmetric positive definite
    np.testing.assert_allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    assert np.linalg.eigvalsh(H).min() > 0
    # Jacobi diagonal
    np.testing.assert_allclose(jacobi_diag(o["dW"], h, par).ravel(),
                               np.diag(H), rtol=1e-12)


def test_hessvec_symmetry_3d():
    shape = (3, 4, 3)
    rng = np.random.default_rng(10)
    dW = rng.standard_normal((4, 3) + shape)
    par = ModelParams(alpha=0.2, lam=0.1, reg="curvature")
    v = rng.standard_normal(dW.shape)
    w = rng.standard_normal(dW.shape)
    a = np.sum(w * hessvec(dW, v, 2.0, par))
    b = np.sum(hessvec(dW, w, 2.0, par) * v)
    assert a == pytest.approx(b, rel=1e-12)
    assert np.sum(v * hessvec(dW, v, 2.0, par)) > 0
