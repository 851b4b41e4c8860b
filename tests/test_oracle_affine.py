"""Pins of the affine-linear SqN / L-BFGS oracle (Sec. 2, Sec. 4).

Independent checks: the pair sum of eq. (1) with 1 - rho^2 against the
Schatten 4-norm from numpy.linalg.svd and against numpy.corrcoef; invariance
of the distance under affine intensity changes; the gradient by central
finite differences (2-D and 3-D); the penalty against its closed form for
a translation; the two-loop recursion against the dense BFGS update of the
inverse Hessian; L-BFGS against numpy.linalg.solve on a quadratic; exact
recovery of integer translations and close recovery of a smooth affine
motion; the schedule against hand-written loops.
"""

import numpy as np
import pytest

from oracle import affine as af
from oracle import (restrict, temporal_sets, linear_predict, ls_predict,
                    level_spacing)
from paper_2001_06613_amd import synth


def test_displacement_and_geometry():
    ext = (6, 8)
    xi = af.frame_geometry(ext, ext, 1.0)
    assert xi.shape == (2, 6, 8)
    # centred: cell centres are symmetric about the middle of the grid
    np.testing.assert_allclose(xi[0] + xi[0][::-1], 0.0, atol=1e-15)
    np.testing.assert_allclose(xi[1] + xi[1][:, ::-1], 0.0, atol=1e-15)
    # R = half the largest side (4): the outermost centre of the 8-wide axis
    # is 3.5 pixels from the middle
    assert np.max(np.abs(xi[1])) == pytest.approx((8 / 2 - 0.5) / 4.0)
    theta = np.zeros(6)
    assert np.all(af.displacement(theta, xi) == 0)
    theta[4:] = [1.5, -2.0]
    u = af.displacement(theta, xi)
    assert np.all(u[0] == 1.5) and np.all(u[1] == -2.0)
    theta[:] = [1, 2, 3, 4, 0, 0]
    u = af.displacement(theta, xi)
    np.testing.assert_allclose(u[0], 1 * xi[0] + 2 * xi[1])
    np.testing.assert_allclose(u[1], 3 * xi[0] + 4 * xi[1])
    # a coarser level (h = 2) of the same domain gives the same physical map
    xc = af.frame_geometry(ext, (3, 4), 2.0)
    np.testing.assert_allclose(xc[1][0], 0.5 * (xi[1][0, ::2] + xi[1][0, 1::2]))


def test_sqn_pair_sum_is_schatten4_and_corrcoef():
    rng = np.random.default_rng(0)
    base = rng.standard_normal(200)
    W = np.stack([base + 0.3 * rng.standard_normal(200) for _ in range(5)])
    D, G, M, s = af.sqn_value(W)
    sv = np.linalg.svd(M, compute_uv=False)
    assert D == pytest.approx(25.0 - float(np.sum(sv ** 4)), rel=1e-12)
    rho = np.corrcoef(W)
    assert D == pytest.approx(float(np.sum(1.0 - rho ** 2)), rel=1e-12)
    np.testing.assert_allclose(G, rho, atol=1e-14)
    # two frames: 2 (1 - rho^2)
    D2 = af.sqn_value(W[:2])[0]
    assert D2 == pytest.approx(2.0 * (1.0 - rho[0, 1] ** 2), rel=1e-12)


def test_sqn_invariant_under_intensity_affine_maps():
    rng = np.random.default_rng(1)
    W = rng.standard_normal((4, 150))
    D0 = af.sqn_value(W)[0]
    a = np.array([2.0, -0.5, 7.0, 0.1])[:, None]
    c = np.array([3.0, -1.0, 0.0, 10.0])[:, None]
    assert af.sqn_value(a * W + c)[0] == pytest.approx(D0, rel=1e-12)
    # perfectly correlated frames: D = 0 (up to rounding)
    same = a * W[:1] + c
    assert abs(af.sqn_value(same)[0]) < 1e-12


def _fd_check(frames, theta, K, h, ext_f, par, eps=1e-6, tol=1e-6):
    o = af.objective(frames, theta, K, h, ext_f, par)
    g = o["g"]
    num = np.zeros_like(g)
    for j, k in enumerate(K):
        for i in range(theta.shape[1]):
            tp, tm = theta.copy(), theta.copy()
            tp[k, i] += eps
            tm[k, i] -= eps
            num[j, i] = (af.objective_value(frames, tp, K, h, ext_f, par)[0] -
                         af.objective_value(frames, tm, K, h, ext_f, par)[0]) \
                / (2 * eps)
    err = np.max(np.abs(num - g)) / np.max(np.abs(g))
    assert err < tol, err


def test_gradient_finite_differences_2d():
    rng = np.random.default_rng(2)
    frames = np.stack([synth.base_image(rng, (14, 12)) for _ in range(3)])
    frames = frames.astype(np.float32)
    theta = rng.uniform(-0.8, 0.8, (3, 6))
    _fd_check(frames, theta, [0, 1, 2], 1.0, (14, 12), af.AffineParams(0.05))
    # a coarse level of a larger finest grid, subset of frames
    _fd_check(frames, theta, [0, 2], 2.0, (28, 24), af.AffineParams(0.05))


def test_gradient_finite_differences_3d():
    rng = np.random.default_rng(3)
    frames = np.stack([synth.base_image(rng, (7, 6, 8)) for _ in range(2)])
    frames = frames.astype(np.float32)
    theta = rng.uniform(-0.5, 0.5, (2, 12))
    _fd_check(frames, theta, [0, 1], 1.0, (7, 6, 8), af.AffineParams(0.02))


def test_penalty_closed_form_for_translations():
    frames = np.ones((3, 5, 7), np.float32) + \
        np.arange(35, dtype=np.float32).reshape(5, 7)
    theta = np.zeros((3, 6))
    theta[:, 4:] = [[1.0, 2.0], [3.0, -1.0], [-0.5, 0.5]]
    lam, h = 0.3, 2.0
    o = af.objective(frames, theta, [0, 1, 2], h, (10, 14),
                     af.AffineParams(lam))
    bbar = theta[:, 4:].mean(axis=0)
    assert o["P"] == pytest.approx(lam * h * h * 35 * float(bbar @ bbar),
                                   rel=1e-13)


def _dense_bfgs(g, S, Y, gamma):
    """-H g with H built by the BFGS update of the inverse Hessian,
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T, from gamma I."""
    n = g.size
    H = gamma * np.identity(n)
    for s, y in zip(S, Y):
        rho = 1.0 / float(s @ y)
        V = np.identity(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return -H @ g


def test_two_loop_recursion_equals_dense_bfgs():
    rng = np.random.default_rng(4)
    n = 9
    A = rng.standard_normal((n, n))
    A = A @ A.T + n * np.identity(n)
    S = [rng.standard_normal(n) for _ in range(5)]
    Y = [A @ s for s in S]                  # s.y > 0
    g = rng.standard_normal(n)
    for m in (1, 3, 5):
        gamma = float(S[-1] @ Y[-1] / (Y[-1] @ Y[-1]))
        np.testing.assert_allclose(
            af.lbfgs_direction(g, S[-m:], Y[-m:], gamma),
            _dense_bfgs(g, S[-m:], Y[-m:], gamma), rtol=1e-11, atol=1e-12)


class _Quadratic:
    def __init__(self, A, b):
        self.A, self.b = A, b

    def value(self, x):
        return 0.5 * float(x @ self.A @ x) - float(self.b @ x)

    def evaluate(self, x):
        return self.value(x), self.A @ x - self.b


def test_lbfgs_minimises_quadratic():
    rng = np.random.default_rng(5)
    n = 12
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T / n + np.identity(n)
    b = rng.standard_normal(n)
    res = af.lbfgs_minimise(_Quadratic(A, b), np.zeros(n), max_iter=200,
                            mem=5, tol_J=0.0, tol_u=0.0, fixed=True)
    np.testing.assert_allclose(res.x, np.linalg.solve(A, b), rtol=1e-6,
                               atol=1e-8)
    # the first direction is -g / max|g|, and on this quadratic the unit
    # step is accepted: x1 = b / max|b|
    r1 = af.lbfgs_minimise(_Quadratic(A, b), np.zeros(n), max_iter=1,
                           fixed=True)
    assert r1.steps == [1.0]
    np.testing.assert_allclose(r1.x, b / np.max(np.abs(b)), rtol=1e-15)


def test_registration_recovers_integer_translations():
    shifts = np.array([[1.0, -1.0], [-1.0, 0.0], [0.0, 1.0]])   # sum 0
    frames = synth.translated_sequence(shifts, (32, 32), seed=1)
    theta0 = np.zeros((3, 6))
    res = af.register(frames, theta0, [0, 1, 2], 1.0, (32, 32),
                      af.AffineParams(1e-3), max_iter=60, tol_J=0.0,
                      tol_u=0.0)
    assert res.J < 1e-8
    np.testing.assert_allclose(res.x[:, 4:], shifts, atol=1e-3)
    np.testing.assert_allclose(res.x[:, :4], 0.0, atol=1e-3)


def _analytic(pts):
    """Smooth test image on physical points (d, ...): sum of Gaussians."""
    y, x = pts
    return (np.exp(-((x - 14) ** 2 + (y - 12) ** 2) / 30.0) +
            0.7 * np.exp(-((x - 22) ** 2 + (y - 20) ** 2) / 18.0) +
            0.5 * np.exp(-((x - 9) ** 2 + (y - 23) ** 2) / 12.0))


def test_registration_recovers_smooth_affine_motion():
    # frame k shows the image at x + u_k(x) with known affine u_k (mean 0);
    # registering frame k by y_k(x) = x + v_k(x) aligns all frames when
    # x + v_k(x) + u_k(x + v_k(x)) is the same map for every k; for small
    # motion v_k ~ -u_k + (common part fixed by the penalty)
    ext = (32, 32)
    xi = af.frame_geometry(ext, ext, 1.0)
    x = np.stack(np.meshgrid(np.arange(32) + 0.5, np.arange(32) + 0.5,
                             indexing="ij"))
    true = np.array([[0.6, -0.3, 0.2, 0.4, 0.8, -0.5],
                     [-0.4, 0.5, -0.3, -0.2, -1.0, 0.3],
                     [-0.2, -0.2, 0.1, -0.2, 0.2, 0.2]])
    frames = np.stack([_analytic(x + af.displacement(t, xi)) for t in true])
    res = af.register(frames.astype(np.float32), np.zeros((3, 6)), [0, 1, 2],
                      1.0, ext, af.AffineParams(1e-2), max_iter=100,
                      tol_J=0.0, tol_u=0.0)
    # composition of the two affine maps, to first order: v_k = -u_k
    for k in range(3):
        v = af.displacement(res.x[k], xi)
        u = af.displacement(true[k], xi)
        err = np.abs(v + u)[:, 6:-6, 6:-6].max()
        assert err < 0.1, (k, err)


def _tiny_seq(n=9):
    return synth.sinusoid_sequence(n, (24, 20), 1.5, 1, seed=8)[0]


def test_single_temporal_level_is_spatial_multilevel():
    frames = _tiny_seq()
    o = af.AffineSTMLOptions(n_spatial=2, n_temporal=1, iter_max=3,
                             parity_mode=True)
    u, st = af.affine_stml_run(frames, o)
    par = af.AffineParams(o.lam)
    allk = list(range(9))
    r0 = af.register(restrict(frames), np.zeros((9, 6)), allk, 2.0, (24, 20),
                     par, max_iter=3, fixed=True)
    r1 = af.register(frames, r0.x, allk, 1.0, (24, 20), par, max_iter=3,
                     fixed=True)
    np.testing.assert_array_equal(u, r1.x)


def test_hand_written_affine_schedule():
    frames = _tiny_seq()
    o = af.AffineSTMLOptions(n_spatial=2, n_temporal=3, iter_max=2,
                             parity_mode=True, beta=1e-3)
    u, st = af.affine_stml_run(frames, o)
    par = af.AffineParams(o.lam)
    Ks = temporal_sets(9, 3)
    pyr = [restrict(np.asarray(frames, np.float64)),
           np.asarray(frames, np.float64)]
    y = None
    for lvl in range(2):
        h = level_spacing(2, lvl)
        z = np.zeros((9, 6)) if lvl == 0 else y.copy()  # same parameters
        y = af.register(pyr[lvl], z, Ks[0], h, (24, 20), par, max_iter=2,
                        fixed=True).x
        for q in range(2):
            z = linear_predict(y, Ks[q]) if lvl == 0 else \
                ls_predict(y, z, Ks[q], o.beta)
            y = af.register(pyr[lvl], z, Ks[q + 1], h, (24, 20), par,
                            max_iter=2, fixed=True).x
    np.testing.assert_array_equal(u, y)
    assert [(e["level"], e["nK"]) for e in st.log] == \
        [(0, 3), (0, 5), (0, 9), (1, 3), (1, 5), (1, 9)]


def test_affine_eq3_trace_and_stop():
    frames = _tiny_seq()
    base = dict(n_spatial=1, n_temporal=3, iter_max=3, tol_J=0.0, tol_u=0.0)
    _, free = af.affine_stml_run(frames, af.AffineSTMLOptions(
        eps_stop=1e-300, **base))
    tr = free.stop_trace[0]
    assert len(tr) == 2 and free.stop_q == [-1]
    # the trace is D over all frames at the prediction (coarsest level:
    # linear interpolation, which keeps K_q as registered)
    st = af.AffineSTMLState(frames, af.AffineSTMLOptions(**base))
    st.predict(0, 0)
    st.register_level(0, 0)
    st.predict(0, 1)
    assert tr[0] == pytest.approx(st.all_frame_D(0, st.Y[0]), rel=1e-12)
    d = abs(tr[1] - tr[0])
    _, fire = af.affine_stml_run(frames, af.AffineSTMLOptions(
        eps_stop=2 * d, **base))
    assert fire.stop_q == [1]
    assert [e["nK"] for e in fire.log] == [3, 5]


def test_lbfgs_second_direction_uses_scaled_identity():
    # after one step the direction is the dense BFGS update of gamma I with
    # gamma = s.y / y.y (the newest pair), applied to the new gradient
    rng = np.random.default_rng(6)
    n = 8
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T / n + 0.5 * np.identity(n)
    b = rng.standard_normal(n)
    m = _Quadratic(A, b)
    r2 = af.lbfgs_minimise(m, np.zeros(n), max_iter=2, fixed=True)
    x1 = b / np.max(np.abs(b))
    s0, y0 = x1, A @ x1               # g0 = -b, g1 = A x1 - b
    g1 = A @ x1 - b
    d1 = _dense_bfgs(g1, [s0], [y0], float(s0 @ y0 / (y0 @ y0)))
    J1 = m.value(x1)
    t = 1.0
    while m.value(x1 + t * d1) > J1 + 1e-4 * t * float(g1 @ d1):
        t *= 0.5
    assert r2.steps[1] == t
    np.testing.assert_allclose(r2.x, x1 + t * d1, rtol=1e-13, atol=1e-15)
