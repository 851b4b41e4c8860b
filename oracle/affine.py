"""Affine-linear groupwise registration with the SqN distance and L-BFGS
(oracle).

Test infrastructure only (see ``oracle/__init__.py``).

The paper's experiments register every frame by an affine-linear map
(Sec. 4), measure the distance with the correlation-based SqN measure it
cites (Sec. 2, eq. (1)), penalise the mean transformation (Sec. 2, P) and
minimise with L-BFGS (Sec. 2).  Readings (the same bind the HIP path):

* Map.  y_k(x) = x + u_k(x), u_k(x) = B_k xi(x) + b_k with
  xi(x) = (x - c) / R, c the centre of the finest grid and R half its
  largest side (physical units, finest h = 1).  The parameters
  theta_k = (B_k row-major, b_k) (p = d^2 + d numbers) are all in pixels
  (B_k is the displacement at distance R from the centre), identity is 0,
  and the same parameters mean the same map on every spatial level.
* Distance.  Eq. (1) sums D over ordered pairs; with the correlation
  based pair distance D(W_i, W_j) = 1 - rho_ij^2, rho_ij the correlation
  coefficient of the warped frames over the grid,
      D = sum_{i,j in K} (1 - rho_ij^2) = |K|^2 - ||M||_S4^4,
  where M holds the frames centred and scaled to unit norm as columns and
  ||M||_S4 is its Schatten 4-norm (sum of the fourth powers of its singular
  values), i.e. the SVD based SqN measure with q = 4.  D is 0 exactly when
  every pair is perfectly correlated and does not change under an affine
  change of intensity of any frame.
* Regulariser.  None (the paper's S sentence is garbled; an affine map
  needs no smoother).
* Penalty.  P = lambda h^d sum_x ||ubar(x)||^2, ubar = mean_k u_k over K
  (mean(y) - Id = ubar), as for the non-parametric model.
* Optimiser.  L-BFGS (two-loop recursion, the last ``mem`` pairs with
  s.y > 1e-10 |s| |y|, initial matrix gamma I with gamma = s.y / y.y of the
  newest pair; before any pair the direction is -g / max|g|, a first step of
  at most one pixel per parameter), the Armijo search of the Gauss-Newton
  solver (t = 1, 1/2, ..., 2^-ls_max, c1), the same stop test (relative
  decrease of J and root mean square of the accepted step, in pixels), and
  a fixed iteration count in parity mode.
"""

from dataclasses import dataclass

import numpy as np

from .warp import interp_with_grad
from .grid import level_extents, level_spacing, temporal_sets, restrict
from .predictor import linear_predict, ls_predict
from .solver import armijo


def n_params(d):
    return d * d + d


def frame_geometry(ext_finest, ext, h):
    """xi(x) of every voxel of a level: array (d, *ext)."""
    d = len(ext)
    c = np.array([m / 2.0 for m in ext_finest])
    R = max(ext_finest) / 2.0
    axes = [((np.arange(m) + 0.5) * h - c[a]) / R for a, m in enumerate(ext)]
    return np.stack(np.meshgrid(*axes, indexing="ij"))


def displacement(theta, xi):
    """u(x) = B xi(x) + b for one frame; theta (p,), xi (d, *ext)."""
    d = xi.shape[0]
    B = np.asarray(theta[:d * d], np.float64).reshape(d, d)
    b = np.asarray(theta[d * d:], np.float64)
    return np.tensordot(B, xi, axes=(1, 0)) + b.reshape((d,) + (1,) * d)


def sqn_value(W):
    """D = sum_{i,j} (1 - rho_ij^2) over the rows of W (|K|, N): the pair
    sum of eq. (1)."""
    C = W - W.mean(axis=1, keepdims=True)
    s = np.sqrt(np.sum(C * C, axis=1))
    M = C / s[:, None]
    G = M @ M.T
    return float(np.sum(1.0 - G * G)), G, M, s


@dataclass
class AffineParams:
    lam: float = 1e-3


def objective(frames, theta, K, h, ext_finest, params, with_grad=True):
    """J = D_SqN + P over the frames K at parameters theta (n, p).

    Returns dict J, D, P and, with_grad, g of shape (|K|, p) in the order of
    K (rows: d(B row-major), d(b)).
    """
    frames = np.asarray(frames, np.float64)
    theta = np.asarray(theta, np.float64)
    K = list(K)
    ext = frames.shape[1:]
    d = len(ext)
    hd = h ** d
    xi = frame_geometry(ext_finest, ext, h)
    W, dW = [], []
    for k in K:
        w, dw = interp_with_grad(frames[k], displacement(theta[k], xi), h)
        W.append(w.ravel())
        dW.append(dw.reshape(d, -1))
    W = np.stack(W)
    D, G, M, s = sqn_value(W)
    ubar = np.mean([displacement(theta[k], xi) for k in K], axis=0)
    P = params.lam * hd * float(np.sum(ubar * ubar))
    out = {"J": D + P, "D": D, "P": P}
    if not with_grad:
        return out
    nk = len(K)
    # dD/dW_i = -(4 / s_i) [(M^T G)_i - (G^2)_ii m_i]: D depends on W_i
    # through m_i = centred W_i / s_i; the projection removes the part along
    # m_i (the norm is fixed) and the mean (every m_b has zero mean)
    MG = G @ M
    G2 = np.sum(G * G, axis=1)
    r = -(4.0 / s)[:, None] * (MG - G2[:, None] * M)
    xi_f = xi.reshape(d, -1)
    g = np.zeros((nk, n_params(d)))
    for j in range(nk):
        rd = r[j][None, :] * dW[j]                      # (d, N)
        g[j, :d * d] = (rd @ xi_f.T).ravel()            # dD/dB[a][e]
        g[j, d * d:] = rd.sum(axis=1)                   # dD/db[a]
    # penalty: dP/dtheta_k = (1/|K|) dP/dthetabar
    ub = ubar.reshape(d, -1)
    gp = np.zeros(n_params(d))
    gp[:d * d] = (2.0 * params.lam * hd * (ub @ xi_f.T)).ravel()
    gp[d * d:] = 2.0 * params.lam * hd * ub.sum(axis=1)
    out["g"] = g + gp[None, :] / nk
    return out


def objective_value(frames, theta, K, h, ext_finest, params):
    o = objective(frames, theta, K, h, ext_finest, params, with_grad=False)
    return o["J"], o["D"], o["P"]


def lbfgs_direction(g, S, Y, gamma):
    """-H g by the two-loop recursion over the pairs (S[i], Y[i]) (oldest
    first), with the initial matrix gamma I."""
    q = np.array(g, np.float64, copy=True)
    rhos = [1.0 / float(np.sum(s * y)) for s, y in zip(S, Y)]
    alphas = []
    for s, y, rho in reversed(list(zip(S, Y, rhos))):
        a = rho * float(np.sum(s * q))
        alphas.append(a)
        q = q - a * y
    r = gamma * q
    for (s, y, rho), a in zip(zip(S, Y, rhos), reversed(alphas)):
        b = rho * float(np.sum(y * r))
        r = r + (a - b) * s
    return -r


@dataclass
class LBFGSResult:
    x: np.ndarray
    J0: float
    J: float
    iterations: int
    steps: list
    J_history: list
    pairs: list            # pairs kept after each iteration
    status: str = "ok"


def lbfgs_minimise(model, x0, max_iter=10, mem=5, ls_max=10, c1=1e-4,
                   fixed=False, tol_J=1e-3, tol_u=1e-2):
    """L-BFGS with the Armijo search; ``model`` supplies
    ``evaluate(x) -> (J, g)`` and ``value(x) -> J``."""
    x = np.array(x0, np.float64, copy=True)
    J, g = model.evaluate(x)
    res = LBFGSResult(x=x, J0=J, J=J, iterations=0, steps=[],
                      J_history=[], pairs=[])
    S, Y = [], []
    for _ in range(max_iter):
        if S:
            gamma = float(np.sum(S[-1] * Y[-1]) / np.sum(Y[-1] * Y[-1]))
            d = lbfgs_direction(g, S, Y, gamma)
        else:
            gmax = float(np.max(np.abs(g)))
            if gmax == 0.0:
                d = np.zeros_like(g)
            else:
                d = -g / gmax
        slope = float(np.sum(g * d))
        if not slope < 0.0 and S:           # not a descent direction: restart
            S, Y = [], []
            gmax = float(np.max(np.abs(g)))
            d = -g / gmax if gmax > 0 else np.zeros_like(g)
            slope = float(np.sum(g * d))
        t, Jt = armijo(lambda s: model.value(x + s * d), J, slope, ls_max,
                       c1)
        if t is None:
            res.status = "linesearch"
            break
        x_new = x + t * d
        J_new, g_new = model.evaluate(x_new)
        s_vec, y_vec = x_new - x, g_new - g
        sy = float(np.sum(s_vec * y_vec))
        if sy > 1e-10 * float(np.linalg.norm(s_vec) * np.linalg.norm(y_vec)):
            S.append(s_vec)
            Y.append(y_vec)
            if len(S) > mem:
                S.pop(0)
                Y.pop(0)
        step_rms = t * float(np.sqrt(np.mean(d * d)))
        x, g, J_prev, J = x_new, g_new, J, J_new
        res.iterations += 1
        res.steps.append(t)
        res.J_history.append(J)
        res.pairs.append(len(S))
        res.J = J
        if not fixed and (J_prev - J) <= tol_J * abs(J_prev) and \
                step_rms <= tol_u:
            break
    res.x = x
    return res


class _AffineGroup:
    """J of one level over the frames K as a function of theta[K] (flat)."""

    def __init__(self, frames, theta, K, h, ext_finest, params):
        self.frames, self.K, self.h = frames, list(K), h
        self.ext_finest, self.params = ext_finest, params
        self.theta = np.array(theta, np.float64, copy=True)
        self.p = self.theta.shape[1]

    def full(self, xK):
        th = self.theta.copy()
        th[self.K] = xK.reshape(len(self.K), self.p)
        return th

    def evaluate(self, xK):
        o = objective(self.frames, self.full(xK), self.K, self.h,
                      self.ext_finest, self.params)
        return o["J"], o["g"].ravel()

    def value(self, xK):
        return objective_value(self.frames, self.full(xK), self.K, self.h,
                               self.ext_finest, self.params)[0]


def register(frames, theta0, K, h, ext_finest, params, **kw):
    """L-BFGS on the parameters of the frames K; the others keep theta0."""
    m = _AffineGroup(frames, theta0, K, h, ext_finest, params)
    res = lbfgs_minimise(m, m.theta[list(K)].ravel(), **kw)
    res.x = m.full(res.x)
    return res


@dataclass
class AffineSTMLOptions:
    n_spatial: int = 2
    n_temporal: int = 2
    lam: float = 1e-3
    beta: float = 1e-5
    eps_stop: float = 0.0
    stop_relative: bool = False
    iter_max: int = 10
    mem: int = 5
    ls_max: int = 10
    c1: float = 1e-4
    tol_J: float = 1e-3
    tol_u: float = 1e-2
    parity_mode: bool = False


class AffineSTMLState:
    """Sec. 3's schedule on affine parameters (n, p) per level: the same
    parameters on every spatial level (physical coordinates), so the
    spatial transfer copies them; linear interpolation on the coarsest
    level and eq. (2) on finer ones act on each parameter; eq. (3) on D
    over all frames."""

    def __init__(self, frames, opts):
        frames = np.asarray(frames)
        self.opts = opts
        self.n = frames.shape[0]
        self.d = frames.ndim - 1
        self.ext_finest = frames.shape[1:]
        self.extents = level_extents(frames.shape[1:], opts.n_spatial)
        pyr = [np.asarray(frames, np.float64)]
        for _ in range(opts.n_spatial - 1):
            pyr.append(restrict(pyr[-1]))
        self.pyramid = pyr[::-1]
        self.K = temporal_sets(self.n, opts.n_temporal)
        self.Y = [None] * opts.n_spatial
        self.Z = [None] * opts.n_spatial
        self.log = []
        self.stop_trace = [[] for _ in range(opts.n_spatial)]
        self.stop_q = [-1] * opts.n_spatial

    def h(self, level):
        return level_spacing(self.opts.n_spatial, level)

    def predict(self, level, q_next):
        o = self.opts
        if q_next == 0:
            z = np.zeros((self.n, n_params(self.d))) if level == 0 else \
                self.Y[level - 1].copy()
        elif level == 0:
            z = linear_predict(self.Y[level], self.K[q_next - 1])
        else:
            z = ls_predict(self.Y[level], self.Z[level], self.K[q_next - 1],
                           o.beta)
        self.Z[level] = z
        self.Y[level] = z.copy()

    def register_level(self, level, q):
        o = self.opts
        res = register(self.pyramid[level], self.Y[level], self.K[q],
                       self.h(level), self.ext_finest, AffineParams(o.lam),
                       max_iter=o.iter_max, mem=o.mem, ls_max=o.ls_max,
                       c1=o.c1, fixed=o.parity_mode, tol_J=o.tol_J,
                       tol_u=o.tol_u)
        self.Y[level] = res.x
        self.log.append({"level": level, "q": q, "nK": len(self.K[q]),
                         "iters": res.iterations, "steps": res.steps,
                         "J0": res.J0, "J": res.J, "status": res.status})
        return res

    correct = register_level

    def all_frame_D(self, level, theta):
        return objective_value(self.pyramid[level], theta, range(self.n),
                               self.h(level), self.ext_finest,
                               AffineParams(self.opts.lam))[1]

    def run(self):
        o = self.opts
        for level in range(o.n_spatial):
            self.predict(level, 0)
            self.register_level(level, 0)
            D_prev = None
            for q in range(o.n_temporal - 1):
                Kq = self.K[q]
                y_now = self.Y[level].copy()
                self.predict(level, q + 1)
                if o.eps_stop > 0 and not o.parity_mode:
                    est = self.Y[level].copy()
                    est[Kq] = y_now[Kq]
                    Dq = self.all_frame_D(level, est)
                    self.stop_trace[level].append(Dq)
                    tol = o.eps_stop * (abs(Dq) if o.stop_relative else 1.0)
                    if D_prev is not None and abs(Dq - D_prev) <= tol:
                        self.Y[level] = est
                        self.stop_q[level] = q
                        break
                    D_prev = Dq
                self.correct(level, q + 1)
        return self.Y[-1]


def affine_stml_run(frames, opts):
    st = AffineSTMLState(frames, opts)
    return st.run(), st
