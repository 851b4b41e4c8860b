"""Groupwise objective, gradient, Gauss-Newton Hessian product (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

The paper's objective (Sec. 2, eq. (1)) over a frame subset K is

    J(Y) = sum_{i in K} sum_{j in K} D(R_i o y_i, R_j o y_j) + S(Y) + P(Y),
    P(Y) = lambda * || (1/|K|) sum_{j in K} y_j - Id ||^2.

The paper's experiments use an affine model with a correlation distance; the
non-parametric instance computed here (the same one the HIP path computes)
takes, with W_k = R_k o (x + u_k) on a cell-centred grid of width h in d
dimensions:

* D: sum of squared differences over all ordered pairs, normalised by
  1/(2|K|) so that the data weight of one frame does not grow with |K|:
      D = h^d/(2|K|) sum_{i,j in K} ||W_i - W_j||^2 = h^d sum_k ||W_k - Wbar||^2
  (for |K| = 2 this is the usual pair SSD (h^d/2)||W_1 - W_2||^2).
* S = (alpha/2) h^d sum_{k in K} sum_c ||B u_k^c||^2 with
    diffusion: B = forward differences across interior faces / h,
    curvature: B = L / h^2, L the Neumann graph Laplacian of the grid
               (diagonal = -(number of in-grid neighbours), neighbours = 1).
* P = lambda h^d sum_x ||ubar(x)||^2, ubar = (1/|K|) sum_{k in K} u_k
  (y_k = x + u_k, so mean(y) - Id = ubar).

Gradient:  g_k = 2 h^d (W_k - Wbar) dW_k + alpha h^d B^T B u_k
                 + (2 lambda h^d / |K|) ubar.
Gauss-Newton Hessian (second derivatives of the images dropped):
    (H v)_k = 2 h^d dW_k (s_k - sbar) + alpha h^d B^T B v_k
              + (2 lambda h^d / |K|) vbar,   s_k = dW_k . v_k.
Jacobi diagonal:
    M = 2 h^d (1 - 1/|K|) (d_c W_k)^2 + alpha h^d diag(B^T B)
        + 2 lambda h^d / |K|^2.
"""

from dataclasses import dataclass

import numpy as np

from .warp import interp_with_grad


@dataclass
class ModelParams:
    alpha: float = 1e-2          # regulariser weight
    lam: float = 1e-2            # penalty weight lambda (Sec. 2)
    reg: str = "diffusion"       # "diffusion" or "curvature"


def _spatial_axes(v, d):
    return tuple(range(v.ndim - d, v.ndim))


def neumann_laplacian(v, d):
    """Graph Laplacian of the grid on the last d axes, Neumann boundary.

    (L v)_i = sum over in-grid neighbours j of (v_j - v_i).
    """
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    for ax in _spatial_axes(v, d):
        m = v.shape[ax]
        if m < 2:
            continue
        lo = [slice(None)] * v.ndim
        hi = [slice(None)] * v.ndim
        lo[ax] = slice(0, m - 1)
        hi[ax] = slice(1, m)
        diff = v[tuple(hi)] - v[tuple(lo)]      # v_{i+1} - v_i on faces
        out[tuple(lo)] += diff
        out[tuple(hi)] -= diff
    return out


def _forward_diffs(v, d):
    outs = []
    for ax in _spatial_axes(v, d):
        m = v.shape[ax]
        if m < 2:
            continue
        lo = [slice(None)] * v.ndim
        hi = [slice(None)] * v.ndim
        lo[ax] = slice(0, m - 1)
        hi[ax] = slice(1, m)
        outs.append(v[tuple(hi)] - v[tuple(lo)])
    return outs


def reg_value(v, reg, h, d):
    """sum ||B v||^2 over the last d axes (and any leading axes)."""
    v = np.asarray(v, dtype=np.float64)
    if reg == "diffusion":
        return sum(float(np.sum(f * f)) for f in _forward_diffs(v, d)) / h**2
    if reg == "curvature":
        Lv = neumann_laplacian(v, d)
        return float(np.sum(Lv * Lv)) / h**4
    raise ValueError(reg)


def reg_apply_BtB(v, reg, h, d):
    """B^T B v on the last d axes."""
    if reg == "diffusion":
        return -neumann_laplacian(v, d) / h**2
    if reg == "curvature":
        return neumann_laplacian(neumann_laplacian(v, d), d) / h**4
    raise ValueError(reg)


def reg_diag(extent, reg, h):
    """Diagonal of B^T B for one scalar field on ``extent``."""
    deg = np.zeros(extent)
    for a, m in enumerate(extent):
        idx = np.arange(m)
        nb = (idx > 0).astype(np.float64) + (idx < m - 1).astype(np.float64)
        shape = [1] * len(extent)
        shape[a] = m
        deg = deg + nb.reshape(shape)
    if reg == "diffusion":
        return deg / h**2
    if reg == "curvature":
        return (deg * deg + deg) / h**4
    raise ValueError(reg)


def _warp_set(frames, u, K, h):
    W, dW = [], []
    for k in K:
        w, dw = interp_with_grad(frames[k], u[k], h)
        W.append(w)
        dW.append(dw)
    return np.stack(W), np.stack(dW)


def objective(frames, u, K, h, params, with_grad=True):
    """Evaluate J = D + S + P over subset K, with gradient.

    frames : (n, *extent) images of this level.
    u      : (n, d, *extent) displacement of every frame; only K is used.
    K      : list of frame indices.
    Returns dict with J, D, S, P (floats) and, if with_grad, g and dW of
    shape (|K|, d, *extent) in the order of K.
    """
    frames = np.asarray(frames, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    d = frames.ndim - 1
    nk = len(K)
    hd = h ** d
    uK = u[list(K)]
    W, dW = _warp_set(frames, u, K, h)
    Wbar = W.mean(axis=0)
    r = W - Wbar
    D = hd * float(np.sum(r * r))
    S = 0.5 * params.alpha * hd * reg_value(uK, params.reg, h, d)
    ubar = uK.mean(axis=0)
    P = params.lam * hd * float(np.sum(ubar * ubar))
    out = {"J": D + S + P, "D": D, "S": S, "P": P}
    if with_grad:
        g = 2.0 * hd * r[:, None] * dW
        g = g + params.alpha * hd * reg_apply_BtB(uK, params.reg, h, d)
        g = g + (2.0 * params.lam * hd / nk) * ubar[None]
        out["g"] = g
        out["dW"] = dW
    return out


def objective_value(frames, u, K, h, params):
    """(J, D, S, P) over subset K, no gradient."""
    o = objective(frames, u, K, h, params, with_grad=False)
    return o["J"], o["D"], o["S"], o["P"]


def hessvec(dW, v, h, params):
    """Gauss-Newton Hessian times v; dW and v have shape (|K|, d, *extent)."""
    dW = np.asarray(dW, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    nk = v.shape[0]
    d = v.shape[1]
    hd = h ** d
    s = np.sum(dW * v, axis=1)                    # (|K|, *extent)
    sbar = s.mean(axis=0)
    vbar = v.mean(axis=0)
    Hv = 2.0 * hd * dW * (s - sbar)[:, None]
    Hv = Hv + params.alpha * hd * reg_apply_BtB(v, params.reg, h, d)
    Hv = Hv + (2.0 * params.lam * hd / nk) * vbar[None]
    return Hv


def jacobi_diag(dW, h, params):
    """Diagonal of the Gauss-Newton Hessian; shape (|K|, d, *extent)."""
    dW = np.asarray(dW, dtype=np.float64)
    nk = dW.shape[0]
    d = dW.shape[1]
    hd = h ** d
    ext = dW.shape[2:]
    M = 2.0 * hd * (1.0 - 1.0 / nk) * dW * dW
    M = M + params.alpha * hd * reg_diag(ext, params.reg, h)
    M = M + 2.0 * params.lam * hd / nk ** 2
    return M
