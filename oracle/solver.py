"""Jacobi-preconditioned CG and Gauss-Newton with Armijo search (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

The paper minimises eq. (1) with L-BFGS (Sec. 2) and states that any
numerical optimisation scheme can be used.  The non-parametric instance here
uses Gauss-Newton: each iteration solves H delta = -g approximately by
Jacobi-preconditioned conjugate gradients started at 0, then takes the first
step t in {1, 1/2, ..., 2^-ls_max} that meets the Armijo condition
J(x + t delta) <= J(x) + c1 t g.delta.

``gn_minimise`` is that iteration for any model that supplies J, g, a
Gauss-Newton Hessian product and its diagonal; ``gauss_newton`` applies it to
the registration objective of ``objective.py`` over the frames of K.

``fixed=True`` (parity mode) runs exactly ``gn_max`` Gauss-Newton and
``cg_max`` CG iterations with no convergence exits; only the exact-zero and
breakdown guards below stop early, and they are the same on the HIP path.
"""

from dataclasses import dataclass, field

import numpy as np

from .objective import objective, objective_value, hessvec, jacobi_diag


def pcg(apply_H, diag, b, cg_max, rtol=0.1, fixed=False):
    """Solve H x = b from x = 0 with the Jacobi preconditioner ``diag``.

    Returns (x, iterations, status); status is "ok" or "breakdown"
    (p.Hp <= 0, the last iterate is kept).  Stops early when r.z becomes
    exactly 0, and, unless ``fixed``, when ||r|| <= rtol ||r_0||.
    """
    x = np.zeros_like(b)
    r = b.copy()
    z = r / diag
    p = z.copy()
    rz = float(np.sum(r * z))
    r0 = float(np.sqrt(np.sum(r * r)))
    iters = 0
    if rz == 0.0:
        return x, iters, "ok"
    for _ in range(cg_max):
        q = apply_H(p)
        pq = float(np.sum(p * q))
        if not pq > 0.0:
            return x, iters, "breakdown"
        a = rz / pq
        x = x + a * p
        r = r - a * q
        iters += 1
        z = r / diag
        rz_new = float(np.sum(r * z))
        if not fixed and float(np.sqrt(np.sum(r * r))) <= rtol * r0:
            break
        if rz_new == 0.0:
            break
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
    return x, iters, "ok"


def armijo(value, J, slope, ls_max=10, c1=1e-4):
    """First t in {1, 1/2, ..., 2^-ls_max} with value(t) <= J + c1 t slope.

    Returns (t, value(t)) or (None, last value tried) if none qualifies.
    """
    t = 1.0
    Jt = J
    for _ in range(ls_max + 1):
        Jt = value(t)
        if Jt <= J + c1 * t * slope:
            return t, Jt
        t *= 0.5
    return None, Jt


@dataclass
class GNResult:
    u: np.ndarray
    J0: float
    J: float
    iterations: int
    cg_iterations: list = field(default_factory=list)
    steps: list = field(default_factory=list)      # accepted t per iteration
    J_history: list = field(default_factory=list)
    status: str = "ok"


def gn_minimise(model, x0, gn_max=10, cg_max=20, cg_rtol=0.1, ls_max=10,
                c1=1e-4, fixed=False, tol_J=1e-3, tol_u=1e-2):
    """Gauss-Newton with Jacobi-PCG directions and the Armijo search.

    ``model`` supplies ``evaluate(x) -> (J, g, state)``, ``value(x) -> J``,
    ``hessvec(state, v)`` and ``diag(state)``.  Unless ``fixed``, stop once
    an accepted step lowers J by at most tol_J |J| and the root mean square
    of the accepted step t delta is at most tol_u.  Returns a GNResult whose
    ``u`` is the final x.
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    res = GNResult(u=x, J0=float("nan"), J=float("nan"), iterations=0)
    for it in range(gn_max):
        J, g, state = model.evaluate(x)
        if it == 0:
            res.J0 = J
            res.J = J
        delta, cgi, st = pcg(lambda v: model.hessvec(state, v),
                             model.diag(state), -g, cg_max, cg_rtol, fixed)
        res.cg_iterations.append(cgi)
        if st != "ok":
            res.status = st
        slope = float(np.sum(g * delta))
        t, Jt = armijo(lambda s: model.value(x + s * delta), J, slope,
                       ls_max, c1)
        if t is None:
            res.status = "linesearch"
            break
        x = x + t * delta
        res.iterations += 1
        res.steps.append(t)
        res.J_history.append(Jt)
        res.J = Jt
        if st == "breakdown":
            break
        if not fixed:
            if (J - Jt) <= tol_J * abs(J) and \
                    t * float(np.sqrt(np.mean(delta * delta))) <= tol_u:
                break
    res.u = x
    return res


class _GroupRegistration:
    """Eq. (1) instance of ``objective.py`` as a function of u on K only."""

    def __init__(self, frames, u, K, h, params):
        self.frames, self.K, self.h, self.params = frames, list(K), h, params
        self.u = np.array(u, dtype=np.float64, copy=True)

    def _full(self, uK):
        full = self.u.copy()
        full[self.K] = uK
        return full

    def evaluate(self, uK):
        o = objective(self.frames, self._full(uK), self.K, self.h,
                      self.params, with_grad=True)
        return o["J"], o["g"], o["dW"]

    def value(self, uK):
        return objective_value(self.frames, self._full(uK), self.K, self.h,
                               self.params)[0]

    def hessvec(self, dW, v):
        return hessvec(dW, v, self.h, self.params)

    def diag(self, dW):
        return jacobi_diag(dW, self.h, self.params)


def gauss_newton(frames, u0, K, h, params, gn_max=10, cg_max=20,
                 cg_rtol=0.1, ls_max=10, c1=1e-4, fixed=False,
                 tol_J=1e-3, tol_u=1e-2):
    """Minimise J over the frames in K, starting from u0 (all n frames).

    Frames outside K keep their displacement.  The stop test's step norm is
    the root mean square over the moved displacements, in finest pixels: the
    paper leaves the optimiser's tests to FAIR, whose tests are relative and
    norm-based; a maximum over voxels is not used because single voxels near
    interpolation kinks can keep moving.
    """
    K = list(K)
    model = _GroupRegistration(frames, u0, K, h, params)
    res = gn_minimise(model, model.u[K], gn_max, cg_max, cg_rtol, ls_max, c1,
                      fixed, tol_J, tol_u)
    res.u = model._full(res.u)
    return res
