"""Spatio-temporal multilevel (STML) driver (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 3 of the paper: spatial levels l run coarse to fine; on each level a
predictor-corrector loop walks the temporal tree K_0 ... K_T:

* l = coarsest, q = 0: register K_0 from the identity (u = 0).
* l > coarsest, q = 0: the start guess of every frame is the result of the
  previous spatial level, transferred to this grid (prolongation).
* q -> q + 1: predict all n frames from the registered frames of K_q
  (linear interpolation on the coarsest level, eq. (2) on finer ones), then
  correct by registering K_{q+1} from that prediction.
* optional stopping rule, eq. (3): after the prediction that follows the
  registration of K_q (q >= 1), stop the level if D over all frames, at the
  all-frame estimate, changed by at most eps from the previous one
  (|D_q - D_{q-1}| <= eps, as printed; ``stop_relative`` selects the test
  |D_q - D_{q-1}| <= eps |D_q| instead).  The all-frame estimate is the
  prediction for every frame, with the frames of K_q as registered.

Reading of eq. (2)'s reference omega: it is the all-frame start guess of the
current temporal level, z(l, q, all); for q = 0 that is the prolonged
result of the previous spatial level, which is the paper's choice for q = 0.

The class mirrors the C-ABI call sequence (set_sequence, predict,
register_level / correct, get_displacements) so tests can drive the oracle
and the HIP path through the same steps.
"""

from dataclasses import dataclass

import numpy as np

from .grid import level_extents, level_spacing, temporal_sets, restrict, \
    prolong
from .objective import ModelParams, objective_value
from .solver import gauss_newton
from .predictor import linear_predict, ls_predict


@dataclass
class STMLOptions:
    n_spatial: int = 2
    n_temporal: int = 2
    reg: str = "diffusion"
    alpha: float = 1e-2
    lam: float = 1e-2
    beta: float = 1e-5
    eps_stop: float = 0.0          # 0 disables eq. (3)
    stop_relative: bool = False    # eq. (3) as |dD| <= eps |D|
    gn_max: int = 10
    cg_max: int = 20
    cg_rtol: float = 0.1
    ls_max: int = 10
    c1: float = 1e-4
    tol_J: float = 1e-3
    tol_u: float = 1e-2
    parity_mode: bool = False      # fixed GN/CG counts, no early exits

    def params(self):
        return ModelParams(alpha=self.alpha, lam=self.lam, reg=self.reg)


class STMLState:
    """Oracle state for one sequence: image pyramid, Y and Z per level."""

    def __init__(self, frames, opts):
        frames = np.asarray(frames)
        self.opts = opts
        self.n = frames.shape[0]
        self.d = frames.ndim - 1
        self.extents = level_extents(frames.shape[1:], opts.n_spatial)
        pyr = [np.asarray(frames, dtype=np.float64)]
        for _ in range(opts.n_spatial - 1):
            pyr.append(restrict(pyr[-1]))
        self.pyramid = pyr[::-1]
        self.K = temporal_sets(self.n, opts.n_temporal)
        self.Y = [None] * opts.n_spatial
        self.Z = [None] * opts.n_spatial
        self.log = []
        # eq. (3): D over all frames at each q of each level, when enabled
        self.stop_trace = [[] for _ in range(opts.n_spatial)]
        self.stop_q = [-1] * opts.n_spatial

    def h(self, level):
        return level_spacing(self.opts.n_spatial, level)

    def predict(self, level, q_next):
        o = self.opts
        if q_next == 0:
            ext = self.extents[level]
            if level == 0:
                z = np.zeros((self.n, self.d) + ext)
            else:
                z = prolong(self.Y[level - 1], ext)
        else:
            Kq = self.K[q_next - 1]
            if level == 0:
                z = linear_predict(self.Y[level], Kq)
            else:
                z = ls_predict(self.Y[level], self.Z[level], Kq, o.beta)
        self.Z[level] = z
        self.Y[level] = z.copy()

    def register_level(self, level, q):
        o = self.opts
        res = gauss_newton(self.pyramid[level], self.Y[level], self.K[q],
                           self.h(level), o.params(), gn_max=o.gn_max,
                           cg_max=o.cg_max, cg_rtol=o.cg_rtol,
                           ls_max=o.ls_max, c1=o.c1, fixed=o.parity_mode,
                           tol_J=o.tol_J, tol_u=o.tol_u)
        self.Y[level] = res.u
        self.log.append({"level": level, "q": q, "nK": len(self.K[q]),
                         "gn": res.iterations, "cg": res.cg_iterations,
                         "steps": res.steps, "J0": res.J0, "J": res.J,
                         "status": res.status})
        return res

    correct = register_level

    def all_frame_D(self, level, U):
        return objective_value(self.pyramid[level], U, range(self.n),
                               self.h(level), self.opts.params())[1]

    def run(self):
        o = self.opts
        T = o.n_temporal - 1
        for level in range(o.n_spatial):
            self.predict(level, 0)
            self.register_level(level, 0)
            D_prev = None
            for q in range(T):
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
                        self.log.append({"level": level, "stop_at_q": q})
                        break
                    D_prev = Dq
                self.correct(level, q + 1)
        return self.Y[-1]


def stml_run(frames, opts):
    """Run the whole schedule; returns (u_finest, state)."""
    st = STMLState(frames, opts)
    u = st.run()
    return u, st
