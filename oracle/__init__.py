"""Plain FP64 CPU oracle for spatio-temporal multilevel (STML) registration.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (no kernels, headers, helpers, tables or constant generators).

The oracle follows the paper (Aggrawal & Modersitzki, "Accelerating the
Registration of Image Sequences by Spatio-temporal Multilevel Strategies",
arXiv 2001.06613) for the outer schedule and the predictors, and a textbook
non-parametric groupwise model for the inner registration:

* Sec. 2, eq. (1): objective J = sum_ij D + S + P over a frame subset K, and
  the penalty P on the mean transformation.
* Sec. 3, Fig. 1: the binary temporal tree K_0 ... K_T.
* Sec. 3: linear (midpoint) predictor on the coarse spatial level.
* Sec. 3, eq. (2): least-squares temporal predictor, solved by the Thomas
  algorithm (tridiagonal, O(n)).
* Sec. 3, eq. (3): optional stopping rule on the change of D.
* Sec. 4: spatial multilevel data, smoothing in space only.
* Sec. 2 and Sec. 4 (``affine.py``): the paper's experimental model, one
  affine-linear map per frame, the correlation-based SqN distance and
  L-BFGS, with the same schedule acting on the parameters.

Every floating-point quantity is computed in float64 from float32 inputs.

Parity status per function is stated in each module header; every function
here is pinned by at least one ``-m "not gpu"`` test against a closed form, a
library routine, an invariant or brute force, except where a module says
"parity unpinned".
"""

from .grid import (level_extents, level_spacing, temporal_sets, restrict,
                   prolong)
from .warp import interp_with_grad
from .objective import (ModelParams, objective, objective_value, hessvec,
                        jacobi_diag, reg_apply_BtB, reg_value,
                        neumann_laplacian)
from .solver import pcg, gauss_newton, GNResult
from .predictor import (linear_predict, ls_predict, thomas_solve,
                        ls_system)
from .stml import STMLOptions, stml_run

__all__ = [
    "level_extents", "level_spacing", "temporal_sets", "restrict", "prolong",
    "interp_with_grad", "ModelParams", "objective", "objective_value",
    "hessvec", "jacobi_diag", "reg_apply_BtB", "reg_value",
    "neumann_laplacian", "pcg", "gauss_newton", "GNResult", "linear_predict",
    "ls_predict", "thomas_solve", "ls_system", "STMLOptions", "stml_run",
]
