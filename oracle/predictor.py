"""Temporal predictors of the STML scheme (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

* Coarse spatial level (Sec. 3): frames of K_q keep their registered
  transformation (injection); every other frame k gets the linear
  interpolation between its neighbours left(k) = max{z < k, z in K_q} and
  right(k) = min{z > k, z in K_q}.  At a midpoint this is the paper's
  0.5/0.5 rule; away from the midpoint (possible because the last frame is
  always kept) the weights are the distances, (r - k)/(r - l) and
  (k - l)/(r - l).
* Finer spatial levels (Sec. 3, eq. (2)): per component, zeta minimises
      sum_{k in K_q} (zeta_k - eta_k)^2
      + beta sum_{k=0}^{n-2} [(zeta_{k+1} - zeta_k) - (omega_{k+1} - omega_k)]^2,
  i.e. (M + beta D^T D) zeta = M eta + beta D^T D omega with M the 0/1
  diagonal selecting K_q and D the (n-1) x n forward difference.  The
  matrix is tridiagonal, symmetric positive definite and weakly diagonally
  dominant, so the Thomas algorithm (Gaussian elimination without pivoting
  on a tridiagonal matrix) solves it in O(n) (Sec. 3, citing Higham).
"""

import numpy as np


def linear_predict(Y, Kq):
    """Linear temporal interpolation over all n frames from the frames Kq.

    Y : (n, ...) array; only Y[Kq] is read.
    """
    Y = np.asarray(Y, dtype=np.float64)
    n = Y.shape[0]
    Kq = sorted(Kq)
    Z = np.empty_like(Y)
    kset = set(Kq)
    for k in range(n):
        if k in kset:
            Z[k] = Y[k]
            continue
        left = max(z for z in Kq if z < k)
        right = min(z for z in Kq if z > k)
        wl = (right - k) / (right - left)
        wr = (k - left) / (right - left)
        Z[k] = wl * Y[left] + wr * Y[right]
    return Z


def ls_system(n, Kq, beta):
    """Tridiagonal A = M + beta D^T D of eq. (2): (sub, diag, sup), each (n,)."""
    m = np.zeros(n)
    m[list(Kq)] = 1.0
    ndiff = np.full(n, 2.0)          # differences touching k
    ndiff[0] = 1.0
    ndiff[-1] = 1.0
    if n == 1:
        ndiff[0] = 0.0
    diag = m + beta * ndiff
    sub = np.full(n, -beta)
    sup = np.full(n, -beta)
    sub[0] = 0.0
    sup[-1] = 0.0
    return sub, diag, sup


def _dtd(omega):
    """D^T D omega along axis 0 (D = forward differences)."""
    n = omega.shape[0]
    out = np.zeros_like(omega)
    if n < 2:
        return out
    diff = omega[1:] - omega[:-1]      # (n-1, ...)
    out[:-1] -= diff
    out[1:] += diff
    return out


def thomas_solve(sub, diag, sup, rhs):
    """Thomas algorithm for a tridiagonal system, many right-hand sides.

    sub[k] multiplies x[k-1] in row k, sup[k] multiplies x[k+1]; rhs has
    shape (n, ...).  Forward elimination then back substitution, no pivoting.
    """
    rhs = np.asarray(rhs, dtype=np.float64)
    n = rhs.shape[0]
    cp = np.zeros(n)
    dp = np.zeros_like(rhs)
    cp[0] = sup[0] / diag[0]
    dp[0] = rhs[0] / diag[0]
    for k in range(1, n):
        den = diag[k] - sub[k] * cp[k - 1]
        cp[k] = sup[k] / den
        dp[k] = (rhs[k] - sub[k] * dp[k - 1]) / den
    x = np.zeros_like(rhs)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def ls_predict(eta, omega, Kq, beta):
    """Solve eq. (2) for every component at once.

    eta   : (n, ...) registered transformations; only rows Kq are read.
    omega : (n, ...) reference for the local temporal changes.
    Returns zeta with the shape of omega.
    """
    eta = np.asarray(eta, dtype=np.float64)
    omega = np.asarray(omega, dtype=np.float64)
    n = omega.shape[0]
    m = np.zeros(n)
    m[list(Kq)] = 1.0
    shape = (n,) + (1,) * (omega.ndim - 1)
    rhs = m.reshape(shape) * np.where(m.reshape(shape) > 0, eta, 0.0) \
        + beta * _dtd(omega)
    sub, diag, sup = ls_system(n, Kq, beta)
    return thomas_solve(sub, diag, sup, rhs)
