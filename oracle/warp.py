"""Bi/trilinear warp of a frame with its analytic derivative (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

The paper writes the transformed image as R_i o y_i (Sec. 2, eq. (1)).  With
a displacement field, y(x) = x + u(x).  The reading used here and on the HIP
path:

* the grid is cell-centred, so the index coordinate of y(x_i) along each
  axis is p = i + u / h;
* p is formed in float64 from the float32 displacement, so both sides take
  the same floor decisions;
* p is clamped to [0, m - 1] (replicate the edge); i0 = min(floor(p), m - 2)
  and f = p - i0; the value is the tensor-product linear interpolant;
* the derivative along axis a is the weighted difference T[i0 + 1] - T[i0]
  (other axes interpolated), divided by h, where 0 <= p_a <= m - 1 before
  clamping, and 0 outside (the clamped interpolant is flat there).  On a
  grid line (f = 0) this is the one-sided forward difference.
"""

import itertools

import numpy as np


def interp_with_grad(img, u, h):
    """Return (W, dW) for one frame.

    img : array (*extent), float32 or float64 frame values.
    u   : array (d, *extent), displacement in finest-pixel units.
    h   : cell width of this level (finest-pixel units).

    W[x]     = img interpolated at x + u(x)
    dW[a][x] = d W / d u_a (x), the partial derivative wrt displacement
               component a, in 1/finest-pixel units.
    """
    img = np.asarray(img, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    ext = img.shape
    d = len(ext)
    grids = np.meshgrid(*[np.arange(m, dtype=np.float64) for m in ext],
                        indexing="ij")
    i0s, fs, inside = [], [], []
    for a in range(d):
        m = ext[a]
        p = grids[a] + u[a] / h
        inside.append((p >= 0.0) & (p <= m - 1.0))
        pc = np.clip(p, 0.0, m - 1.0)
        if m == 1:
            i0 = np.zeros(pc.shape, dtype=np.int64)
            f = np.zeros(pc.shape)
        else:
            i0 = np.minimum(np.floor(pc).astype(np.int64), m - 2)
            f = pc - i0
        i0s.append(i0)
        fs.append(f)

    W = np.zeros(ext)
    dW = np.zeros((d,) + ext)
    for corner in itertools.product((0, 1), repeat=d):
        idx = tuple(np.minimum(i0s[a] + corner[a], ext[a] - 1)
                    for a in range(d))
        val = img[idx]
        w_axis = [fs[a] if corner[a] else 1.0 - fs[a] for a in range(d)]
        w = np.ones(ext)
        for a in range(d):
            w = w * w_axis[a]
        W += w * val
        for a in range(d):
            # derivative of the weight product wrt f_a: +/-1 times the others
            wo = np.ones(ext)
            for b in range(d):
                if b != a:
                    wo = wo * w_axis[b]
            sign = 1.0 if corner[a] else -1.0
            dW[a] += sign * wo * val
    for a in range(d):
        dW[a] = np.where(inside[a], dW[a] / h, 0.0)
    return W, dW
