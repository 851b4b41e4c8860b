"""Spatial levels, the temporal tree, restriction and prolongation (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Conventions (the paper leaves them open; the same readings bind the HIP
path):

* Cell-centred grids.  Voxel i of an axis with spacing h has its centre at
  (i + 1/2) h.  The finest level has h = 1 (pixel units); every coarser
  level doubles h.
* Extents halve with ceiling division, reproducing the grid sizes of
  Sec. 4, Table 1 (225 -> 113 -> 57 -> 29).
* Displacements are stored in finest-pixel physical units, so a
  displacement field moves between levels without rescaling.
"""

import numpy as np


def level_extents(extent, n_levels):
    """Extents of every spatial level, coarse first (Sec. 4, Table 1 sizes).

    ``extent`` is the finest extent, slowest axis first.  Each coarser level
    has ceil(m / 2) cells per axis.
    """
    ext = [tuple(int(m) for m in extent)]
    for _ in range(n_levels - 1):
        ext.append(tuple((m + 1) // 2 for m in ext[-1]))
    return ext[::-1]


def level_spacing(n_levels, level):
    """Cell width h of ``level`` (0 = coarsest) in finest-pixel units."""
    return float(2 ** (n_levels - 1 - level))


def temporal_sets(n, n_temporal):
    """Binary-tree frame subsets K_0 ... K_T, 0-based (Sec. 3, Fig. 1).

    K_T holds all n frames, K_{T-1} every second frame, K_{T-2} every fourth,
    and so on; the last frame is always kept so that every frame has a left
    and a right neighbour in each subset.  With n = 17 and T = 3 this gives
    Fig. 1's K_0 = {1, 9, 17} and K_1 = {1, 5, 9, 13, 17} (1-based), and with
    n = 129 the subset sizes 17 and 33 of the experiments in Sec. 4.
    """
    T = n_temporal - 1
    sets = []
    for q in range(n_temporal):
        step = 2 ** (T - q)
        ks = set(range(0, n, step))
        ks.add(n - 1)
        sets.append(sorted(ks))
    return sets


def restrict(img):
    """One restriction step in space only (Sec. 4: smoothing is spatial only).

    ``img`` has shape (n, *extent).  Coarse cell I is the plain mean of the
    fine cells 2I + {0,1}^d that exist; an odd extent leaves a last coarse
    cell that averages fewer fine cells.  Computed in float64.
    """
    img = np.asarray(img, dtype=np.float64)
    n = img.shape[0]
    fine = img.shape[1:]
    d = len(fine)
    coarse = tuple((m + 1) // 2 for m in fine)
    acc = np.zeros((n,) + coarse)
    cnt = np.zeros(coarse)
    for off in np.ndindex(*([2] * d)):
        # fine cells with index 2I + off that exist
        sl_f = []
        sl_c = []
        for a in range(d):
            nf = (fine[a] - off[a] + 1) // 2   # number of valid I along axis a
            sl_f.append(slice(off[a], off[a] + 2 * nf, 2))
            sl_c.append(slice(0, nf))
        acc[(slice(None),) + tuple(sl_c)] += img[(slice(None),) + tuple(sl_f)]
        cnt[tuple(sl_c)] += 1.0
    return acc / cnt


def _linear_weights(p, m):
    """Clamped cell-centred linear interpolation along one axis.

    Returns (i0, i1, f) such that the interpolant at index coordinate p is
    (1 - f) * v[i0] + f * v[i1].
    """
    pc = np.clip(p, 0.0, m - 1.0)
    if m == 1:
        z = np.zeros(np.shape(p), dtype=np.int64)
        return z, z, np.zeros(np.shape(p))
    i0 = np.minimum(np.floor(pc).astype(np.int64), m - 2)
    f = pc - i0
    return i0, i0 + 1, f


def prolong(field, fine_extent):
    """Prolong a cell-centred field to the next finer grid.

    ``field`` has shape (..., *coarse_extent).  The coarse cell-centred
    piecewise (bi/tri)linear interpolant, clamped at the boundary, is sampled
    at the fine cell centres: fine index i sits at coarse index coordinate
    (i + 1/2) / 2 - 1/2, which gives the weights 3/4 and 1/4 in the interior.
    Values keep their units (displacements are in finest-pixel units), so no
    rescaling.  This is the spatial transfer of y(l-1, T, all) to level l
    that Sec. 3 uses as the starting guess at q = 0.
    """
    field = np.asarray(field, dtype=np.float64)
    d = len(fine_extent)
    coarse = field.shape[-d:]
    out = field
    # separable: interpolate axis by axis (tensor-product linear interpolant)
    for a in range(d):
        m_c = coarse[a]
        i = np.arange(fine_extent[a], dtype=np.float64)
        p = (i + 0.5) / 2.0 - 0.5
        i0, i1, f = _linear_weights(p, m_c)
        ax = out.ndim - d + a
        v0 = np.take(out, i0, axis=ax)
        v1 = np.take(out, i1, axis=ax)
        shape = [1] * out.ndim
        shape[ax] = fine_extent[a]
        f = f.reshape(shape)
        out = (1.0 - f) * v0 + f * v1
    return out
