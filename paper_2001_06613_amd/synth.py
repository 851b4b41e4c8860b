"""Seeded synthetic OCT-like image sequences.

This module only draws inputs.  It holds none of the registration method's
arithmetic and is shared by the tests, the benchmark and the oracle checks;
sampling and smoothing use SciPy's library routines.

The paper's data are private 4D-OCT sequences of retinal layers whose
consecutive frames are highly correlated and move smoothly in time (Sec. 4);
the phantoms below stand in for them:

* base image: 8 bands across the layer axis (axis 0) with sorted uniform
  boundaries (thickness >= 3 px) and intensities U(0.2, 1.0), edges
  Gaussian-smoothed (sigma 1 px); 12 Gaussian blobs (sigma 3 px, amplitude
  U(-0.3, 0.3)); clipped to [0.2, 1.0];
* multiplicative Rayleigh speckle with mean 1 and standard deviation 0.3,
  drawn once per pixel and baked into the base image, so every frame is an
  exact warp of the same speckled image;
* motion: i.i.d. normal noise per component, Gaussian-smoothed with
  sigma = side / 8 and scaled to max_x |phi(x)| = 1; a frame is
  frame_t(x) = B(x - g_t(x)) (linear sampling, edge clamp), so the
  displacement that registers frame t is close to g_t.
"""

import math

import numpy as np
from scipy import ndimage


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def band_edges(rng, H, n_bands=8, min_thick=3):
    """Inner boundaries (n_bands - 1, sorted) of horizontal bands over [0, H):
    uniform boundaries conditioned on every band being at least min_thick
    thick (unconditioned when H < n_bands * min_thick)."""
    slack = H - n_bands * min_thick
    if slack >= 0 and (slack / H) ** (n_bands - 1) < 1e-3:
        # the gaps are min_thick plus the slack split by uniform spacings;
        # drawn directly because rejection would accept with probability
        # (slack / H)^(n_bands - 1) only (0 at slack 0)
        u = np.sort(rng.uniform(0, 1, n_bands - 1))
        gaps = min_thick + slack * np.diff(np.concatenate([[0.0], u, [1.0]]))
        return np.cumsum(gaps)[:-1]
    while True:
        b = np.sort(rng.uniform(0, H, n_bands - 1))
        edges = np.concatenate([[0.0], b, [float(H)]])
        if np.min(np.diff(edges)) >= min_thick or slack < 0:
            return b


def base_image(rng, shape, n_bands=8, min_thick=3, n_blobs=12,
               blob_sigma=3.0, speckle_std=0.3):
    """Layered phantom with blobs and speckle, float64, shape ``shape``."""
    H = shape[0]
    b = band_edges(rng, H, n_bands, min_thick)
    inten = rng.uniform(0.2, 1.0, n_bands)
    y = np.arange(H) + 0.5
    band = np.searchsorted(b, y)
    prof = ndimage.gaussian_filter1d(inten[band], 1.0, mode="nearest")
    img = np.broadcast_to(prof.reshape((H,) + (1,) * (len(shape) - 1)),
                          shape).astype(np.float64).copy()
    grids = np.meshgrid(*[np.arange(m) + 0.5 for m in shape], indexing="ij")
    for _ in range(n_blobs):
        c = [rng.uniform(0, m) for m in shape]
        amp = rng.uniform(-0.3, 0.3)
        r2 = sum((g - cc) ** 2 for g, cc in zip(grids, c))
        img += amp * np.exp(-r2 / (2 * blob_sigma ** 2))
    img = np.clip(img, 0.2, 1.0)
    R = rng.rayleigh(1.0, shape)
    mean_r = math.sqrt(math.pi / 2)
    std_r = math.sqrt((4 - math.pi) / 2)
    img *= 1.0 + speckle_std * (R - mean_r) / std_r
    return img


def smooth_field(rng, shape, sigma=None):
    """Smooth random vector field (d, *shape) with max_x |phi(x)| = 1."""
    d = len(shape)
    if sigma is None:
        sigma = max(shape) / 8.0
    phi = rng.standard_normal((d,) + tuple(shape))
    for c in range(d):
        phi[c] = ndimage.gaussian_filter(phi[c], sigma, mode="wrap")
    nrm = np.sqrt(np.sum(phi * phi, axis=0)).max()
    return phi / nrm


def warp_image(img, disp):
    """Sample img at x - disp(x) (index units), linear, edge clamp."""
    shape = img.shape
    grids = np.meshgrid(*[np.arange(m, dtype=np.float64) for m in shape],
                        indexing="ij")
    coords = np.stack([g - disp[a] for a, g in enumerate(grids)])
    return ndimage.map_coordinates(img, coords, order=1, mode="nearest")


def sequence_from_motion(B, motion):
    """Frames (n, *shape) float32 from base image B and motions (n, d, ...)."""
    return np.stack([warp_image(B, motion[t]) for t in
                     range(motion.shape[0])]).astype(np.float32)


def sinusoid_sequence(n, shape, max_disp, n_sin, seed, period=None):
    """Sequence whose motion is a sum of n_sin temporal sinusoids.

    g_t = sum_j sin(2 pi j t / period + theta_j) phi_j, scaled so that
    max_{t,x} |g_t(x)| = max_disp.  Returns (frames float32, motion float64).
    """
    rng = _rng(seed)
    B = base_image(rng, shape)
    if period is None:
        period = n
    fields = [smooth_field(rng, shape) for _ in range(n_sin)]
    theta = rng.uniform(0, 2 * math.pi, n_sin) if n_sin > 1 else [0.0]
    t = np.arange(n, dtype=np.float64)
    g = np.zeros((n, len(shape)) + tuple(shape))
    for j in range(n_sin):
        a = np.sin(2 * math.pi * (j + 1) * t / period + theta[j])
        g += a.reshape((n,) + (1,) * (len(shape) + 1)) * fields[j][None]
    mx = np.sqrt(np.sum(g * g, axis=1)).max()
    if mx > 0:
        g *= max_disp / mx
    return sequence_from_motion(B, g), g


def config_small(seed=0):
    """8 frames of 64x64, u_t = 2 sin(2 pi t / 8) phi (max 2 px), seed 0."""
    rng = _rng(seed)
    shape = (64, 64)
    B = base_image(rng, shape)
    phi = smooth_field(rng, shape)
    t = np.arange(8, dtype=np.float64)
    g = 2.0 * np.sin(2 * math.pi * t / 8).reshape(8, 1, 1, 1) * phi[None]
    return sequence_from_motion(B, g), g


def config_large(seed=1):
    """64 frames of 256x256, 3 temporal sinusoids, max 5 px, seed 1."""
    return sinusoid_sequence(64, (256, 256), 5.0, 3, seed)


def config_batch(master_seed=2, count=32, n_range=(16, 128),
                 side_range=(128, 512)):
    """(n, side, seed) of the uneven batch: n ~ U{16..128}, side ~ U{128..512}.

    Sequence s is drawn with seed 100 + s by ``sinusoid_sequence``.
    """
    rng = _rng(master_seed)
    out = []
    for s in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        side = int(rng.integers(side_range[0], side_range[1] + 1))
        out.append((n, side, 100 + s))
    return out


def config_volume(seed=3, n=32, shape=(128, 128, 64), max_disp=4.0):
    """3D sequence: n frames of 128x128x64 volumes, max 4 px."""
    return sinusoid_sequence(n, shape, max_disp, 3, seed)


def config_volume_batch(master_seed=4, count=4, n_range=(24, 40)):
    """(n, seed) of the 3D batch: n ~ U{24..40} frames of 128x128x64.

    Sequence s is drawn with seed 30 + s by ``sinusoid_sequence`` (3
    temporal sinusoids, max 4 px); the frame counts by the master seed.
    """
    rng = _rng(master_seed)
    return [(int(rng.integers(n_range[0], n_range[1] + 1)), 30 + s)
            for s in range(count)]


def translated_sequence(shifts, shape, seed=0, sigma=2.0, n_blobs=6):
    """Compact blob phantom translated by integer shifts (n, d).

    The background is 0 and blobs stay away from the border, so every frame
    is an exact integer translate of frame-independent content.
    frame_t(x) = B(x - s_t).
    """
    rng = _rng(seed)
    d = len(shape)
    grids = np.meshgrid(*[np.arange(m, dtype=np.float64) for m in shape],
                        indexing="ij")
    margin = 4 * sigma + np.max(np.abs(shifts)) + 2
    centres = [[rng.uniform(margin, m - 1 - margin) for m in shape]
               for _ in range(n_blobs)]
    amps = rng.uniform(0.5, 1.0, n_blobs)
    frames = []
    for s in shifts:
        img = np.zeros(shape)
        for c, a in zip(centres, amps):
            r2 = sum((grids[ax] - (c[ax] + s[ax])) ** 2 for ax in range(d))
            img += a * np.exp(-r2 / (2 * sigma ** 2))
        frames.append(img)
    return np.stack(frames).astype(np.float32)


def random_displacement(shape_nd, n, max_px, seed, smooth=True):
    """Random float32 displacement (n, d, *shape) for kernel-level tests."""
    rng = _rng(seed)
    d = len(shape_nd)
    if smooth:
        u = np.stack([smooth_field(rng, shape_nd, max(shape_nd) / 4.0)
                      for _ in range(n)])
        u *= max_px
    else:
        u = rng.uniform(-max_px, max_px, (n, d) + tuple(shape_nd))
    return u.astype(np.float32)


def affine_motion(n, d, max_disp, extent, seed, n_sin=2):
    """Per-frame affine motions (n, d, d + 1): row a of frame t maps a voxel
    centre x to the displacement sum_e M[a, e] (x_e - m_e / 2) / (m_e / 2)
    + M[a, d], a sum of n_sin temporal sinusoids of random matrices, scaled
    so that the largest displacement over the grid corners and frames is
    max_disp pixels."""
    rng = _rng(seed)
    mats = rng.standard_normal((n_sin, d, d + 1))
    mats[:, :, :d] *= 0.5                      # strain smaller than shift
    phase = rng.uniform(0, 2 * math.pi, n_sin)
    t = np.arange(n, dtype=np.float64)
    M = np.zeros((n, d, d + 1))
    for j in range(n_sin):
        M += np.sin(2 * math.pi * (j + 1) * t / n + phase[j])[:, None, None] \
            * mats[j][None]
    corners = np.array(np.meshgrid(*[[-1.0, 1.0]] * d, indexing="ij")) \
        .reshape(d, -1)
    disp = np.einsum("tae,ec->tac", M[:, :, :d], corners) + M[:, :, d:]
    mx = np.sqrt(np.sum(disp * disp, axis=1)).max()
    return M * (max_disp / mx)


def affine_frame(B, M):
    """One frame B(x - g(x)) for an affine motion M (d, d + 1) of
    ``affine_motion`` (linear sampling, edge clamp)."""
    shape = B.shape
    d = len(shape)
    grids = np.meshgrid(*[np.arange(m, dtype=np.float64) for m in shape],
                        indexing="ij")
    rel = [(grids[e] + 0.5 - shape[e] / 2.0) / (shape[e] / 2.0)
           for e in range(d)]
    coords = np.stack([grids[a] - (sum(M[a, e] * rel[e] for e in range(d))
                                   + M[a, d]) for a in range(d)])
    return ndimage.map_coordinates(B, coords, order=1,
                                   mode="nearest").astype(np.float32)


def affine_sequence(n, shape, max_disp, seed, workers=None):
    """OCT-like phantom moved by temporally smooth affine motions: the
    stand-in for the paper's affine experiments (Sec. 4).  Returns (frames
    float32 (n, *shape), motions (n, d, d + 1)).  With ``workers`` > 1 the
    frames are sampled by forked processes."""
    rng = _rng(seed)
    B = base_image(rng, shape)
    M = affine_motion(n, len(shape), max_disp, shape, seed + 1)
    if workers and workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            frames = pool.starmap(affine_frame, [(B, M[t]) for t in range(n)],
                                  chunksize=4)
    else:
        frames = [affine_frame(B, M[t]) for t in range(n)]
    return np.stack(frames), M
