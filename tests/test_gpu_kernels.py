"""GPU parity of the kernel-level entry points against the FP64 oracle.

Every call goes through the C-ABI (libstml.so via ctypes).  Shapes span
several 64-voxel tiles with a ragged tail; subsets are non-contiguous.
Tolerances: objective and gradient 1e-5 relative (float64 arithmetic on
float32 data, float32 outputs), Hessian product 1e-5 relative (float32
derivative cache), restriction bit-exact (a mean of 1, 2, 4 or 8 float32
values is exact in float64 and rounded once), transfers and predictors at
float32 rounding.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2001_06613_amd import synth
from paper_2001_06613_amd.binding import STML, default_opts, STMLError, \
    STML_EINVAL, STML_ESTATE

pytestmark = pytest.mark.gpu

CASES = [
    # (name, n, extent, levels, reg, K)
    ("2d_ragged_diff", 5, (37, 53), 2, "diffusion", [0, 2, 3, 4]),
    ("2d_ragged_curv", 6, (41, 45), 2, "curvature", [0, 1, 3, 5]),
    ("3d_ragged_curv", 4, (9, 10, 11), 2, "curvature", [0, 1, 3]),
    ("3d_ragged_diff", 3, (7, 12, 13), 1, "diffusion", [0, 1, 2]),
    ("2d_thin_row", 4, (1, 150), 1, "curvature", [0, 1, 2, 3]),
    ("2d_single_frame", 3, (20, 70), 1, "curvature", [1]),
    # several 32 x 16 columns of 16 planes, each axis with a ragged tail
    ("3d_columns_curv", 3, (37, 20, 35), 1, "curvature", [0, 2]),
    ("3d_columns_diff", 2, (20, 33, 17), 1, "diffusion", [0, 1]),
    ("3d_columns_wide", 2, (18, 17, 70), 1, "curvature", [0, 1]),
    # z-extents that are multiples of the 64-voxel tile: the evaluation
    # takes its tiles in bands of 16 y-lines; two tiles per z-line and a
    # ragged last band (16, 16, 5 lines), and a single short band
    ("3d_line_bands", 3, (5, 37, 128), 1, "curvature", [0, 2]),
    ("3d_line_short", 2, (9, 7, 64), 1, "diffusion", [0, 1]),
]


def _frames(n, ext, seed):
    rng = np.random.default_rng(seed)
    base = synth.base_image(rng, ext)
    f = np.stack([base * (1 + 0.05 * rng.standard_normal(ext))
                  for _ in range(n)])
    return f.astype(np.float32)


def _ctx(n, ext, levels, reg, **kw):
    o = default_opts(dim=len(ext), n_spatial=levels, n_temporal=1, reg=reg,
                     alpha=0.05, lam=0.1, **kw)
    return STML(n, ext, opts=o)


def _params(reg):
    return oracle.ModelParams(alpha=0.05, lam=0.1, reg=reg)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _elementwise(got, ref, tol, what):
    """max |got - ref| <= tol max |ref| over every element; also reports
    the largest error on the voxels next to a domain face."""
    err = np.abs(got - ref)
    scale = float(np.max(np.abs(ref)))
    d = ref.ndim - 2
    face = np.zeros(ref.shape[2:], bool)
    for a in range(d):
        sl = [slice(None)] * d
        for idx in (0, -1):
            sl[a] = idx
            face[tuple(sl)] = True
    print(f"  {what}: max err {err.max():.3e} (faces {err[..., face].max():.3e})"
          f" vs max|ref| {scale:.3e}", flush=True)
    assert float(err.max()) <= tol * scale, what


def _setup(case, seed=0):
    name, n, ext, levels, reg, K = case
    frames = _frames(n, ext, seed)
    st = _ctx(n, ext, levels, reg)
    st.set_sequence(torch.from_numpy(frames).cuda())
    level = levels - 1
    h = oracle.level_spacing(levels, level)
    u = synth.random_displacement(ext, n, 2.5, seed + 1, smooth=False)
    return st, frames, u, level, h, reg, K


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_eval_parity(case):
    st, frames, u, level, h, reg, K = _setup(case)
    print(f"eval parity {case[0]}", flush=True)
    out = st.eval(level, K, torch.from_numpy(u))
    ref = oracle.objective(frames, u, K, h, _params(reg))
    for key in ("J", "D", "S", "P"):       # each to its own size
        assert abs(out[key] - ref[key]) <= 1e-5 * abs(ref[key]) + 1e-12, key
    g = out["g"].cpu().numpy()
    assert _rel(g, ref["g"]) <= 1e-5
    _elementwise(g, ref["g"], 1e-5, "g")
    dW = out["dW"].cpu().numpy()
    np.testing.assert_allclose(dW, ref["dW"], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_hessvec_parity(case):
    st, frames, u, level, h, reg, K = _setup(case, seed=3)
    print(f"hessvec parity {case[0]}", flush=True)
    rng = np.random.default_rng(9)
    v = rng.standard_normal((len(K), len(case[2])) + case[2]).astype(
        np.float32)
    hv, vhv = st.hessvec(level, K, torch.from_numpy(u), torch.from_numpy(v))
    ref = oracle.objective(frames, u, K, h, _params(reg))
    # the library's Hessian uses dW/du rounded to float32; so does this check
    dW32 = ref["dW"].astype(np.float32)
    Hv_ref = oracle.hessvec(dW32, v, h, _params(reg))
    assert _rel(hv.cpu().numpy(), Hv_ref) <= 1e-5
    _elementwise(hv.cpu().numpy(), Hv_ref, 1e-5, "Hv")
    assert vhv == pytest.approx(float(np.sum(v * Hv_ref)), rel=1e-5)


def test_restrict_bit_exact():
    """Each level is stored in float32 and restricted from the stored
    finer level: one step is bit-exact against the oracle's float64 mean
    rounded once; the whole pyramid is within 2 float32 ulps of the oracle's
    float64 pyramid."""
    for ext in [(37, 53), (64, 64), (9, 10, 11), (1, 7)]:
        n = 3
        frames = _frames(n, ext, 5)
        st = _ctx(n, ext, 3, "diffusion")
        st.set_sequence(torch.from_numpy(frames).cuda())
        f64 = frames.astype(np.float64)
        prev = None
        for level in (2, 1, 0):
            got = st.get_level_frames(level).cpu().numpy()
            if prev is None:
                np.testing.assert_array_equal(got, frames)
            else:
                step = oracle.restrict(prev.astype(np.float64))
                np.testing.assert_array_equal(got, step.astype(np.float32))
                f64 = oracle.restrict(f64)
                np.testing.assert_allclose(got, f64, rtol=2.5e-7, atol=0)
            prev = got


def _fields_setup(n, ext, levels):
    o = default_opts(dim=len(ext), n_spatial=levels, n_temporal=3)
    st = STML(n, ext, opts=o)
    st.set_sequence(torch.from_numpy(_frames(n, ext, 1)).cuda())
    return st


@pytest.mark.parametrize("ext", [(37, 53), (9, 10, 11), (64, 64)])
def test_prolong_parity(ext):
    n = 3
    st = _fields_setup(n, ext, 2)
    cext = st.level_extent(0)
    yc = synth.random_displacement(cext, n, 3.0, 4, smooth=False)
    st.set_displacements(0, torch.from_numpy(yc))
    st.predict(1, 0)
    got = st.get_displacements(1).cpu().numpy()
    ref = oracle.prolong(yc, ext)
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-6)
    np.testing.assert_array_equal(st.get_prediction(1).cpu().numpy(), got)


@pytest.mark.parametrize("n", [9, 17, 64])
def test_linear_predictor_parity(n):
    ext = (13, 21)
    st = _fields_setup(n, ext, 1)
    K = oracle.temporal_sets(n, 3)
    assert st.temporal_set(0) == K[0] and st.temporal_set(1) == K[1]
    Y = synth.random_displacement(ext, n, 3.0, 6, smooth=False)
    for q in (0, 1):
        st.set_displacements(0, torch.from_numpy(Y))
        st.predict(0, q + 1)
        ref = oracle.linear_predict(Y, K[q])
        np.testing.assert_allclose(st.get_prediction(0).cpu().numpy(), ref,
                                   rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(st.get_displacements(0).cpu().numpy(), ref,
                                   rtol=1e-6, atol=1e-6)


# 32 and 64 frames take the form with the sweep's pivots in registers
@pytest.mark.parametrize("n,beta", [(9, 1e-5), (17, 0.5), (32, 0.5),
                                    (64, 1e-5), (129, 1e-5), (200, 3.0)])
def test_ls_predictor_parity(n, beta):
    ext = (11, 19)
    o = default_opts(dim=2, n_spatial=2, n_temporal=3, beta=beta)
    st = STML(n, ext, opts=o)
    st.set_sequence(torch.from_numpy(_frames(n, ext, 2)).cuda())
    K = oracle.temporal_sets(n, 3)
    eta = synth.random_displacement(ext, n, 3.0, 7, smooth=False)
    omega = synth.random_displacement(ext, n, 3.0, 8, smooth=False)
    for q in (0, 1):
        st.set_displacements(1, torch.from_numpy(eta))
        st.set_prediction(1, torch.from_numpy(omega))
        st.predict(1, q + 1)
        ref = oracle.ls_predict(eta, omega, K[q], beta)
        got = st.get_prediction(1).cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-5)
        np.testing.assert_array_equal(st.get_displacements(1).cpu().numpy(),
                                      got)


def test_errors_and_state():
    o = default_opts()
    st = STML(4, (16, 16), opts=o)
    with pytest.raises(STMLError) as e:
        st.predict(0, 0)
    assert e.value.code == STML_ESTATE
    bad = np.ones((4, 16, 16), np.float32)
    bad[2, 3, 4] = np.nan
    with pytest.raises(STMLError) as e:
        st.set_sequence(torch.from_numpy(bad).cuda())
    assert e.value.code == STML_EINVAL
    st.set_sequence(torch.ones(4, 16, 16).cuda())
    u = torch.zeros(4, 2, 16, 16)
    with pytest.raises(STMLError) as e:
        st.eval(1, [2, 1], u)                 # not ascending
    assert e.value.code == STML_EINVAL
    with pytest.raises(STMLError) as e:
        st.eval(5, [0], u)                    # no such level
    assert e.value.code == STML_EINVAL
