"""GPU parity of the affine-linear SqN / L-BFGS path against the oracle.

The paper's experimental model (Sec. 2, Sec. 4) through the C-ABI: the
objective (D, P and J to 1e-9 of their own size: float64 warps and Gram
sums on both sides) and the parameter gradient (element-wise within 1e-5
of its largest entry: dD/dW is stored in float32 between passes) on ragged
2-D and 3-D grids, fine and coarse levels and frame subsets; L-BFGS
registrations with fixed iteration counts (identical Armijo steps,
parameters within 1e-4 px, so u within 1e-3 px); the whole schedule on the
8-frame 64x64 sequence; eq. (3) on the parameters; the displacement field
written from the parameters; exact recovery of integer translations; and
the entry points that do not apply to the affine model.
"""

import numpy as np
import pytest
import torch

from oracle import affine as af
from oracle import restrict
from paper_2001_06613_amd import synth
from paper_2001_06613_amd.binding import STML, Batch, STMLError, \
    default_opts

pytestmark = pytest.mark.gpu

LAM = 1e-2


def _ctx(frames, L=1, T1=1, lam=LAM, **kw):
    n, ext = frames.shape[0], frames.shape[1:]
    o = default_opts(dim=len(ext), n_spatial=L, n_temporal=T1,
                     model="affine", lam=lam, **kw)
    st = STML(n, ext, opts=o)
    st.set_sequence(torch.from_numpy(np.ascontiguousarray(frames)).cuda())
    return st


def _pyramid(frames, L):
    """Levels as the library stores them: each restricted from the stored
    finer level and rounded to float32 (bit-exact, see the restriction
    parity test)."""
    pyr = [np.asarray(frames, np.float32)]
    for _ in range(L - 1):
        pyr.append(restrict(pyr[-1].astype(np.float64)).astype(np.float32))
    return pyr[::-1]


CASES = [
    # (name, n, extent, levels, level, K)
    ("2d_ragged", 5, (37, 53), 2, 1, [0, 2, 3, 4]),
    ("2d_coarse", 5, (37, 53), 2, 0, [0, 1, 4]),
    ("2d_single", 3, (20, 70), 1, 0, [1]),
    ("3d_ragged", 4, (9, 10, 11), 1, 0, [0, 1, 3]),
    ("3d_coarse", 3, (17, 12, 21), 2, 0, [0, 1, 2]),
    # more frames than one 16-row tile of the Gram matrix
    ("2d_many", 40, (24, 20), 1, 0, list(range(0, 40, 1))),
    # more Gram tiles than the waves of a block hold (several tile groups,
    # each warping the frames again) and more than one group of row tiles
    # of dD/dW per wave
    ("2d_groups", 210, (12, 10), 1, 0, list(range(0, 210, 1))),
    ("3d_groups", 150, (5, 6, 7), 1, 0, list(range(0, 150, 1))),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_affine_eval_parity(case):
    name, n, ext, L, level, K = case
    frames = synth.sinusoid_sequence(n, ext, 1.5, 1, seed=41)[0]
    st = _ctx(frames, L)
    rng = np.random.default_rng(42)
    theta = rng.uniform(-1.5, 1.5, (n, len(ext) ** 2 + len(ext)))
    h = float(2 ** (L - 1 - level))
    print(f"affine eval {name}", flush=True)
    out, g = st.eval_params(level, K, theta)
    ref = af.objective(_pyramid(frames, L)[level], theta, K, h, ext,
                       af.AffineParams(LAM))
    for key in ("J", "D", "P"):
        assert abs(out[key] - ref[key]) <= 1e-9 * abs(ref[key]) + 1e-12, \
            (key, out[key], ref[key])
    err = float(np.max(np.abs(g - ref["g"])))
    scale = float(np.max(np.abs(ref["g"])))
    print(f"  J {out['J']:.10g} vs {ref['J']:.10g}; grad max err {err:.2e}"
          f" of {scale:.2e}", flush=True)
    assert err <= 1e-5 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_affine_register_parity(dim):
    if dim == 2:
        frames = synth.sinusoid_sequence(6, (24, 20), 1.5, 1, seed=8)[0]
        K = [0, 1, 2, 3, 4, 5]
    else:
        frames = synth.sinusoid_sequence(4, (10, 12, 14), 1.2, 1, seed=9)[0]
        K = [0, 1, 2, 3]
    n, ext = frames.shape[0], frames.shape[1:]
    p = dim * dim + dim
    theta0 = np.random.default_rng(3).uniform(-0.5, 0.5, (n, p))
    st = _ctx(frames, 1, 1, gn_max=6, parity_mode=True)
    st.predict(0, 0)
    st.set_params(0, theta0)
    print(f"affine register {dim}-D", flush=True)
    st.register_level(0, 0)
    lg = st.logs()[0]
    res = af.register(np.asarray(frames, np.float64), theta0, K, 1.0, ext,
                      af.AffineParams(LAM), max_iter=6, mem=5, fixed=True)
    print("  steps", lg["steps"], res.steps, flush=True)
    assert lg["steps"] == res.steps
    assert lg["J"] == pytest.approx(res.J, rel=1e-6)
    th = st.get_params(0)
    assert np.max(np.abs(th - res.x)) <= 1e-4
    u = st.get_displacements(0).cpu().numpy()
    xi = af.frame_geometry(ext, ext, 1.0)
    u_ref = np.stack([af.displacement(res.x[k], xi) for k in range(n)])
    assert np.max(np.abs(u - u_ref)) <= 1e-3


def test_affine_stml_run_parity_small():
    """The whole schedule on the 8-frame 64x64 sequence: 2 spatial x 2
    temporal levels, fixed L-BFGS iterations."""
    frames, _ = synth.config_small(0)
    kw = dict(n_spatial=2, n_temporal=2, parity_mode=True)
    st = _ctx(frames, 2, 2, gn_max=5, parity_mode=True)
    st.run()
    u_ref, ost = af.affine_stml_run(frames, af.AffineSTMLOptions(
        lam=LAM, iter_max=5, **kw))
    steps = [lg["steps"] for lg in st.logs()]
    print("steps", steps, flush=True)
    assert steps == [e["steps"] for e in ost.log]
    assert [(lg["level"], lg["nK"]) for lg in st.logs()] == \
        [(e["level"], e["nK"]) for e in ost.log]
    th = st.get_params()
    assert np.max(np.abs(th - u_ref)) <= 1e-4
    u = st.get_displacements().cpu().numpy()
    xi = af.frame_geometry((64, 64), (64, 64), 1.0)
    assert np.max(np.abs(u - np.stack([af.displacement(t, xi)
                                       for t in u_ref]))) <= 1e-3


def test_affine_eq3_stop_rule_parity():
    frames = synth.sinusoid_sequence(9, (24, 20), 1.5, 1, seed=8)[0]
    base = dict(n_spatial=1, n_temporal=3, iter_max=3, tol_J=0.0,
                tol_u=0.0, lam=LAM)
    _, free = af.affine_stml_run(frames, af.AffineSTMLOptions(
        eps_stop=1e-300, **base))
    tr = free.stop_trace[0]
    eps = 2.0 * abs(tr[1] - tr[0])
    _, ost = af.affine_stml_run(frames, af.AffineSTMLOptions(
        eps_stop=eps, **base))
    assert ost.stop_q == [1]
    st = _ctx(frames, 1, 3, gn_max=3, tol_J=0.0, tol_u=0.0, eps_stop=eps)
    st.run()
    trace, q = st.stop_trace(0)
    print("trace", trace, ost.stop_trace[0], flush=True)
    assert q == 1
    np.testing.assert_allclose(trace, ost.stop_trace[0], rtol=1e-8)
    assert [lg["nK"] for lg in st.logs()] == [3, 5]
    assert np.max(np.abs(st.get_params(0) - ost.Y[0])) <= 1e-4


def test_affine_recovers_integer_translations():
    shifts = np.array([[1.0, -1.0], [-1.0, 0.0], [0.0, 1.0]])
    frames = synth.translated_sequence(shifts, (32, 32), seed=1)
    # the oracle's pin of the same recovery uses lambda = 1e-3
    st = _ctx(frames, 1, 1, lam=1e-3, gn_max=60, tol_J=0.0, tol_u=0.0)
    st.predict(0, 0)
    st.register_level(0, 0)
    th = st.get_params(0)
    assert st.logs()[0]["J"] < 1e-8
    np.testing.assert_allclose(th[:, 4:], shifts, atol=1e-3)
    np.testing.assert_allclose(th[:, :4], 0.0, atol=1e-3)


def test_affine_rejects_field_entry_points():
    frames = synth.sinusoid_sequence(4, (16, 16), 1.0, 1, seed=1)[0]
    st = _ctx(frames, 1, 1)
    u = torch.zeros((4, 2, 16, 16), device="cuda")
    with pytest.raises(STMLError):
        st.eval(0, [0, 1], u)
    with pytest.raises(STMLError):
        st.set_displacements(0, u)
    with pytest.raises(STMLError):
        Batch([st, _ctx(frames, 1, 1)])
    with pytest.raises(STMLError):
        STML(4, (16, 16), opts=default_opts(model="affine", predictor=1))
    # a frame without contrast after warping has no correlation
    flat = np.ones((3, 16, 16), np.float32)
    st = _ctx(flat, 1, 1)
    with pytest.raises(STMLError):
        st.eval_params(0, [0, 1, 2], np.zeros((3, 6)))
