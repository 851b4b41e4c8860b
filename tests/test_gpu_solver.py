"""GPU parity of the solver and the schedule against the FP64 oracle.

CG directions after a fixed number of iterations, Gauss-Newton registration
of one subset and the whole spatio-temporal multilevel schedule in parity
mode (fixed GN/CG counts).  The accepted Armijo steps must agree exactly
(several correct iterates exist in principle; with identical step sequences
the displacements must agree to 1e-3 px).  The large case runs the
evaluation, the Hessian product and a CG direction at the full 64-frame
256x256 level, in the launch configuration the benchmark times.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2001_06613_amd import synth
from paper_2001_06613_amd.binding import STML, STML_EBREAKDOWN, default_opts

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _elementwise(got, ref, tol, what):
    err = float(np.max(np.abs(got - ref)))
    scale = float(np.max(np.abs(ref)))
    print(f"  {what}: max err {err:.3e} vs max|ref| {scale:.3e}", flush=True)
    assert err <= tol * scale, what


def _small():
    frames, g = synth.config_small(0)
    return frames


@pytest.mark.parametrize("reg,cg", [("diffusion", 10), ("curvature", 10),
                                    ("curvature", 1), ("curvature", 2),
                                    ("diffusion", 5)])
def test_gn_direction_parity(reg, cg):
    # x is written every second CG step: cg = 1 and 5 end on a step that
    # completes x alone, 2 and 10 on one that adds two steps' terms
    frames = _small()
    n, ext = 8, frames.shape[1:]
    o = default_opts(n_spatial=1, n_temporal=2, reg=reg, cg_max=cg,
                     parity_mode=True)
    st = STML(n, ext, opts=o)
    st.set_sequence(torch.from_numpy(frames).cuda())
    u = synth.random_displacement(ext, n, 1.5, 2)
    K = [0, 2, 4, 6, 7]
    print(f"gn_direction {reg} cg={cg}", flush=True)
    delta, iters = st.gn_direction(0, K, torch.from_numpy(u))
    par = oracle.ModelParams(reg=reg)
    ref = oracle.objective(frames, u, K, 1.0, par)
    diag = oracle.jacobi_diag(ref["dW"], 1.0, par)
    d_ref, it_ref, _ = oracle.pcg(
        lambda v: oracle.hessvec(ref["dW"], v, 1.0, par), diag, -ref["g"],
        cg, fixed=True)
    assert iters == it_ref == cg
    d = delta.cpu().numpy()
    assert _rel(d, d_ref) <= 1e-4
    assert np.abs(d - d_ref).max() <= 1e-3


@pytest.mark.parametrize("reg,nt", [("diffusion", 2), ("curvature", 2)])
def test_register_level_parity(reg, nt):
    frames = _small()
    n, ext = 8, frames.shape[1:]
    kw = dict(n_spatial=1, n_temporal=nt, reg=reg, gn_max=5, cg_max=10,
              parity_mode=True)
    st = STML(n, ext, opts=default_opts(**kw))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.predict(0, 0)
    st.register_level(0, 0)
    ost = oracle.stml.STMLState(frames, oracle.STMLOptions(**kw))
    ost.predict(0, 0)
    ost.register_level(0, 0)
    lg, olg = st.logs()[0], ost.log[0]
    print("steps", lg["steps"], olg["steps"], flush=True)
    assert lg["steps"] == olg["steps"]
    assert lg["cg"] == olg["cg"]
    assert lg["J"] == pytest.approx(olg["J"], rel=1e-5)
    u = st.get_displacements(0).cpu().numpy()
    assert np.abs(u - ost.Y[0]).max() <= 1e-3


@pytest.mark.parametrize("reg", ["diffusion", "curvature"])
def test_register_level_convergence_stop(reg):
    """Outside parity mode CG stops at cg_rtol and Gauss-Newton at the
    tol_J / tol_u test; the counts, steps and result match the oracle."""
    frames = _small()
    n, ext = 8, frames.shape[1:]
    kw = dict(n_spatial=1, n_temporal=2, reg=reg, gn_max=40, cg_max=20,
              tol_J=1e-3, tol_u=2e-2, parity_mode=False)
    st = STML(n, ext, opts=default_opts(**kw))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.predict(0, 0)
    st.register_level(0, 0)
    ost = oracle.stml.STMLState(frames, oracle.STMLOptions(**kw))
    ost.predict(0, 0)
    ost.register_level(0, 0)
    lg, olg = st.logs()[0], ost.log[0]
    print("gn", lg["gn"], olg["gn"], "cg", lg["cg"], olg["cg"], flush=True)
    assert lg["gn"] == olg["gn"] < kw["gn_max"]
    assert lg["cg"] == olg["cg"]
    assert lg["steps"] == olg["steps"]
    assert lg["J"] == pytest.approx(olg["J"], rel=1e-5)
    u = st.get_displacements(0).cpu().numpy()
    assert np.abs(u - ost.Y[0]).max() <= 1e-3


@pytest.mark.parametrize("reg", ["diffusion", "curvature"])
def test_stml_run_parity_small(reg):
    """Whole schedule: 2 spatial x 2 temporal levels, 8 frames of 64x64."""
    frames = _small()
    kw = dict(n_spatial=2, n_temporal=2, reg=reg, gn_max=5, cg_max=10,
              parity_mode=True)
    st = STML(8, frames.shape[1:], opts=default_opts(**kw))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.run()
    u_ref, ost = oracle.stml_run(frames, oracle.STMLOptions(**kw))
    steps = [lg["steps"] for lg in st.logs()]
    steps_ref = [lg["steps"] for lg in ost.log]
    print("steps", steps, flush=True)
    assert steps == steps_ref
    u = st.get_displacements().cpu().numpy()
    assert np.abs(u - u_ref).max() <= 1e-3


def test_stml_run_parity_ls_predictor():
    """Three temporal levels on two spatial levels: eq. (2) on the fine one."""
    frames, _ = synth.sinusoid_sequence(17, (48, 40), 3.0, 2, seed=5)
    kw = dict(n_spatial=2, n_temporal=3, reg="curvature", alpha=0.1,
              gn_max=3, cg_max=8, parity_mode=True, beta=1e-3)
    st = STML(17, frames.shape[1:], opts=default_opts(**kw))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.run()
    u_ref, ost = oracle.stml_run(frames, oracle.STMLOptions(**kw))
    assert [lg["steps"] for lg in st.logs()] == \
        [lg["steps"] for lg in ost.log]
    assert np.abs(st.get_displacements().cpu().numpy() - u_ref).max() <= 1e-3


def test_zero_motion_stays_zero():
    f = synth.base_image(np.random.default_rng(3), (40, 40)).astype(
        np.float32)
    frames = np.repeat(f[None], 5, axis=0)
    st = STML(5, (40, 40), opts=default_opts(n_spatial=2, n_temporal=2,
                                              gn_max=3, cg_max=5,
                                              parity_mode=True))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.run()
    assert torch.count_nonzero(st.get_displacements()).item() == 0
    assert all(lg["J"] == 0.0 for lg in st.logs())


def test_translation_recovery():
    shifts = np.array([[1.0, -1.0], [-1.0, 0.0], [0.0, 1.0]])
    frames = synth.translated_sequence(shifts, (32, 32), seed=1)
    st = STML(3, (32, 32), opts=default_opts(
        n_spatial=1, n_temporal=1, alpha=1e-2, lam=1e-1, gn_max=40,
        cg_max=200, cg_rtol=1e-8, tol_J=0.0, tol_u=0.0))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.predict(0, 0)
    st.register_level(0, 0)
    u = st.get_displacements(0).cpu().numpy()
    for k in range(3):
        for a in range(2):
            assert np.abs(u[k, a] - shifts[k, a]).max() < 2e-3


def test_repeat_runs_bitwise_identical():
    frames = _small()
    kw = dict(n_spatial=2, n_temporal=2, gn_max=3, cg_max=6,
              parity_mode=True)
    outs = []
    for _ in range(2):
        st = STML(8, frames.shape[1:], opts=default_opts(**kw))
        st.set_sequence(torch.from_numpy(frames).cuda())
        st.run()
        outs.append((st.get_displacements().cpu().numpy(),
                     [lg["J"] for lg in st.logs()]))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]


def test_timing_counts_and_leaves_results_unchanged():
    """Timed runs (all launches, or every 3rd) count the launches the
    schedule makes and give the untimed run's displacements."""
    frames = _small()
    kw = dict(n_spatial=2, n_temporal=2, gn_max=3, cg_max=6,
              parity_mode=True)
    st = STML(8, frames.shape[1:], opts=default_opts(**kw))
    f = torch.from_numpy(frames).cuda()
    st.set_sequence(f)
    st.run()
    ref = st.get_displacements().clone()
    n_upd = sum(sum(lg["cg"]) for lg in st.logs())
    print("timing", flush=True)
    for every in (1, 3):
        st.timing(["cg_update", "hessvec"], every=every)
        st.set_sequence(f)
        st.run()
        t = st.timing_get("cg_update")
        st.timing(None)
        assert torch.equal(st.get_displacements(), ref)
        assert t["launches"] == -(-n_upd // every)
        assert t["ms"] > 0 and t["bytes"] > 0
        assert st.timing_get("eval")["launches"] == 0


def test_large_level_parity():
    """64 frames of 256x256 (the benchmark's finest level), all frames."""
    frames, _ = synth.config_large(1)
    n, ext = 64, (256, 256)
    o = default_opts(n_spatial=4, n_temporal=3, reg="curvature", alpha=0.1,
                     cg_max=3, parity_mode=True)
    st = STML(n, ext, opts=o)
    st.set_sequence(torch.from_numpy(frames).cuda())
    u = synth.random_displacement(ext, n, 4.0, 11)
    K = list(range(n))
    print("large eval", flush=True)
    out = st.eval(3, K, torch.from_numpy(u))
    par = oracle.ModelParams(alpha=0.1, reg="curvature")
    ref = oracle.objective(frames, u, K, 1.0, par)
    for key in ("J", "D", "S", "P"):
        assert abs(out[key] - ref[key]) <= 1e-5 * abs(ref[key]), key
    assert _rel(out["g"].cpu().numpy(), ref["g"]) <= 1e-5
    _elementwise(out["g"].cpu().numpy(), ref["g"], 1e-5, "g")
    print("large hessvec", flush=True)
    v = np.random.default_rng(1).standard_normal(ref["g"].shape).astype(
        np.float32)
    hv, _ = st.hessvec(3, K, torch.from_numpy(u), torch.from_numpy(v))
    Hv_ref = oracle.hessvec(ref["dW"].astype(np.float32), v, 1.0, par)
    assert _rel(hv.cpu().numpy(), Hv_ref) <= 1e-5
    _elementwise(hv.cpu().numpy(), Hv_ref, 1e-5, "Hv")


def test_large_volume_level_parity():
    """8 frames of 128x128x64 (the volume workload's finest extent), all
    frames, in the launch configuration the benchmark uses."""
    n, ext = 8, (128, 128, 64)
    frames = synth.sinusoid_sequence(n, ext, 4.0, 3, 3)[0]
    o = default_opts(dim=3, n_spatial=3, n_temporal=3, reg="curvature",
                     alpha=0.1, cg_max=3, parity_mode=True)
    st = STML(n, ext, opts=o)
    st.set_sequence(torch.from_numpy(frames).cuda())
    u = synth.random_displacement(ext, n, 3.0, 12)
    K = list(range(n))
    print("large volume eval", flush=True)
    out = st.eval(2, K, torch.from_numpy(u))
    par = oracle.ModelParams(alpha=0.1, reg="curvature")
    ref = oracle.objective(frames, u, K, 1.0, par)
    for key in ("J", "D", "S", "P"):
        assert abs(out[key] - ref[key]) <= 1e-5 * abs(ref[key]), key
    assert _rel(out["g"].cpu().numpy(), ref["g"]) <= 1e-5
    _elementwise(out["g"].cpu().numpy(), ref["g"], 1e-5, "g")
    print("large volume hessvec", flush=True)
    v = np.random.default_rng(2).standard_normal(ref["g"].shape).astype(
        np.float32)
    hv, _ = st.hessvec(2, K, torch.from_numpy(u), torch.from_numpy(v))
    Hv_ref = oracle.hessvec(ref["dW"].astype(np.float32), v, 1.0, par)
    assert _rel(hv.cpu().numpy(), Hv_ref) <= 1e-5
    _elementwise(hv.cpu().numpy(), Hv_ref, 1e-5, "Hv")


def _volume(n, ext, seed):
    return synth.sinusoid_sequence(n, ext, 1.5, 1, seed)[0]


@pytest.mark.parametrize("reg,cg", [("diffusion", 8), ("curvature", 8),
                                    ("curvature", 5)])
@pytest.mark.parametrize("ext", [(10, 12, 18), (37, 20, 70), (5, 37, 128)])
def test_gn_direction_parity_3d(reg, cg, ext):
    # ragged against 32 x 16 x 16 columns; the second spans several columns
    # on every axis (CG steps > 0 take beta and the sums of p from the sums
    # kernel); the third has whole 64-voxel z-line tiles, which the
    # evaluation takes in bands of 16 y-lines (the last band ragged)
    n = 4
    frames = _volume(n, ext, 21)
    o = default_opts(dim=3, n_spatial=1, n_temporal=2, reg=reg, cg_max=cg,
                     parity_mode=True)
    st = STML(n, ext, opts=o)
    st.set_sequence(torch.from_numpy(frames).cuda())
    u = synth.random_displacement(ext, n, 1.2, 4)
    K = [0, 1, 3]
    print(f"gn_direction 3d {reg} cg={cg} {ext}", flush=True)
    delta, iters = st.gn_direction(0, K, torch.from_numpy(u))
    par = oracle.ModelParams(reg=reg)
    ref = oracle.objective(frames, u, K, 1.0, par)
    diag = oracle.jacobi_diag(ref["dW"], 1.0, par)
    d_ref, it_ref, _ = oracle.pcg(
        lambda v: oracle.hessvec(ref["dW"], v, 1.0, par), diag, -ref["g"], cg,
        fixed=True)
    assert iters == it_ref == cg
    d = delta.cpu().numpy()
    assert _rel(d, d_ref) <= 1e-4
    assert np.abs(d - d_ref).max() <= 1e-3


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("brk", [0, 1, 2, 3])
def test_forced_cg_breakdown(dim, brk):
    """A CG that breaks down (p.Hp <= 0, forced from the host at step brk)
    keeps the iterate of the steps before it and reports EBREAKDOWN; a
    breakdown right after an even step adds that step's pending term of x
    (brk = 1, 3)."""
    if dim == 2:
        frames = _small()
        n, ext, K = 8, frames.shape[1:], [0, 2, 4, 6, 7]
        u = synth.random_displacement(ext, n, 1.5, 2)
    else:
        n, ext, K = 4, (10, 12, 18), [0, 1, 3]
        frames = _volume(n, ext, 21)
        u = synth.random_displacement(ext, n, 1.2, 4)
    o = default_opts(dim=dim, n_spatial=1, n_temporal=2, reg="curvature",
                     cg_max=8, parity_mode=True)
    st = STML(n, ext, opts=o)
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.force_cg_breakdown(brk)
    print(f"forced breakdown {dim}-D at CG step {brk}", flush=True)
    delta, iters, rc = st.gn_direction(0, K, torch.from_numpy(u),
                                       allow_breakdown=True)
    assert rc == STML_EBREAKDOWN
    assert iters == brk
    d = delta.cpu().numpy()
    if brk == 0:
        assert not np.any(d)
    else:
        par = oracle.ModelParams(reg="curvature")
        ref = oracle.objective(frames, u, K, 1.0, par)
        diag = oracle.jacobi_diag(ref["dW"], 1.0, par)
        d_ref, it_ref, _ = oracle.pcg(
            lambda v: oracle.hessvec(ref["dW"], v, 1.0, par), diag, -ref["g"],
            brk, fixed=True)
        assert it_ref == brk
        assert _rel(d, d_ref) <= 1e-4
        assert np.abs(d - d_ref).max() <= 1e-3
    st.force_cg_breakdown(-1)
    _, iters2 = st.gn_direction(0, K, torch.from_numpy(u))
    assert iters2 == 8


@pytest.mark.parametrize("reg", ["diffusion", "curvature"])
def test_register_level_convergence_stop_3d(reg):
    """Volumes outside parity mode: CG stops at cg_rtol after odd and even
    steps (after an even one the first kernel of the next step, which finds
    the convergence, completes x), Gauss-Newton at tol_J / tol_u; counts,
    steps and result match the oracle."""
    ext = (10, 12, 18)
    n = 4
    frames = _volume(n, ext, 25)
    kw = dict(dim=3, n_spatial=1, n_temporal=2, reg=reg, gn_max=20,
              cg_max=20, tol_J=1e-3, tol_u=2e-2, parity_mode=False)
    st = STML(n, ext, opts=default_opts(**kw))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.predict(0, 0)
    st.register_level(0, 0)
    ost = oracle.stml.STMLState(frames, oracle.STMLOptions(
        **{k: v for k, v in kw.items() if k != "dim"}))
    ost.predict(0, 0)
    ost.register_level(0, 0)
    lg, olg = st.logs()[0], ost.log[0]
    print("3d gn", lg["gn"], olg["gn"], "cg", lg["cg"], olg["cg"], flush=True)
    assert lg["gn"] == olg["gn"]
    assert lg["cg"] == olg["cg"]
    assert lg["steps"] == olg["steps"]
    assert lg["J"] == pytest.approx(olg["J"], rel=1e-5)
    u = st.get_displacements(0).cpu().numpy()
    assert np.abs(u - ost.Y[0]).max() <= 1e-3


@pytest.mark.parametrize("reg", ["diffusion", "curvature"])
@pytest.mark.parametrize("ext", [(10, 12, 18), (4, 21, 64)])
def test_register_level_parity_3d(reg, ext):
    # the second: evaluation and trial sweeps in bands of 16 y-lines of
    # whole z-line tiles (16 and 5 lines)
    n = 4
    frames = _volume(n, ext, 22)
    kw = dict(dim=3, n_spatial=1, n_temporal=2, reg=reg, gn_max=3, cg_max=6,
              parity_mode=True)
    st = STML(n, ext, opts=default_opts(**kw))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.predict(0, 0)
    st.register_level(0, 0)
    ost = oracle.stml.STMLState(frames, oracle.STMLOptions(
        **{k: v for k, v in kw.items() if k != "dim"}))
    ost.predict(0, 0)
    ost.register_level(0, 0)
    lg, olg = st.logs()[0], ost.log[0]
    print("3d steps", lg["steps"], olg["steps"], flush=True)
    assert lg["steps"] == olg["steps"]
    assert lg["cg"] == olg["cg"]
    assert lg["J"] == pytest.approx(olg["J"], rel=1e-5)
    u = st.get_displacements(0).cpu().numpy()
    assert np.abs(u - ost.Y[0]).max() <= 1e-3


def test_spml_run_parity_and_staged_schedule():
    """SpML (one temporal level: every frame on every spatial level) against
    the oracle; and the schedule driven stage by stage through the entry
    points (as the benchmark's SpML/STML comparison times it) equals
    stml_run bit for bit."""
    frames = _small()
    kw = dict(n_spatial=2, n_temporal=1, reg="curvature", gn_max=5,
              cg_max=10, parity_mode=True)
    st = STML(8, frames.shape[1:], opts=default_opts(**kw))
    st.set_sequence(torch.from_numpy(frames).cuda())
    print("spml run", flush=True)
    st.run()
    u_ref, ost = oracle.stml_run(frames, oracle.STMLOptions(**kw))
    assert [lg["steps"] for lg in st.logs()] == \
        [lg["steps"] for lg in ost.log]
    assert len(st.logs()) == 2
    assert np.abs(st.get_displacements().cpu().numpy() - u_ref).max() <= 1e-3
    kw3 = dict(kw, n_temporal=2)
    st3 = STML(8, frames.shape[1:], opts=default_opts(**kw3))
    st3.set_sequence(torch.from_numpy(frames).cuda())
    st3.run()
    whole = st3.get_displacements().cpu().numpy()
    st3.set_sequence(torch.from_numpy(frames).cuda())
    print("stml staged", flush=True)
    for lv in range(2):
        for q in range(2):
            st3.predict(lv, q)
            st3.register_level(lv, q)
    assert len(st3.logs()) == 4
    np.testing.assert_array_equal(st3.get_displacements().cpu().numpy(),
                                  whole)


def test_objective_target_stops_registration():
    """stml_set_targets: GIR stops at the first accepted step whose
    objective is at or below the target, and takes no step when the start
    already is; the steps before are those of the run without a target."""
    frames = _small()
    kw = dict(n_spatial=1, n_temporal=2, reg="curvature", alpha=0.1,
              gn_max=8, cg_max=10, tol_J=0.0, tol_u=0.0)
    st = STML(8, frames.shape[1:], opts=default_opts(**kw))
    fr = torch.from_numpy(frames).cuda()
    st.set_sequence(fr)
    st.predict(0, 0)
    st.register_level(0, 0)
    free = st.logs()[0]
    assert free["gn"] == 8
    targets = np.full((1, 2), -np.inf)
    targets[0, 0] = free["J_iter"][2]
    st.set_targets(targets)
    st.set_sequence(fr)
    st.predict(0, 0)
    st.register_level(0, 0)
    lg = st.logs()[0]
    assert lg["gn"] == 3 and lg["J"] == free["J_iter"][2]
    assert lg["steps"] == free["steps"][:3]
    targets[0, 0] = free["J0"]                  # the start meets it
    st.set_targets(targets)
    st.set_sequence(fr)
    st.predict(0, 0)
    st.register_level(0, 0)
    lg = st.logs()[0]
    assert lg["gn"] == 0 and lg["J"] == free["J0"]
    assert torch.count_nonzero(st.get_displacements(0)).item() == 0
    st.set_targets(None)
