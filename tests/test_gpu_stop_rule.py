"""GPU parity of the eq. (3) stopping rule and of Gauss-Newton steps that
CG or the Armijo search leave empty.

Eq. (3) (Sec. 3): from q = 1 on, a spatial level stops when D over all
frames, at the estimate after the prediction from K_q, changed by at most
eps.  The oracle's trace without a stop fixes two tolerances: 2|D_1 - D_0|
of the coarsest level (the rule fires at q = 1 on every level, at least a
factor 1.5 from its threshold) and half the smallest change (it never
fires).  Convergence exits of CG and Gauss-Newton are switched off
(cg_rtol = tol_J = tol_u = 0) so that the rule is the only decision.  The
stop q, the D trace, the accepted steps and u must agree with the oracle.

No-step cases: a context whose workspace starts as NaN bytes must give the
zero direction of CG from x0 = 0 when CG takes no step (cg_max = 0, or
r.z = 0 at identical frames), single and batched, and an Armijo search
that finds no step (ls_max = 0 where the oracle backtracks) must report
STML_WLINESEARCH with the last accepted iterate.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2001_06613_amd import synth
from paper_2001_06613_amd.binding import STML, Batch, default_opts

pytestmark = pytest.mark.gpu

EQ3_CASES = {
    "2d": (lambda: synth.sinusoid_sequence(9, (32, 32), 2.0, 2, seed=5)[0],
           dict(n_spatial=2, n_temporal=3, gn_max=3, cg_max=5,
                reg="curvature", alpha=0.1)),
    "3d": (lambda: synth.sinusoid_sequence(9, (12, 16, 20), 1.5, 1,
                                           seed=23)[0],
           dict(dim=3, n_spatial=1, n_temporal=3, gn_max=3, cg_max=5,
                reg="curvature", alpha=0.1)),
}
NO_EXITS = dict(tol_J=0.0, tol_u=0.0, cg_rtol=0.0)


def _oracle(frames, eps, kw):
    okw = {k: v for k, v in kw.items() if k != "dim"}
    return oracle.stml_run(frames, oracle.STMLOptions(eps_stop=eps,
                                                      **NO_EXITS, **okw))


@pytest.mark.parametrize("case", ["2d", "3d"])
@pytest.mark.parametrize("mode", ["fires", "never"])
def test_eq3_stop_rule_parity(case, mode):
    make, kw = EQ3_CASES[case]
    frames = make()
    n = frames.shape[0]
    _, free = _oracle(frames, 1e-300, kw)
    changes = [abs(t[1] - t[0]) for t in free.stop_trace]
    eps = 2.0 * changes[0] if mode == "fires" else 0.5 * min(changes)
    u_ref, ost = _oracle(frames, eps, kw)
    for tr in ost.stop_trace:                 # decisions far from eps
        if len(tr) >= 2:
            ratio = abs(tr[1] - tr[0]) / eps
            assert ratio <= 2.0 / 3.0 or ratio >= 1.5
    want = [1] * kw["n_spatial"] if mode == "fires" else \
        [-1] * kw["n_spatial"]
    assert ost.stop_q == want
    print(f"eq3 {case} {mode} eps={eps:.6g} oracle trace {ost.stop_trace}",
          flush=True)
    st = STML(n, frames.shape[1:], opts=default_opts(eps_stop=eps,
                                                     **NO_EXITS, **kw))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.run()
    for lvl in range(kw["n_spatial"]):
        tr, q = st.stop_trace(lvl)
        print(f"  level {lvl}: gpu trace {tr} stop {q}", flush=True)
        assert q == ost.stop_q[lvl]
        np.testing.assert_allclose(tr, ost.stop_trace[lvl], rtol=1e-5)
    logs, ologs = st.logs(), [e for e in ost.log if "nK" in e]
    assert [(lg["level"], lg["nK"]) for lg in logs] == \
        [(e["level"], e["nK"]) for e in ologs]
    assert [lg["steps"] for lg in logs] == [e["steps"] for e in ologs]
    u = st.get_displacements().cpu().numpy()
    assert np.abs(u - u_ref).max() <= 1e-3


def test_eq3_relative_option():
    make, kw = EQ3_CASES["2d"]
    frames = make()
    _, free = _oracle(frames, 1e-300, kw)
    tr = free.stop_trace[0]
    d = abs(tr[1] - tr[0])
    eps = 0.5 * (d / abs(tr[1]) + d)      # relative fires, absolute not
    st = STML(9, frames.shape[1:], opts=default_opts(
        eps_stop=eps, stop_relative=True, **NO_EXITS, **kw))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.run()
    assert st.stop_trace(0)[1] == 1
    st = STML(9, frames.shape[1:], opts=default_opts(
        eps_stop=eps, **NO_EXITS, **kw))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.run()
    assert st.stop_trace(0)[1] == -1


NAN_BYTES = 0xFF            # every float32 of the workspace is a NaN


def _oracle_register(frames, K, kw):
    ost = oracle.stml.STMLState(frames, oracle.STMLOptions(**kw))
    ost.predict(0, 0)
    res = ost.register_level(0, 0)
    return ost, res


@pytest.mark.parametrize("dim", [2, 3])
def test_cg_max_zero_gives_zero_direction(dim):
    if dim == 2:
        frames = synth.config_small(0)[0][:, ::2, ::2].copy()
    else:
        frames = synth.sinusoid_sequence(5, (10, 12, 18), 1.5, 1, 21)[0]
    n, ext = frames.shape[0], frames.shape[1:]
    kw = dict(n_spatial=1, n_temporal=2, gn_max=3, cg_max=0,
              parity_mode=True)
    st = STML(n, ext, opts=default_opts(dim=dim, **kw),
              workspace_fill=NAN_BYTES)
    st.set_sequence(torch.from_numpy(frames).cuda())
    u = synth.random_displacement(ext, n, 1.0, 3)
    K = [0, n - 1]
    delta, iters = st.gn_direction(0, K, torch.from_numpy(u))
    assert iters == 0
    assert torch.count_nonzero(delta).item() == 0
    st.predict(0, 0)
    assert st.register_level(0, 0) == 0
    lg = st.logs()[0]
    ost, res = _oracle_register(frames, K, kw)
    assert lg["steps"] == res.steps == [1.0] * 3
    assert lg["status"] == 0 and res.status == "ok"
    assert torch.count_nonzero(st.get_displacements(0)).item() == 0


def test_identical_frames_give_zero_direction_single_and_batched():
    f = synth.base_image(np.random.default_rng(3), (40, 40)).astype(
        np.float32)
    frames = np.repeat(f[None], 5, axis=0)
    kw = dict(n_spatial=1, n_temporal=2, gn_max=2, cg_max=4,
              parity_mode=True)
    sts = []
    for _ in range(2):
        st = STML(5, (40, 40), opts=default_opts(**kw),
                  workspace_fill=NAN_BYTES)
        st.set_sequence(torch.from_numpy(frames).cuda())
        sts.append(st)
    delta, iters = sts[0].gn_direction(0, [0, 2, 4],
                                       torch.zeros(5, 2, 40, 40))
    assert iters == 0 and torch.count_nonzero(delta).item() == 0
    sts[0].predict(0, 0)
    sts[0].register_level(0, 0)
    lg = sts[0].logs()[0]
    assert lg["steps"] == [1.0, 1.0] and lg["J"] == 0.0
    assert torch.count_nonzero(sts[0].get_displacements(0)).item() == 0
    # batched, cg_max = 0 as well
    for cg in (4, 0):
        bs = [STML(5, (40, 40), opts=default_opts(**dict(kw, cg_max=cg)),
                   workspace_fill=NAN_BYTES) for _ in range(2)]
        for b in bs:
            b.set_sequence(torch.from_numpy(frames).cuda())
        B = Batch(bs)
        B.run()
        for b in bs:
            u = b.get_displacements()
            assert torch.count_nonzero(u).item() == 0
            assert all(lg["steps"] == [1.0, 1.0] for lg in b.logs())
        B.close()


def test_linesearch_failure_warning_parity():
    # the oracle backtracks (t = 1/2) at the sixth iteration of this
    # registration; with ls_max = 0 no step qualifies there (t = 1 misses
    # the Armijo bound by 1.7e-3 |J|)
    frames = synth.config_small(0)[0]
    kw = dict(n_spatial=1, n_temporal=2, reg="diffusion", gn_max=6,
              cg_max=10, ls_max=0, parity_mode=True)
    st = STML(8, frames.shape[1:], opts=default_opts(**kw))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.predict(0, 0)
    rc = st.register_level(0, 0)
    ost, res = _oracle_register(frames, [0, 2, 4, 6, 7], kw)
    assert res.status == "linesearch" and res.iterations == 5
    lg = st.logs()[0]
    assert rc == 2 and lg["status"] == 2          # STML_WLINESEARCH
    assert lg["gn"] == 5 and lg["steps"] == res.steps
    u = st.get_displacements(0).cpu().numpy()
    assert np.abs(u - res.u).max() <= 1e-3
