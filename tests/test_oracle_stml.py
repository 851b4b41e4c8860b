"""Pins of the oracle's STML driver (Sec. 3).

Independent checks: with one temporal level the schedule is the plain
spatial multilevel method (a hand-written loop of restriction, prolongation
and Gauss-Newton); with one spatial level it runs only the temporal levels;
the predictor-corrector schedule lowers the objective below the unregistered
one.
"""

import numpy as np
import pytest

from oracle import (STMLOptions, stml_run, restrict, prolong, gauss_newton,
                    objective_value, level_extents, level_spacing,
                    temporal_sets, linear_predict, ls_predict)
from oracle.stml import STMLState
from paper_2001_06613_amd import synth


def _small():
    frames, g = synth.config_small(0)
    return frames[:, ::2, ::2].copy(), g     # 8 x 32 x 32


def test_single_temporal_level_is_spatial_multilevel():
    frames, _ = _small()
    opts = STMLOptions(n_spatial=2, n_temporal=1, gn_max=2, cg_max=4,
                       parity_mode=True)
    u, st = stml_run(frames, opts)
    # hand-written SpML: coarse GN on all frames, prolong, fine GN
    coarse = restrict(frames)
    par = opts.params()
    allk = list(range(8))
    r0 = gauss_newton(coarse, np.zeros((8, 2, 16, 16)), allk, 2.0, par,
                      gn_max=2, cg_max=4, fixed=True)
    r1 = gauss_newton(frames, prolong(r0.u, (32, 32)), allk, 1.0, par,
                      gn_max=2, cg_max=4, fixed=True)
    np.testing.assert_array_equal(u, r1.u)


def test_single_spatial_level_runs_temporal_levels():
    frames, _ = _small()
    opts = STMLOptions(n_spatial=1, n_temporal=2, gn_max=2, cg_max=4,
                       parity_mode=True)
    u, st = stml_run(frames, opts)
    assert [e["nK"] for e in st.log] == [5, 8]
    assert [e["level"] for e in st.log] == [0, 0]


def test_stml_lowers_objective():
    frames, _ = _small()
    opts = STMLOptions(n_spatial=2, n_temporal=2, gn_max=4, cg_max=10)
    u, st = stml_run(frames, opts)
    par = opts.params()
    J0 = objective_value(frames, np.zeros_like(u), range(8), 1.0, par)[0]
    J1 = objective_value(frames, u, range(8), 1.0, par)[0]
    assert J1 < 0.5 * J0
    assert [(e["level"], e["nK"]) for e in st.log] == \
        [(0, 5), (0, 8), (1, 5), (1, 8)]


def test_stopping_rule_ends_level_early():
    frames, _ = _small()
    opts = STMLOptions(n_spatial=1, n_temporal=3, gn_max=3, cg_max=5,
                       eps_stop=1e6)         # always met at q = 1
    u, st = stml_run(frames, opts)
    assert any(e.get("stop_at_q") == 1 for e in st.log)
    assert [e["nK"] for e in st.log if "nK" in e] == [3, 5]


# --- hand-written schedules -------------------------------------------------

def _nine():
    """9 frames of 32 x 32: K_0 = {0, 4, 8}, K_1 = {0, 2, 4, 6, 8}, K_2 = all
    for three temporal levels."""
    return synth.sinusoid_sequence(9, (32, 32), 2.0, 2, seed=5)[0]


def _by_hand(frames, L, T1, gn, cg, beta, fixed, eq3_trace=None):
    """The schedule of Sec. 3 written out from the primitives:

    coarsest level: z(0,0) = Id, y = GIR(K_0, z); z(q+1) = linear
    interpolation of y over K_q (injection on K_q); y = GIR(K_{q+1}, z(q+1)).
    finer levels: z(l,0) = prolongation of y(l-1,T,all); then
    z(l,q+1) = argmin of eq. (2) with eta = y(l,q) on K_q and
    omega = z(l,q,all), the start guess of the temporal level just
    registered (= the prolonged y(l-1,T,all) for q = 0).

    When eq3_trace is a list, appends per level the list of
    (D over all frames at the prediction with K_q as registered,
     D over all frames at the plain prediction,
     D over K_q at y(l,q)).
    """
    par = STMLOptions().params()
    n = frames.shape[0]
    pyr = [np.asarray(frames, np.float64)]
    for _ in range(L - 1):
        pyr.append(restrict(pyr[-1]))
    pyr = pyr[::-1]
    ext = level_extents(frames.shape[1:], L)
    Ks = temporal_sets(n, T1)
    y = None
    for lvl in range(L):
        h = level_spacing(L, lvl)
        z = np.zeros((n, 2) + ext[lvl]) if lvl == 0 else prolong(y, ext[lvl])
        y = gauss_newton(pyr[lvl], z, Ks[0], h, par, gn_max=gn, cg_max=cg,
                         fixed=fixed).u
        rows = []
        for q in range(T1 - 1):
            if lvl == 0:
                z = linear_predict(y, Ks[q])
            else:
                z = ls_predict(y, z, Ks[q], beta)
            if eq3_trace is not None:
                est = z.copy()
                est[Ks[q]] = y[Ks[q]]
                rows.append((objective_value(pyr[lvl], est, range(n), h,
                                             par)[1],
                             objective_value(pyr[lvl], z, range(n), h,
                                             par)[1],
                             objective_value(pyr[lvl], y, Ks[q], h, par)[1]))
            y = gauss_newton(pyr[lvl], z, Ks[q + 1], h, par, gn_max=gn,
                             cg_max=cg, fixed=fixed).u
        if eq3_trace is not None:
            eq3_trace.append(rows)
    return y


def test_hand_written_schedule_with_eq2_reference():
    frames = _nine()
    opts = STMLOptions(n_spatial=2, n_temporal=3, gn_max=2, cg_max=4,
                       parity_mode=True)
    u, st = stml_run(frames, opts)
    ref = _by_hand(frames, 2, 3, 2, 4, opts.beta, True)
    np.testing.assert_array_equal(u, ref)
    assert [(e["level"], e["nK"]) for e in st.log] == \
        [(0, 3), (0, 5), (0, 9), (1, 3), (1, 5), (1, 9)]


def test_eq2_reference_is_the_start_guess_not_the_estimate():
    # omega := y(l,q,all) (the current estimate) would make the prediction
    # the estimate itself on every frame; omega := z(l,q,all) does not
    frames = _nine()
    opts = STMLOptions(n_spatial=2, n_temporal=2, gn_max=2, cg_max=4,
                       parity_mode=True)
    st = STMLState(frames, opts)
    st.predict(0, 0)
    st.register_level(0, 0)
    st.predict(0, 1)
    st.register_level(0, 1)
    st.predict(1, 0)
    z0 = st.Z[1].copy()
    st.register_level(1, 0)
    y0 = st.Y[1].copy()
    st.predict(1, 1)
    np.testing.assert_array_equal(st.Z[1], ls_predict(y0, z0, st.K[0],
                                                      opts.beta))
    assert np.max(np.abs(st.Z[1] - ls_predict(y0, y0, st.K[0], opts.beta))) \
        > 1e-3


def test_eq3_trace_is_all_frames_with_registered_subset():
    frames = _nine()
    # beta large enough that eq. (2) visibly departs from eta on K_q
    opts = STMLOptions(n_spatial=2, n_temporal=3, gn_max=2, cg_max=4,
                       beta=0.5, eps_stop=1e-300)  # enabled, never met
    u, st = stml_run(frames, opts)
    trace = []
    ref = _by_hand(frames, 2, 3, 2, 4, opts.beta, False, eq3_trace=trace)
    np.testing.assert_array_equal(u, ref)
    assert st.stop_q == [-1, -1]
    for lvl in range(2):
        np.testing.assert_allclose(st.stop_trace[lvl],
                                   [r[0] for r in trace[lvl]], rtol=1e-12)
    # on the finer level eq. (2) does not reproduce eta on K_q, so the
    # injected estimate differs from the plain prediction there
    inj = np.array([r[0] for r in trace[1]])
    plain = np.array([r[1] for r in trace[1]])
    assert np.all(np.abs(inj - plain) > 1e-4 * np.abs(inj))


def test_eq3_absolute_all_frame_decisions():
    frames = _nine()
    base = dict(n_spatial=1, n_temporal=3, gn_max=2, cg_max=4)
    trace = []
    _by_hand(frames, 1, 3, 2, 4, 1e-5, False, eq3_trace=trace)
    (Da0, _, Dk0), (Da1, _, Dk1) = trace[0]
    dD = abs(Da1 - Da0)           # all frames, as eq. (3) is read
    dK = abs(Dk1 - Dk0)           # K_q only
    assert abs(Da1) > 2.0         # relative and absolute tests differ
    assert max(dD, dK) > 1.5 * min(dD, dK)

    def run(eps, relative=False):
        return stml_run(frames, STMLOptions(eps_stop=eps,
                                            stop_relative=relative, **base))

    # fires at q = 1: K_2 is never registered, y is the injected estimate
    u, st = run(2.0 * dD)
    assert st.stop_q == [1]
    assert [e["nK"] for e in st.log if "nK" in e] == [3, 5]
    np.testing.assert_allclose(st.stop_trace[0], [Da0, Da1], rtol=1e-12)
    # never fires
    u, st = run(0.5 * dD)
    assert st.stop_q == [-1]
    assert [e["nK"] for e in st.log if "nK" in e] == [3, 5, 9]
    # absolute, not relative: eps between dD/|D| and dD
    eps = 0.5 * (dD / abs(Da1) + dD)
    assert run(eps)[1].stop_q == [-1]
    assert run(eps, relative=True)[1].stop_q == [1]
    # all frames, not K_q only: eps between the two changes
    eps = 0.5 * (dD + dK)
    assert run(eps)[1].stop_q == ([1] if dD <= eps else [-1])
    assert (dD <= eps) != (dK <= eps)
