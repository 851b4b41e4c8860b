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
                    objective_value, level_extents)
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
