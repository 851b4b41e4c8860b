"""The learned predictor inside the schedule (GPU).

* With the trained parameters shipped in the package, held-out synthetic
  sequences of the 64-frame 256x256 workload (and 32-frame 128x128x64
  volumes, with the 3-D network) need fewer corrector Gauss-Newton
  iterations, in total and to reach the objective the paper's predictor
  ends each registration with, and end at a lower objective than with the
  paper's predictor alone.
* The fallback: every prediction step keeps the start guess with the lower
  objective on K_{q+1}, and the registration starts from exactly that
  objective; a net whose correction is zero reproduces the linear
  interpolation, which ties the paper's predictor on the coarsest level
  (the tie keeps the paper's).
* Training end to end (plain-method targets from batched registration,
  Adam steps in the library) lowers the loss.
"""

import numpy as np
import pytest
import torch

from paper_2001_06613_amd import learned
from paper_2001_06613_amd.binding import STML, Net, STMLError

pytestmark = pytest.mark.gpu


def test_trained_predictor_gains_on_held_out_sequences():
    net = Net(8, (256, 256))
    net.set_params(learned.load_params(learned.TRAINED_C2))
    seqs = [(s, learned.sequence(s)) for s in (20000, 20001, 20002)]
    print("learned vs paper predictor, 3 sequences", flush=True)
    rows = learned.compare(net, seqs, opts=learned.schedule_opts(gn_max=40),
                           warmup=0)
    s = learned.summarise(rows)
    print(s, flush=True)
    assert s["corrector_gn_learned"] < s["corrector_gn_plain"]
    assert s["J_final_learned_mean"] < s["J_final_plain_mean"]
    assert s["learned_picks"] > 0
    # at equal objective, stage by stage
    assert s["corrector_gn_to_plain_J"] < s["corrector_gn_plain_matched"]


def test_trained_predictor_3d_gains_on_held_out_volumes():
    n, ext, md = learned.RECIPE[3]
    net = Net(1, ext, dim=3)
    net.set_params(learned.load_params(learned.TRAINED_C5))
    seqs = [(s, learned.sequence(s, n, ext, md)) for s in (21000, 21001)]
    print("3-D learned vs paper predictor, 2 volumes", flush=True)
    rows = learned.compare(net, seqs, opts=learned.schedule_opts(
        dim=3, gn_max=40), warmup=0)
    s = learned.summarise(rows)
    print(s, flush=True)
    assert s["corrector_gn_learned"] < s["corrector_gn_plain"]
    assert s["J_final_learned_mean"] < s["J_final_plain_mean"]
    assert s["learned_picks"] > 0
    # at equal objective, stage by stage
    assert s["corrector_gn_to_plain_J"] < s["corrector_gn_plain_matched"]


def _check_fallback_logs(logs):
    steps = [g for g in logs if g["predictor"] >= 0]
    assert steps
    for g in steps:
        assert g["predictor"] in (0, 1)
        assert np.isfinite(g["J_paper"]) and np.isfinite(g["J_learned"])
        lo = min(g["J_paper"], g["J_learned"])
        assert g["J0"] == pytest.approx(lo, rel=1e-12)
        if g["predictor"] == 1:
            assert g["J_learned"] < g["J_paper"]
    for g in logs:
        if g["q"] == 0:
            assert g["predictor"] == -1
    return steps


def test_fallback_keeps_the_lower_start_objective():
    frames = learned.sequence(20003, 32, (64, 64), 3.0, 3)
    st = STML(32, (64, 64), opts=learned.schedule_opts(n_spatial=2,
                                                       gn_max=10))
    net = Net(8, (64, 64))
    net.set_params(learned.init_params(3))      # untrained
    st.set_predictor_net(net)
    st.set_sequence(torch.from_numpy(frames).cuda())
    print("fallback, untrained net", flush=True)
    st.run()
    _check_fallback_logs(st.logs())
    # zero correction: the learned guess is the linear interpolation
    net.set_params(np.zeros(net.nparam, np.float32))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.run()
    steps = _check_fallback_logs(st.logs())
    coarse = [g for g in steps if g["level"] == 0]
    assert coarse
    for g in coarse:
        assert g["J_learned"] == pytest.approx(g["J_paper"], rel=1e-6)
        assert g["predictor"] == 0 or g["J_learned"] < g["J_paper"]


def test_net_requires_a_context_made_for_it():
    st = STML(8, (32, 32), opts=learned.schedule_opts(predictor=0,
                                                      n_spatial=1))
    with pytest.raises(STMLError):
        st.set_predictor_net(Net(1, (32, 32)))
    # a volume net does not serve an image sequence, nor the reverse
    st2 = STML(8, (32, 32), opts=learned.schedule_opts(n_spatial=1))
    with pytest.raises(STMLError):
        st2.set_predictor_net(Net(1, (8, 16, 16), dim=3))
    st3 = STML(8, (8, 16, 16), opts=learned.schedule_opts(dim=3,
                                                         n_spatial=1))
    with pytest.raises(STMLError):
        st3.set_predictor_net(Net(1, (32, 32)))


def test_fallback_keeps_the_lower_start_objective_3d():
    ext = (16, 16, 32)
    frames = learned.sequence(21100, 16, ext, 2.0, 2)
    st = STML(16, ext, opts=learned.schedule_opts(dim=3, n_spatial=2,
                                                  gn_max=8))
    net = Net(1, ext, dim=3)
    net.set_params(learned.init_params(4, dim=3))      # untrained
    st.set_predictor_net(net)
    st.set_sequence(torch.from_numpy(frames).cuda())
    print("fallback 3d, untrained net", flush=True)
    st.run()
    _check_fallback_logs(st.logs())
    net.set_params(np.zeros(net.nparam, np.float32))
    st.set_sequence(torch.from_numpy(frames).cuda())
    st.run()
    steps = _check_fallback_logs(st.logs())
    coarse = [g for g in steps if g["level"] == 0]
    assert coarse
    for g in coarse:
        assert g["J_learned"] == pytest.approx(g["J_paper"], rel=1e-6)
        assert g["predictor"] == 0 or g["J_learned"] < g["J_paper"]


def test_training_on_plain_method_targets_lowers_the_loss():
    seqs = [(s, learned.sequence(s, 32, (64, 64), 3.0, 3))
            for s in range(31000, 31016)]
    print("dataset of 16 sequences", flush=True)
    ds, _ = learned.build_dataset(
        iter(seqs), len(seqs),
        opts=learned.schedule_opts(predictor=0, n_spatial=2, gn_max=20),
        group=8)
    assert ds.count == 16
    net = Net(8, (64, 64))
    net.set_params(learned.init_params(0))
    losses = learned.train(net, ds, 800, pixels=8 * 64 * 64)
    print("loss", np.mean(losses[:50]), np.mean(losses[-50:]), flush=True)
    assert np.mean(losses[-100:]) < 0.95 * np.mean(losses[:100])
