"""Batched registration of uneven sequences against per-sequence runs.

A batch deals the blocks of every launch to its sequences in the shares each
sequence gets alone, so the batched displacements, objectives and iteration
logs must equal the per-sequence ones bit for bit: with and without the
captured graph, with fixed iteration counts and with the convergence stop.
One batched sequence is also compared with the oracle.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2001_06613_amd import synth
from paper_2001_06613_amd.binding import Batch, STML, STMLError, default_opts

pytestmark = pytest.mark.gpu

# (frames, extent, seed): uneven lengths and shapes, ragged tiles
CASES = [(8, (64, 64), 0), (12, (48, 40), 1), (16, (32, 72), 2),
         (6, (24, 24), 3)]


def _frames(n, shape, seed):
    return synth.sinusoid_sequence(n, shape, 2.0, 2, 50 + seed)[0]


def _opts(parity):
    return default_opts(n_spatial=2, n_temporal=3, reg="curvature",
                        alpha=0.1, gn_max=4 if parity else 25,
                        cg_max=6 if parity else 20, parity_mode=parity)


def _pair(parity):
    singles, batched = [], []
    for n, shape, seed in CASES:
        f = torch.from_numpy(_frames(n, shape, seed)).cuda()
        a = STML(n, shape, opts=_opts(parity))
        a.set_sequence(f)
        b = STML(n, shape, opts=_opts(parity))
        b.set_sequence(f)
        singles.append(a)
        batched.append(b)
    return singles, batched


def _assert_same(a, b):
    for level in range(a.levels):
        ua, ub = a.get_displacements(level), b.get_displacements(level)
        assert torch.equal(ua, ub), f"level {level}"
    la, lb = a.logs(), b.logs()
    assert len(la) == len(lb)
    for x, y in zip(la, lb):
        for key in ("level", "q", "gn", "cg", "steps", "J", "J0", "status"):
            assert x[key] == y[key], key


@pytest.mark.parametrize("parity,graph", [(True, True), (True, False),
                                          (False, True)])
def test_batch_equals_single_runs(parity, graph):
    singles, batched = _pair(parity)
    print(f"batch parity={parity} graph={graph}", flush=True)
    for a in singles:
        a.run()
    B = Batch(batched, graph=graph)
    B.run()
    torch.cuda.synchronize()
    for a, b in zip(singles, batched):
        _assert_same(a, b)
    if not parity:
        # the convergence stop ended some registrations before gn_max
        gns = [g["gn"] for b in batched for g in b.logs()]
        assert min(gns) < 25


def test_batched_sequence_matches_oracle():
    n, shape, seed = CASES[0]
    frames = _frames(n, shape, seed)
    kw = dict(n_spatial=2, n_temporal=3, reg="curvature", alpha=0.1,
              gn_max=3, cg_max=5, parity_mode=True)
    sts = []
    for nn, sh, sd in CASES[:2]:
        st = STML(nn, sh, opts=default_opts(**kw))
        st.set_sequence(torch.from_numpy(_frames(nn, sh, sd)).cuda())
        sts.append(st)
    print("batched vs oracle", flush=True)
    Batch(sts).run()
    ost = oracle.stml.STMLState(frames, oracle.STMLOptions(**kw))
    ost.run()
    for lg, olg in zip(sts[0].logs(), [x for x in ost.log if "q" in x]):
        assert lg["steps"] == olg["steps"]
        assert lg["J"] == pytest.approx(olg["J"], rel=1e-5)
    u = sts[0].get_displacements(1).cpu().numpy()
    assert np.abs(u - ost.Y[1]).max() <= 1e-3


def test_batch_rejects_mismatched_contexts():
    a = STML(8, (32, 32), opts=default_opts(n_spatial=2, n_temporal=2))
    b = STML(8, (32, 32), opts=default_opts(n_spatial=2, n_temporal=3))
    c = STML(8, (32, 32), opts=default_opts(n_spatial=2, n_temporal=2,
                                            eps_stop=1e-3))
    with pytest.raises(STMLError):
        Batch([a, b])
    with pytest.raises(STMLError):
        Batch([a, c])
    with pytest.raises(STMLError):
        Batch([a, a])
    # a context without a sequence: the run reports it
    B = Batch([a])
    with pytest.raises(STMLError):
        B.run()

