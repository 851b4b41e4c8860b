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


# 3-D: (frames, extent, seed), ragged against the 16 x 16 x 16 columns
CASES3 = [(5, (10, 12, 18), 0), (6, (12, 16, 20), 1), (4, (8, 8, 24), 2)]


def _opts3(parity):
    return default_opts(dim=3, n_spatial=2, n_temporal=2, reg="curvature",
                        alpha=0.1, gn_max=3 if parity else 20,
                        cg_max=5 if parity else 20, parity_mode=parity)


@pytest.mark.parametrize("parity,graph", [(True, True), (False, False)])
def test_batch_3d_equals_single_runs(parity, graph):
    singles, batched = [], []
    for n, ext, seed in CASES3:
        f = torch.from_numpy(
            synth.sinusoid_sequence(n, ext, 1.5, 1, 70 + seed)[0]).cuda()
        for group in (singles, batched):
            st = STML(n, ext, opts=_opts3(parity))
            st.set_sequence(f)
            group.append(st)
    print(f"batch 3d parity={parity} graph={graph}", flush=True)
    for a in singles:
        a.run()
    Batch(batched, graph=graph).run()
    torch.cuda.synchronize()
    for a, b in zip(singles, batched):
        _assert_same(a, b)
    if not parity:
        gns = [g["gn"] for b in batched for g in b.logs()]
        assert min(gns) < 20


def test_batched_3d_sequence_matches_oracle():
    kw = dict(n_spatial=2, n_temporal=2, reg="curvature", alpha=0.1,
              gn_max=3, cg_max=5, parity_mode=True)
    sts, frames0 = [], None
    for n, ext, seed in CASES3[:2]:
        f = synth.sinusoid_sequence(n, ext, 1.5, 1, 70 + seed)[0]
        frames0 = f if frames0 is None else frames0
        st = STML(n, ext, opts=default_opts(dim=3, **kw))
        st.set_sequence(torch.from_numpy(f).cuda())
        sts.append(st)
    print("batched 3d vs oracle", flush=True)
    Batch(sts).run()
    ost = oracle.stml.STMLState(frames0, oracle.STMLOptions(**kw))
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
    v = STML(4, (8, 8, 16), opts=default_opts(dim=3, n_spatial=2,
                                              n_temporal=2))
    with pytest.raises(STMLError):
        Batch([a, v])
    # a context without a sequence: the run reports it
    B = Batch([a])
    with pytest.raises(STMLError):
        B.run()


def test_tuning_changes_only_rounding_and_keeps_batch_identity(tmp_path):
    from paper_2001_06613_amd import autotune

    singles, batched = _pair(True)
    tuned = (64, 128, 1024)
    for a, b in zip(singles, batched):
        a.set_tuning(*tuned)
        b.set_tuning(*tuned)
    print("tuned batch", flush=True)
    for a in singles:
        a.run()
    Batch(batched).run()
    for a, b in zip(singles, batched):
        _assert_same(a, b)
    # the default launch shape gives the same result up to float64 rounding
    ref, _ = _pair(True)
    for r in ref:
        r.run()
    for a, r in zip(singles, ref):
        assert a.get_tuning() == {"tile_blocks": 64, "vox_blocks": 128,
                                  "hv_blocks": 1024}
        assert r.get_tuning() == autotune.DEFAULT
        la, lr = a.logs(), r.logs()
        for x, y in zip(la, lr):
            assert x["steps"] == y["steps"]
            assert x["J"] == pytest.approx(y["J"], rel=1e-9)
        diff = (a.get_displacements() - r.get_displacements()).abs().max()
        assert float(diff) <= 1e-4
    with pytest.raises(STMLError):
        singles[0].set_tuning(12, 512, 2048)
    with pytest.raises(STMLError):
        singles[0].set_tuning(512, 2048, 2048)


def test_autotune_picks_a_valid_setting_and_caches_it(tmp_path):
    from paper_2001_06613_amd import autotune

    _, batched = _pair(True)
    B = Batch(batched)
    B.run()
    before = [b.get_displacements().clone() for b in batched]
    path = str(tmp_path / "tune.json")
    print("autotune", flush=True)
    cfg = autotune.tune(batched, batch=B, cache_path=path, repeats=1)
    for name, values in autotune.CANDIDATES.items():
        assert cfg[name] in values
    # the timings restart from, and leave, the registered displacements
    for b, u in zip(batched, before):
        assert torch.equal(b.get_displacements(), u)
        assert b.get_tuning() == {k: cfg[k] for k in autotune.DEFAULT}
    import json
    with open(path) as f:
        cache = json.load(f)
    key = autotune.cache_key(batched, True)
    assert key in cache
    # a second call reads the cache back
    for b in batched:
        b.set_tuning(512, 512, 2048)
    cfg2 = autotune.tune(batched, batch=B, cache_path=path)
    assert {k: cfg2[k] for k in autotune.DEFAULT} == \
        {k: cfg[k] for k in autotune.DEFAULT}
