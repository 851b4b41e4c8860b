#!/usr/bin/env python
"""Throughput benchmark of the STML registration path on one MI355X.

One step = one whole spatio-temporal multilevel solve of a 64-frame
256x256 synthetic OCT-like sequence (4 spatial x 3 temporal levels,
curvature regulariser, fixed 5 Gauss-Newton x 10 CG iterations per
registration): restriction, prolongation, the temporal predictors and every
Gauss-Newton / PCG / Armijo step, all in libstml.so.  The frames are in HBM
before the timed region starts.

value = voxel-frames pushed through the warp+distance+gradient kernel and
the Hessian-product kernel per second, over the whole step: every
evaluation and every Hessian product over a subset K on a level with N
voxels counts |K| N voxel-frames.  The Armijo trial sweeps, CG vector
updates, predictors and host synchronisation are inside the timed region
but not counted as units.

Prints one JSON line.  Besides the contract's fields it carries the
per-kernel breakdown, a small solve, the 32-sequence batch, the learned
predictor against the paper's (images and volumes), the volume workload,
SpML against STML (the paper's comparison) and the CPU oracle's rate.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
COPY_BYTES = 512 << 20         # plain copy that scales the HBM counters
AUTOTUNE_CACHE = os.environ.get(
    "STML_AUTOTUNE_CACHE",
    os.path.join(ROOT, "paper_2001_06613_amd", "data", "autotune.json"))
# The dominant kernel of the solve (largest share of GPU time in the
# per-kernel breakdown) is timed live in the timed region.  Its algorithmic
# bytes per launch come from the library: every field it must read and
# write, once, in float32 (e.g. the CG update: read p, q, dW/du, r, x and
# write x, r, z -> 32 B per component and voxel-frame).
DOMINANT = "cg_update"
TIME_EVERY = 7
DOMINANT_NAME = "cgv_update_kernel<2, *> (CG vector update, all levels)"

WORKLOAD = dict(n=64, extent=(256, 256), n_spatial=4, n_temporal=3,
                reg="curvature", alpha=0.1, lam=1e-2, beta=1e-5, gn_max=5,
                cg_max=10, parity_mode=True)
VOLUME = dict(n=32, extent=(128, 128, 64), n_spatial=3, n_temporal=3,
              gn_max=5, cg_max=10)


def _units(logs, extents):
    total = 0.0
    for lg in logs:
        N = float(np.prod(extents[lg["level"]]))
        for cg in lg["cg"]:
            total += lg["nK"] * N * (1 + cg)
    return total


def _traffic_record():
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current sources."""
    from paper_2001_06613_amd import pmc_traffic

    path = os.path.join(ROOT, "profiles", "cg_update_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != pmc_traffic.source_sha():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(frames, budget_s=10.0):
    """Oracle timed on the host, one thread: Gauss-Newton iterations
    (evaluation, 10 CG Hessian products, Armijo search) over all 64 frames
    at the finest level, from zero displacement, repeated until budget_s
    seconds have passed."""
    from threadpoolctl import threadpool_limits

    import oracle

    w = WORKLOAD
    par = oracle.ModelParams(alpha=w["alpha"], lam=w["lam"], reg=w["reg"])
    n = frames.shape[0]
    u0 = np.zeros((n, 2) + frames.shape[1:])
    units, reps = 0.0, 0
    with threadpool_limits(1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            res = oracle.gauss_newton(frames, u0, list(range(n)), 1.0, par,
                                      gn_max=1, cg_max=w["cg_max"],
                                      fixed=True)
            units += n * float(np.prod(frames.shape[1:])) * (
                1 + res.cg_iterations[0])
            reps += 1
        dt = time.perf_counter() - t0
    return {"value": units / dt / 1e9, "unit": "Gvoxel-frames/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{reps} x one Gauss-Newton iteration (1 evaluation + "
                      "10 Hessian products + CG + Armijo) over 64 frames x "
                      "256x256 at the finest level, NumPy float64, one "
                      f"thread, {dt:.1f} s"}


HALO_ROWS = 8    # slab halo: Armijo trial steps move up to a few pixels


def _slab_worker(args):
    """One row slab (with halo rows) of the 64-frame 256x256 level: the
    oracle's Gauss-Newton iteration repeated for budget_s seconds on one
    thread; returns (voxel-frame units of its own rows, seconds)."""
    frames, r0, r1, budget_s = args
    from threadpoolctl import threadpool_limits

    import oracle

    w = WORKLOAD
    par = oracle.ModelParams(alpha=w["alpha"], lam=w["lam"], reg=w["reg"])
    lo, hi = max(r0 - HALO_ROWS, 0), min(r1 + HALO_ROWS, frames.shape[1])
    sl = np.ascontiguousarray(frames[:, lo:hi])
    n = sl.shape[0]
    u0 = np.zeros((n, 2) + sl.shape[1:])
    own = n * (r1 - r0) * sl.shape[2]
    units = 0.0
    with threadpool_limits(1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            res = oracle.gauss_newton(sl, u0, list(range(n)), 1.0, par,
                                      gn_max=1, cg_max=w["cg_max"],
                                      fixed=True)
            units += own * (1 + res.cg_iterations[0])
        dt = time.perf_counter() - t0
    return units, dt


def cpu_baseline_slabs(frames, budget_s=10.0):
    """The same oracle iteration on row slabs in parallel processes (one
    thread each), each slab holding all frames of its rows plus halo rows:
    the oracle on this host's cores."""
    import multiprocessing as mp

    cores = min(16, len(os.sched_getaffinity(0)))
    H = frames.shape[1]
    edges = [round(H * i / cores) for i in range(cores + 1)]
    jobs = [(frames, edges[i], edges[i + 1], budget_s) for i in range(cores)]
    with mp.get_context("fork").Pool(cores) as pool:
        out = pool.map(_slab_worker, jobs, chunksize=1)
    units = sum(u for u, _ in out)
    span = max(dt for _, dt in out)
    return {"value": units / span / 1e9, "unit": "Gvoxel-frames/s",
            "cores": cores, "kind": "oracle",
            "sample": f"{cores} row slabs of 64 frames x 256x256 ({HALO_ROWS} "
                      "halo rows each), one process and thread per slab, "
                      "each repeating one Gauss-Newton iteration (1 "
                      "evaluation + 10 Hessian products + CG + Armijo) for "
                      f"{budget_s:.0f} s; rate over the slowest worker's "
                      "timed span"}


def _oracle_schedule_worker(args):
    """Seconds of the oracle's whole schedule on one batch sequence, one
    thread."""
    (n, side, seed), kw = args
    from threadpoolctl import threadpool_limits

    import oracle

    f = _gen_batch_sequence((n, side, seed))
    with threadpool_limits(1):
        t0 = time.perf_counter()
        oracle.stml_run(f, oracle.STMLOptions(**kw))
        return time.perf_counter() - t0


def oracle_batch_extrapolation():
    """The oracle's whole schedule (fixed 5 GN x 10 CG) on the two smallest
    of the 32 batch sequences, one thread each (two processes); seconds per
    voxel-frame times the batch's voxel-frames gives the extrapolated oracle
    time of the batch."""
    from paper_2001_06613_amd import synth

    w = WORKLOAD
    cfg = synth.config_batch()
    total_vf = float(sum(n * side * side for n, side, _ in cfg))
    small = sorted(cfg, key=lambda c: c[0] * c[1] ** 2)[:2]
    kw = dict(n_spatial=w["n_spatial"], n_temporal=w["n_temporal"],
              reg=w["reg"], alpha=w["alpha"], gn_max=w["gn_max"],
              cg_max=w["cg_max"], parity_mode=True)
    import multiprocessing as mp

    with mp.get_context("fork").Pool(2) as pool:
        res = pool.map(_oracle_schedule_worker, [(c, kw) for c in small],
                       chunksize=1)
    secs = sum(r for r in res)
    vf = float(sum(n * side * side for n, side, _ in small))
    return {"sequences": [[n, side] for n, side, _ in small],
            "oracle_s": round(secs, 2), "voxel_frames": vf,
            "s_per_voxel_frame": secs / vf,
            "batch_voxel_frames": total_vf,
            "batch_oracle_s_extrapolated": round(secs / vf * total_vf, 1),
            "cores": 1}


def _gen_batch_sequence(args):
    from paper_2001_06613_amd import synth

    n, side, seed = args
    return synth.sinusoid_sequence(n, (side, side), 5.0, 3, seed)[0]


def batched_comparison(seqs, log):
    """The 32 uneven sequences (16..128 frames, 128..512 px squares, the
    main workload's schedule and fixed iterations) solved one after the
    other and as one batch (autotuned launch shapes); both must give
    bit-identical displacements."""
    import torch
    from paper_2001_06613_amd import autotune
    from paper_2001_06613_amd.binding import STML, Batch, default_opts

    w = WORKLOAD
    opts = default_opts(n_spatial=w["n_spatial"], n_temporal=w["n_temporal"],
                        reg=w["reg"], alpha=w["alpha"], lam=w["lam"],
                        beta=w["beta"], gn_max=w["gn_max"],
                        cg_max=w["cg_max"], parity_mode=True)
    sts = [STML(f.shape[0], f.shape[1:], opts=opts) for f in seqs]
    dev = [torch.from_numpy(f).cuda() for f in seqs]
    vf = float(sum(f.size for f in seqs))
    B = Batch(sts)
    _set_all(sts, dev)
    cfg = autotune.tune(sts, batch=B, cache_path=AUTOTUNE_CACHE, repeats=1)
    log("batch: launch shapes " + json.dumps(
        {k: cfg[k] for k in autotune.DEFAULT}))

    def timed(fn):
        _set_all(sts, dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    timed(lambda: sts[0].run())           # warm-up
    t_loop = timed(lambda: [s.run() for s in sts])
    ref = [s.get_displacements().cpu() for s in sts]
    log("batch: looped done")
    t_batch = timed(B.run)
    same = all(torch.equal(r, s.get_displacements().cpu())
               for r, s in zip(ref, sts))
    log("batch: batched done")
    B.close()
    for s in sts:
        s.close()
    return {"workload": "32 uneven sequences (16-128 frames, 128-512 px), "
                        "same schedule and fixed iterations",
            "voxel_frames": vf, "looped_ms": round(1e3 * t_loop, 1),
            "batched_ms": round(1e3 * t_batch, 1),
            "speedup": round(t_loop / t_batch, 3), "identical": same,
            "tuning": {k: cfg[k] for k in autotune.DEFAULT}}


def _gen_volume_sequence(args):
    from paper_2001_06613_amd import synth

    n, seed = args
    if seed == 3:
        return synth.config_volume(seed)[0]
    return synth.sinusoid_sequence(n, VOLUME["extent"], 4.0, 3, seed)[0]


LEARNED3D_SEEDS = (21000, 21001)   # held out from the 3-D training seeds


def volume_comparison(single, seqs, log):
    """3-D: the 32-frame 128x128x64 volume solved alone (3 spatial x 3
    temporal levels, curvature alpha 0.1, fixed 5 GN x 10 CG), then four
    volumes of 24..40 frames looped and batched (bit-identical results)."""
    import torch
    from paper_2001_06613_amd.binding import STML, Batch, default_opts

    v = VOLUME
    opts = default_opts(dim=3, n_spatial=v["n_spatial"],
                        n_temporal=v["n_temporal"], reg="curvature",
                        alpha=0.1, gn_max=v["gn_max"], cg_max=v["cg_max"],
                        parity_mode=True)

    def sync_time(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    st = STML(single.shape[0], single.shape[1:], opts=opts)
    fr = torch.from_numpy(single).cuda()
    solve = lambda: (st.set_sequence(fr), st.run())  # noqa: E731
    solve()
    t_single = min(sync_time(solve) for _ in range(2))
    ext = [st.level_extent(l) for l in range(v["n_spatial"])]
    units = _units(st.logs(), ext)
    st.timing(True)
    solve()
    st.timing(False)
    kern = {}
    for k in ("eval", "hessvec", "cg_update"):
        t = st.timing_get(k)
        kern[k] = {"ms": round(t["ms"], 3), "launches": t["launches"],
                   "GBs": round(t["bytes"] / (t["ms"] * 1e-3) / 1e9, 1)}
    st.close()
    del fr
    log("volume: single done")

    sts = [STML(f.shape[0], f.shape[1:], opts=opts) for f in seqs]
    dev = [torch.from_numpy(f).cuda() for f in seqs]
    B = Batch(sts)

    def run_loop():
        _set_all(sts, dev)
        for s in sts:
            s.run()

    def run_batch():
        _set_all(sts, dev)
        B.run()

    run_loop()
    t_loop = sync_time(run_loop)
    ref = [s.get_displacements().cpu() for s in sts]
    run_batch()
    t_batch = sync_time(run_batch)
    same = all(torch.equal(r, s.get_displacements().cpu())
               for r, s in zip(ref, sts))
    log("volume: batch done")
    B.close()
    for s in sts:
        s.close()
    return {"workload": "32 x 128x128x64 volumes, 3 spatial x 3 temporal "
                        "levels, curvature alpha 0.1, fixed 5 GN x 10 CG",
            "solve_ms": round(1e3 * t_single, 1),
            "value": round(units / t_single / 1e9, 3),
            "unit": "Gvoxel-frames/s", "kernels_one_solve": kern,
            "batch": {"frames": [int(f.shape[0]) for f in seqs],
                      "looped_ms": round(1e3 * t_loop, 1),
                      "batched_ms": round(1e3 * t_batch, 1),
                      "speedup": round(t_loop / t_batch, 3),
                      "identical": same}}


def _set_all(sts, dev):
    for s, f in zip(sts, dev):
        s.set_sequence(f)
    return True


def _round4(v):
    if isinstance(v, float):
        return round(v, 4)
    if isinstance(v, dict):
        return {k: _round4(x) for k, x in v.items()}
    return v


def learned_comparison(seqs, log):
    """Paper's predictor vs the shipped learned one on held-out 64-frame
    256x256 sequences (convergence-controlled Gauss-Newton)."""
    from paper_2001_06613_amd import learned
    from paper_2001_06613_amd.binding import Net

    net = Net(8, WORKLOAD["extent"])
    net.set_params(learned.load_params(learned.TRAINED_C2))
    rows = learned.compare(net, seqs, opts=learned.schedule_opts(gn_max=40))
    s = learned.summarise(rows)
    log("learned: comparison done")
    net.close()
    return {"sequences": len(rows), "seeds": [r["seed"] for r in rows],
            **{k: _round4(v) for k, v in s.items() if k != "sequences"}}


def copy_ceiling(nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes (read + write), median GB/s."""
    import torch

    x = torch.ones(nbytes // 4, device="cuda")
    y = torch.empty_like(x)
    ts = []
    for _ in range(reps + 1):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    del x, y
    return 2 * nbytes / (float(np.median(ts[1:])) * 1e-3) / 1e9


def small_solve(reps=20):
    """The 8-frame 64x64 sequence (diffusion alpha 1e-2, 2 spatial x 2
    temporal levels, fixed 5 GN x 10 CG): launch-bound, reported without a
    roofline claim."""
    import torch
    from paper_2001_06613_amd import synth
    from paper_2001_06613_amd.binding import STML, default_opts

    frames, _ = synth.config_small(0)
    opts = default_opts(n_spatial=2, n_temporal=2, reg="diffusion",
                        alpha=1e-2, gn_max=5, cg_max=10, parity_mode=True)
    st = STML(8, frames.shape[1:], opts=opts)
    fr = torch.from_numpy(frames).cuda()

    def solve():
        st.set_sequence(fr)
        st.run()

    solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        solve()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    units = _units(st.logs(), [st.level_extent(l) for l in range(2)])
    st.close()
    return {"workload": "8 frames x 64x64, 2 x 2 levels, fixed 5 GN x 10 CG",
            "solve_ms": round(ms, 2), "value": round(units / ms / 1e6, 3),
            "unit": "Gvoxel-frames/s"}


def oracle_full():
    """The oracle's whole schedule on the 8-frame 64x64 and the 64-frame
    256x256 sequences (fixed iterations), on this host's cores."""
    import oracle
    from paper_2001_06613_amd import synth

    # BLAS and OpenMP pools limited to one thread; the affinity set is what
    # the host offers
    out = {"threads": 1, "available_cores": len(os.sched_getaffinity(0)),
           "cpu_count": os.cpu_count()}
    f1, _ = synth.config_small(0)
    kw1 = dict(n_spatial=2, n_temporal=2, reg="diffusion", alpha=1e-2,
               gn_max=5, cg_max=10, parity_mode=True)
    from threadpoolctl import threadpool_limits

    lim = threadpool_limits(1)
    t0 = time.perf_counter()
    oracle.stml_run(f1, oracle.STMLOptions(**kw1))
    out["small_s"] = round(time.perf_counter() - t0, 2)
    w = WORKLOAD
    f2, _ = synth.config_large(1)
    kw2 = dict(n_spatial=w["n_spatial"], n_temporal=w["n_temporal"],
               reg=w["reg"], alpha=w["alpha"], gn_max=w["gn_max"],
               cg_max=w["cg_max"], parity_mode=True)
    t0 = time.perf_counter()
    oracle.stml_run(f2, oracle.STMLOptions(**kw2))
    out["large_s"] = round(time.perf_counter() - t0, 2)
    lim.unregister()
    print(json.dumps({"oracle_full": out}), flush=True)


def learned3d_comparison(seqs, log):
    """Paper's predictor vs the shipped 3-D learned one on held-out
    32-frame 128x128x64 volumes (convergence-controlled Gauss-Newton)."""
    from paper_2001_06613_amd import learned
    from paper_2001_06613_amd.binding import Net

    net = Net(1, VOLUME["extent"], dim=3)
    net.set_params(learned.load_params(learned.TRAINED_C5))
    rows = learned.compare(net, seqs, opts=learned.schedule_opts(
        dim=3, gn_max=40), warmup=0)
    s = learned.summarise(rows)
    log("learned 3-D: comparison done")
    net.close()
    return {"sequences": len(rows), "seeds": [r["seed"] for r in rows],
            **{k: _round4(v) for k, v in s.items() if k != "sequences"}}


def multilevel_comparison(frames, dim, log, reps):
    """The paper's comparison (Sec. 4, Table 1) in this model: the spatial
    multilevel strategy (SpML: every frame registered on every spatial
    level, i.e. one temporal level) against STML with three temporal levels
    (and STML with the eq. (3) stop, eps 1e-3); same inner solver, the
    paper's predictors, convergence-controlled Gauss-Newton (gn_max 40).
    Reported per variant: the wall time of the whole schedule (median of
    `reps` solves) and, from one more solve driven stage by stage (every
    entry point returns synchronised), the time and Gauss-Newton iterations
    of each spatial level, D over all frames relative to the unregistered
    D, and the relative difference of the finest-level displacements from
    SpML's.  Because the variants stop at different objectives, STML's time
    to reach SpML's final objective is estimated too: the stages before the
    last in full, the last one up to the first Gauss-Newton iteration whose
    objective is at or below SpML's (its time prorated by iterations)."""
    import torch
    from paper_2001_06613_amd import learned
    from paper_2001_06613_amd.binding import STML

    n, ext = frames.shape[0], frames.shape[1:]
    fr = torch.from_numpy(frames).cuda()
    out, ys, final_j = {}, {}, None
    for name, nt, eps in (("spml", 1, 0.0), ("stml", 3, 0.0),
                          ("stml_eq3", 3, 1e-3)):
        # eq. (3) with a relative tolerance (the paper gives no epsilon;
        # 1e-3 of D is scale-free across the image and volume sequences)
        st = STML(n, ext, opts=learned.schedule_opts(
            predictor=0, dim=dim, n_temporal=nt, gn_max=40, eps_stop=eps,
            stop_relative=eps > 0))
        L = st.levels
        ts = []
        for _ in range(reps):
            st.set_sequence(fr)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        res = {"wall_ms": round(1e3 * float(np.median(ts)), 2),
               "stages": len(st.logs())}
        if name != "stml_eq3":
            # the same schedule, stage by stage (no eq. (3) stop)
            st.set_sequence(fr)
            stage_ms = []
            for lv in range(L):
                for q in range(nt):
                    t0 = time.perf_counter()
                    st.predict(lv, q)
                    st.register_level(lv, q)
                    stage_ms.append(1e3 * (time.perf_counter() - t0))
            logs = st.logs()
            res["levels"] = [
                {"level": lv, "extent": list(st.level_extent(lv)),
                 "ms": round(sum(stage_ms[lv * nt:(lv + 1) * nt]), 2),
                 "gn": sum(g["gn"] for g in logs if g["level"] == lv)}
                for lv in range(L)]
            last = logs[-1]
            if name == "spml":
                final_j = last["J"]
            else:
                traj = [last["J0"]] + list(last["J_iter"])
                k = next((i for i, J in enumerate(traj) if J <= final_j),
                         None)
                res["final_stage_gn"] = last["gn"]
                res["final_stage_gn_to_spml_J"] = k
                if k is not None:
                    res["est_ms_to_spml_J"] = round(
                        sum(stage_ms[:-1]) +
                        stage_ms[-1] * k / max(last["gn"], 1), 2)
        u = st.get_displacements(L - 1)
        allk = list(range(n))
        d0 = st.eval(L - 1, allk, torch.zeros_like(u), want_grad=False)["D"]
        d1 = st.eval(L - 1, allk, u, want_grad=False)["D"]
        res["D_over_D0_pct"] = round(100.0 * d1 / d0, 3)
        ys[name] = u.double()
        out[name] = res
        st.close()
        log(f"multilevel {dim}-D: {name} done")
    for name in ("stml", "stml_eq3"):
        out[name]["rel_diff_y_vs_spml_pct"] = round(
            100.0 * float((ys[name] - ys["spml"]).norm() /
                          ys["spml"].norm()), 3)
        out[name]["speedup_vs_spml"] = round(
            out["spml"]["wall_ms"] / out[name]["wall_ms"], 3)
    return out

def pmc_probe(st, fr):
    """One solve and a plain copy of known size, for counter runs."""
    import torch

    st.set_sequence(fr)
    st.run()
    x = torch.ones(COPY_BYTES // 4, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": True, "copy_bytes": COPY_BYTES}))


FP64_PEAK_TFS = 78.6           # MI355X float64 vector (and matrix) peak
AFFINE = dict(n=129, extent=(225, 80, 40), n_spatial=3, n_temporal=4,
              lam=1e-3, beta=1e-5, gn_max=20, max_disp=4.0, seed=60)


def _affine_frames():
    from paper_2001_06613_amd import synth

    a = AFFINE
    return synth.affine_sequence(a["n"], a["extent"], a["max_disp"],
                                 a["seed"], workers=16)[0]


def _affine_opts(n_temporal, eps=0.0):
    from paper_2001_06613_amd.binding import default_opts

    a = AFFINE
    return default_opts(dim=3, model="affine", n_spatial=a["n_spatial"],
                        n_temporal=n_temporal, lam=a["lam"], beta=a["beta"],
                        gn_max=a["gn_max"], eps_stop=eps,
                        stop_relative=eps > 0)


def affine_eval_rate(st, reps=20):
    """Objective passes (warp + Gram matrix + SqN) over all 129 frames of the
    finest level: time per pass, voxel-frames per second, and the Gram
    kernel's float64 rate (2 E N flops per pass, E = (|K|+1)(|K|+2)/2
    entries of the Gram matrix of the frames and a row of ones) against the
    float64 peak; the same with the gradient (two more passes)."""
    import torch

    a = AFFINE
    n = a["n"]
    lf = a["n_spatial"] - 1
    K = list(range(n))
    theta = st.get_params(lf)
    N = float(np.prod(a["extent"]))
    out = {}
    for grad in (False, True):
        st.eval_params(lf, K, theta, grad=grad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st.eval_params(lf, K, theta, grad=grad)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out["with_gradient" if grad else "objective"] = {
            "ms": round(1e3 * dt, 3),
            "Gvf_s": round(n * N / dt / 1e9, 2)}
    E = (n + 1) * (n + 2) / 2
    flops = 2.0 * E * N
    tf = flops / (out["objective"]["ms"] * 1e-3) / 1e12
    out["gram"] = {"flops_per_pass": flops, "TFLOPs": round(tf, 2),
                   "peak": FP64_PEAK_TFS, "frac_upper_bound": round(
                       tf / FP64_PEAK_TFS, 4),
                   "note": "objective pass time (warp, Gram, totals, "
                           "finalize, parameter copies) taken as the Gram "
                           "kernel's: a lower bound of its rate"}
    return out


def affine_comparison(frames, log):
    """The paper's experimental model (affine maps per frame, the SqN
    distance, L-BFGS) on the grid sizes of its Table 1 dataset D2: 129
    frames of 225x80x40 volumes, 3 spatial levels (57x20x10, 113x40x20,
    225x80x40), |K_0| = 17, |K_1| = 33 (4 temporal levels), synthetic affine
    motion of at most 4 px.  SpML (one temporal level) against STML (eq. (2)
    on finer levels) and STML with eq. (3) (relative 1e-3); L-BFGS with at
    most 20 iterations and the convergence test per registration.  Columns
    as in Table 1: run time, reduction of D from the unregistered frames
    (all frames, finest level), relative difference of the displacements
    (STML vs SpML)."""
    import torch
    from paper_2001_06613_amd.binding import STML

    a = AFFINE
    n, ext = a["n"], a["extent"]
    fr = torch.from_numpy(frames).cuda()
    lf = a["n_spatial"] - 1
    res, disp = {}, {}
    D0 = None
    for name, nt, eps in (("spml", 1, 0.0), ("stml", a["n_temporal"], 0.0),
                          ("stml_eq3", a["n_temporal"], 1e-3)):
        st = STML(n, ext, opts=_affine_opts(nt, eps))
        ts = []
        for _ in range(2):
            st.set_sequence(fr)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        logs = st.logs()
        theta = st.get_params(lf)
        if D0 is None:
            D0 = st.eval_params(lf, list(range(n)),
                                np.zeros_like(theta), grad=False)[0]["D"]
        D = st.eval_params(lf, list(range(n)), theta, grad=False)[0]["D"]
        disp[name] = st.get_displacements(lf).cpu().numpy()
        res[name] = {"wall_ms": round(1e3 * min(ts), 1),
                     "registrations": len(logs),
                     "lbfgs_iterations": sum(lg["gn"] for lg in logs),
                     "D_reduction_pct": round(100.0 * (D0 - D) / D0, 2)}
        if name == "stml":
            res["eval_rate"] = affine_eval_rate(st)
        st.close()
        log(f"affine: {name} done")
    ref = disp["spml"]
    for name in ("stml", "stml_eq3"):
        res[name]["rel_diff_y_vs_spml_pct"] = round(
            100.0 * float(np.linalg.norm(disp[name] - ref) /
                          np.linalg.norm(ref)), 2)
        res[name]["speedup_vs_spml"] = round(
            res["spml"]["wall_ms"] / res[name]["wall_ms"], 3)
    res["workload"] = ("129 frames x 225x80x40 (Table 1 D2 grid sizes), "
                       "affine motion <= 4 px, 3 spatial x 4 temporal "
                       "levels, SqN distance, lambda 1e-3, L-BFGS <= 20")
    res["paper"] = ("Table 1 D2 (affine, SqN, L-BFGS on private 4D-OCT "
                    "data, hardware not stated): SpML 7681 s, STML 3035 s "
                    "(2.5x)")
    return res


def affine_probe():
    """A few objective and gradient passes of the affine model at full size
    (129 x 225x80x40), for profiler runs."""
    import torch
    from paper_2001_06613_amd.binding import STML

    a = AFFINE
    frames = _affine_frames()
    st = STML(a["n"], a["extent"], opts=_affine_opts(1))
    st.set_sequence(torch.from_numpy(frames).cuda())
    lf = a["n_spatial"] - 1
    K = list(range(a["n"]))
    theta = np.zeros((a["n"], 12))
    for grad in (False, True, False, True):
        st.eval_params(lf, K, theta, grad=grad)
    torch.cuda.synchronize()
    print(json.dumps({"affine_probe": True}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-volume", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--no-multilevel", action="store_true",
                    help="skip the SpML vs STML comparison")
    ap.add_argument("--oracle-full", action="store_true",
                    help="time the oracle's whole schedule (CPU only)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="one solve and a copy of known size (counter runs)")
    ap.add_argument("--no-affine", action="store_true",
                    help="skip the paper's affine SqN / L-BFGS model block")
    ap.add_argument("--affine-probe", action="store_true",
                    help="a few affine evaluations at full size (profiler)")
    args = ap.parse_args()
    if args.affine_probe:
        affine_probe()
        return
    if args.oracle_full:
        oracle_full()
        return
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: this build "
              "runs the registration path on one GPU only", file=sys.stderr)
        sys.exit(2)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    # synthetic inputs of the extra comparisons, generated by forked
    # workers before the GPU is touched
    from paper_2001_06613_amd import learned, synth

    import multiprocessing as mp

    batch_seqs, learned_seqs, volume_seqs = None, None, None
    if not args.pmc_probe and not args.no_batch:
        with mp.get_context("fork").Pool(16) as pool:
            batch_seqs = pool.map(_gen_batch_sequence, synth.config_batch(),
                                  chunksize=1)
        log("batch: sequences generated")
    if not args.pmc_probe and not args.no_volume:
        jobs = [(VOLUME["n"], 3)] + synth.config_volume_batch()
        if not args.no_learned:
            jobs += [(VOLUME["n"], s) for s in LEARNED3D_SEEDS]
        with mp.get_context("fork").Pool(len(jobs)) as pool:
            volume_seqs = pool.map(_gen_volume_sequence, jobs, chunksize=1)
        log("volume: sequences generated")
    if not args.pmc_probe and not args.no_learned:
        learned_seqs = list(learned.generate(range(20000, 20004), workers=4))
    cpu_multi, cpu_batch = None, None
    if not args.pmc_probe and not args.no_cpu_baseline:
        # the host measurements run before the GPU is touched (forked
        # workers)
        frames_c2, _ = synth.config_large(1)
        cpu_multi = cpu_baseline_slabs(frames_c2)
        log("cpu: row slabs done")
        cpu_batch = oracle_batch_extrapolation()
        log("cpu: batch extrapolation done")
    affine_frames = None
    if not args.pmc_probe and not args.no_affine:
        affine_frames = _affine_frames()
        log("affine: sequence generated")

    import torch
    from paper_2001_06613_amd.binding import STML, default_opts

    torch.cuda.set_device(0)
    w = WORKLOAD
    frames, _ = synth.config_large(1)
    opts = default_opts(n_spatial=w["n_spatial"], n_temporal=w["n_temporal"],
                        reg=w["reg"], alpha=w["alpha"], lam=w["lam"],
                        beta=w["beta"], gn_max=w["gn_max"],
                        cg_max=w["cg_max"], parity_mode=w["parity_mode"])
    st = STML(w["n"], w["extent"], opts=opts)
    fr = torch.from_numpy(frames).cuda()
    extents = [st.level_extent(l) for l in range(w["n_spatial"])]

    def step():
        st.set_sequence(fr)
        st.run()

    if args.pmc_probe:
        pmc_probe(st, fr)
        return

    for i in range(args.warmup):
        step()
        print(f"warmup {i + 1}/{args.warmup} done", file=sys.stderr,
              flush=True)
    units_per_step = _units(st.logs(), extents)
    # the dominant kernel's dispatches carry their own timestamps; only
    # every TIME_EVERY-th launch (7 is prime to the 10 CG steps, so every
    # step index and level is sampled) so that the timed steps run within
    # a few per cent of untimed ones
    st.timing([DOMINANT], every=TIME_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        print(f"step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st.timing(0)
    dt = t1 - t0
    ms_per_step = dt / args.steps * 1e3
    value = units_per_step * args.steps / dt / 1e9

    dk = st.timing_get(DOMINANT)
    dim = len(w["extent"])
    bytes_total = dk["bytes"]
    avg_ms = dk["ms"] / max(dk["launches"], 1)
    achieved = bytes_total / (dk["ms"] * 1e-3) / 1e9 if dk["ms"] > 0 else 0.0
    fin = st.timing_get(DOMINANT, w["n_spatial"] - 1)
    fin_gbs = fin["bytes"] / (fin["ms"] * 1e-3) / 1e9 if fin["ms"] > 0 else 0.0
    traffic = _traffic_record()
    copy_gbs = copy_ceiling()
    # per-kernel breakdown from one extra, separately timed solve (every
    # class bracketed), outside the timed region
    st.timing(True)
    step()
    st.timing(False)
    # the metric's own kernels alone (evaluation and Hessian products, as
    # many as the schedule runs) at the finest level, and their roofline
    lf = w["n_spatial"] - 1
    ue, uh = st.timing_get("eval", lf), st.timing_get("hessvec", lf)
    unit_s = (ue["ms"] + uh["ms"]) * 1e-3
    unit_vf = ue["voxel_frames"] + uh["voxel_frames"]
    unit_gbs = (ue["bytes"] + uh["bytes"]) / unit_s / 1e9
    metric_unit = {
        "what": "evaluation (warp, distance, gradient) and Hessian-product "
                "kernels alone, finest level",
        "Gvf_s": round(unit_vf / unit_s / 1e9, 2),
        "GBs": round(unit_gbs, 1),
        "frac": round(unit_gbs / HBM_PEAK_GBS, 4),
        "bytes_per_vf": round((ue["bytes"] + uh["bytes"]) / unit_vf, 2),
        "roofline_Gvf_s": round(HBM_PEAK_GBS * 1e9 /
                                ((ue["bytes"] + uh["bytes"]) / unit_vf) /
                                1e9, 1)}
    kernels = {}
    for k in ("eval", "hessvec", "cg_update", "trial", "cg_init", "accept",
              "predict", "restrict"):
        # cg_init: the one-block kernel of the CG start scalars (r and z
        # are formed by the evaluation)
        t = st.timing_get(k)
        gbs = t["bytes"] / (t["ms"] * 1e-3) / 1e9 if t["ms"] > 0 else 0.0
        kernels[k] = {"ms": round(t["ms"], 4), "launches": t["launches"],
                      "GBs": round(gbs, 1)}

    out = {
        "metric": "warp+dist+grad+Hv Gvoxel-frames/s",
        "value": round(value, 3),
        "unit": "Gvoxel-frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage / f64 accumulate",
        "data": "synthetic",
        "config": {
            "workload": "STML solve, 64 frames x 256x256 OCT-like phantom, "
                        "4 spatial x 3 temporal levels (|K| 17/33/64), "
                        "curvature alpha 0.1, fixed 5 GN x 10 CG",
            "frames": w["n"], "extent": list(w["extent"]),
            "units_per_step": units_per_step,
        },
        "roofline": {
            "kernel": DOMINANT_NAME,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "avg_launch_ms": round(avg_ms, 5),
            "timed_launches": dk["launches"],
            "timed_every": TIME_EVERY,
            "algorithmic_bytes_per_launch": bytes_total / max(dk["launches"], 1),
            "finest_level_GBs": round(fin_gbs, 1),
            "measured_copy_GBs": round(copy_gbs, 1),
        },
        "kernels_one_solve": kernels,
        "metric_unit": metric_unit,
    }
    st.close()
    if not args.no_small:
        out["small"] = small_solve()
    if batch_seqs is not None:
        out["batched"] = batched_comparison(batch_seqs, log)
    if learned_seqs is not None:
        out["learned"] = learned_comparison(learned_seqs, log)
    if volume_seqs is not None:
        nb = len(synth.config_volume_batch())
        out["volume"] = volume_comparison(volume_seqs[0],
                                          volume_seqs[1:1 + nb], log)
        if not args.no_learned:
            out["learned_3d"] = learned3d_comparison(
                list(zip(LEARNED3D_SEEDS, volume_seqs[1 + nb:])), log)
    if not args.no_multilevel:
        out["multilevel"] = {"image": multilevel_comparison(frames, 2, log, 3)}
        if volume_seqs is not None:
            out["multilevel"]["volume"] = multilevel_comparison(
                volume_seqs[0], 3, log, 1)
    if affine_frames is not None:
        out["affine"] = affine_comparison(affine_frames, log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(frames)
        out["cpu_baseline_cores"] = cpu_multi
        out["cpu_batch_extrapolation"] = cpu_batch
        if batch_seqs is not None:
            cpu_batch["gpu_batched_s"] = out["batched"]["batched_ms"] / 1e3
            cpu_batch["ratio"] = round(cpu_batch[
                "batch_oracle_s_extrapolated"] / cpu_batch["gpu_batched_s"], 1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
