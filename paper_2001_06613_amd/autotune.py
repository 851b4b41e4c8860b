"""Autotuner of the 2-D launch shapes, with a JSON cache.

The tuned values are the block caps of stml_tuning: blocks per registration
of the objective and trial kernels, of the voxel-major CG updates, and the
block target of the Hessian product.  For a set of contexts (registered
alone or as a batch) one registration stage is timed for each candidate,
one parameter at a time (coordinate descent from the defaults), starting
every timing from the same displacements; the fastest setting is applied
to every context and stored under a key made of the device name and the
shapes, so a later run with the same shapes reads it back.  The values only
change the order of float64 sums, not what is computed.
"""

import json
import os
import time

CANDIDATES = {
    "tile_blocks": [128, 256, 512, 1024],
    "vox_blocks": [128, 256, 512, 1024],
    "hv_blocks": [1024, 2048, 4096, 8192],
}
DEFAULT = {"tile_blocks": 512, "vox_blocks": 512, "hv_blocks": 2048}


def cache_key(stmls, batched):
    """Device (architecture and compute-unit count: the marketing name is
    not always resolvable), batched or single, and the problem shapes."""
    import torch

    prop = torch.cuda.get_device_properties(stmls[0].device)
    arch = getattr(prop, "gcnArchName", "") or prop.name
    dev = f"{arch.split(':')[0]}x{prop.multi_processor_count}"
    shapes = ";".join(f"{s.n}x" + "x".join(map(str, s.extent)) for s in stmls)
    return f"{dev}|{'batch' if batched else 'single'}|{shapes}"


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _apply(stmls, cfg):
    for s in stmls:
        s.set_tuning(cfg["tile_blocks"], cfg["vox_blocks"], cfg["hv_blocks"])


def tune(stmls, batch=None, level=None, q=None, cache_path=None, repeats=2,
         log=None):
    """Tune the launch shape of `stmls` (their sequences must be set).

    batch: a Batch over stmls to time batched registrations (else each
    context registers in turn).  level, q: the stage to time (default: the
    finest level, the last temporal set).  Returns the applied setting.
    """
    import torch

    key = cache_key(stmls, batch is not None)
    cache = _load(cache_path)
    if key in cache:
        _apply(stmls, cache[key])
        return dict(cache[key])
    level = stmls[0].levels - 1 if level is None else level
    q = stmls[0].opts.n_temporal - 1 if q is None else q
    start = [s.get_displacements(level).clone() for s in stmls]

    def timed(cfg):
        _apply(stmls, cfg)
        best = float("inf")
        for _ in range(repeats):
            for s, u in zip(stmls, start):
                s.set_displacements(level, u)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if batch is not None:
                batch.register_level(level, q)
            else:
                for s in stmls:
                    s.register_level(level, q)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            gn = max(s.logs()[-1]["gn"] for s in stmls)
            best = min(best, dt / max(gn, 1))
        return best

    cfg = dict(DEFAULT)
    best_t = timed(cfg)
    for name, values in CANDIDATES.items():
        for v in values:
            if v == cfg[name]:
                continue
            trial = dict(cfg, **{name: v})
            t = timed(trial)
            if log:
                log(f"{name}={v}: {1e3 * t:.3f} ms per iteration "
                    f"(best {1e3 * best_t:.3f})")
            if t < best_t:
                best_t, cfg = t, trial
    for s, u in zip(stmls, start):
        s.set_displacements(level, u)
    _apply(stmls, cfg)
    if cache_path:
        cache = _load(cache_path)
        cache[key] = dict(cfg, ms_per_iteration=1e3 * best_t)
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return cfg
