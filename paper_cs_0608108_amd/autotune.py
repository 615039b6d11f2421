"""Launch-configuration search for the query kernels.

For one workload shape it times a small grid of launch configurations
(waves per block, queries per work-queue grab, resident blocks per CU, LDS
row buffer) on the device with HIP events and keeps the fastest.  Results
are cached as JSON keyed by the device architecture and the workload shape,
so a later process reuses them without searching again.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

from . import sphidx

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def kernel_version() -> str:
    """Hash of the query kernels' source: a tuning result is reused only for
    the kernels it was measured on."""
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "query.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:12]


def _key(arch, shape: dict) -> str:
    return arch + "|" + kernel_version() + "|" + ",".join(f"{k}={shape[k]}" for k in sorted(shape))


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def load_cache():
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def time_config(run_once, reps=3):
    """Median time (ms) of run_once() over reps, after one warm-up."""
    run_once()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        run_once()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def candidates(schedule):
    if schedule == sphidx.SCHED_PERSISTENT:
        for w, t, b, c, l, i, g in itertools.product((2, 4), (16, 64, 256), (4, 6, 8), (128, 256), (0, 1), (1, 2),
                                                     (0, 1)):
            yield dict(waves_per_block=w, tile=t, blocks_per_cu=b, sort_cap=c, table_in_lds=l, interior=i,
                       grouped=g)
    else:
        for w, t, l, i in itertools.product((2, 4), (1, 4, 16), (0, 1), (1, 2)):
            yield dict(waves_per_block=w, tile=t, sort_cap=256, table_in_lds=l, interior=i)


def tune(shape: dict, make_runner, method=sphidx.METHOD_SPHERE, schedule=sphidx.SCHED_PERSISTENT,
         use_cache=True, save=True, log=None):
    """make_runner(LaunchConfig) -> callable that runs one query pass set.
    Returns the best LaunchConfig fields as a dict."""
    arch = _arch()
    key = _key(arch, dict(shape, method=method, schedule=schedule))
    cache = load_cache()
    if use_cache and key in cache:
        return cache[key]["config"]
    best = None
    for cfg in candidates(schedule):
        ln = sphidx.LaunchConfig(method=method, schedule=schedule, **cfg)
        try:
            ms = time_config(make_runner(ln))
        except sphidx.SphidxError as err:  # e.g. the row table does not fit in LDS
            if log:
                log(f"tune {cfg} -> skipped ({err})")
            continue
        if log:
            log(f"tune {cfg} -> {ms:.3f} ms")
        if best is None or ms < best[0]:
            best = (ms, cfg)
    if save:
        cache = load_cache()
        cache[key] = {"config": best[1], "ms": best[0]}
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    return best[1]
