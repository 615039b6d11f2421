"""Launch-configuration search for the query kernels.

For one workload shape it times a small grid of launch configurations
(waves per block, queries per work-queue grab, resident blocks per CU, LDS
row buffer, row table staged in LDS whole, in per-class chunks or not at
all, the interior shortcut, queries grouped per wavefront) on the device
with HIP events and keeps the fastest; then, with that launch, the waves
that take one long radius row together, and the sub-cell bits of the
tables when the caller can build them.  Results
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
    """Hash of the library's sources (every file under csrc/ and the public
    header): a tuning result is reused only for the code it was measured on,
    launch resolution and workspace planning included."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    csrc = os.path.join(here, "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc))
    files.append(os.path.join(os.path.dirname(here), "include", "sphidx.h"))
    h = hashlib.sha256()
    for f in files:
        if os.path.isfile(f):
            h.update(os.path.basename(f).encode())
            h.update(open(f, "rb").read())
    return h.hexdigest()[:12]


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


def cached(shape: dict, method=sphidx.METHOD_SPHERE, schedule=sphidx.SCHED_PERSISTENT) -> dict:
    """The cached configuration for this code, device and shape, or {} (the
    library's defaults) when none was tuned."""
    ent = load_cache().get(_key(_arch(), dict(shape, method=method, schedule=schedule)))
    return dict(ent["config"]) if ent else {}


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
        for w, t, b, c, l, i, g in itertools.product((2, 4), (16, 64, 256), (4, 6, 8), (128, 256), (0, 1, 2), (1, 2),
                                                     (0, 1)):
            yield dict(waves_per_block=w, tile=t, blocks_per_cu=b, sort_cap=c, table_in_lds=l, interior=i,
                       grouped=g)
    else:
        for w, t, l, i in itertools.product((2, 4), (1, 4, 16), (0, 1, 2), (1, 2)):
            yield dict(waves_per_block=w, tile=t, sort_cap=256, table_in_lds=l, interior=i)


def tune(shape: dict, make_runner, method=sphidx.METHOD_SPHERE, schedule=sphidx.SCHED_PERSISTENT,
         use_cache=True, save=True, log=None, subcell_runner=None, subcell_bits=(0, 1, 2, 3)):
    """make_runner(LaunchConfig) -> callable that runs one query pass set.
    Returns the best LaunchConfig fields as a dict.  With subcell_runner
    ((LaunchConfig, s) -> callable running the same passes with tables of s
    sub-cell bits per axis), the launch is searched first and the sub-cell
    bits then, with that launch; the result then holds "subcell_bits" too
    (not a LaunchConfig field: the caller builds its tables with it)."""
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
    if best is None:
        # every candidate was refused (for instance LDS too small for all of
        # them): the library's defaults, not cached
        if log:
            log(f"tune {shape}: no candidate ran; using the default launch")
        return {}
    # waves per long radius row (one block per row in the write pass; 1:
    # one wave per row, windowed), with the launch found above
    best_lw = None
    for lw in (1, 2, 4, 8):
        cfg = dict(best[1], long_row_waves=lw)
        try:
            ms = time_config(make_runner(sphidx.LaunchConfig(method=method, schedule=schedule, **cfg)))
        except sphidx.SphidxError as err:
            if log:
                log(f"tune long_row_waves={lw} -> skipped ({err})")
            continue
        if log:
            log(f"tune long_row_waves={lw} -> {ms:.3f} ms")
        if best_lw is None or ms < best_lw[0]:
            best_lw = (ms, cfg)
    if best_lw is not None:
        best = best_lw
    if subcell_runner is not None:
        ln = sphidx.LaunchConfig(method=method, schedule=schedule, **best[1])
        best_s = None
        for sb in subcell_bits:
            try:
                ms = time_config(subcell_runner(ln, sb))
            except sphidx.SphidxError as err:
                if log:
                    log(f"tune subcell_bits={sb} -> skipped ({err})")
                continue
            if log:
                log(f"tune subcell_bits={sb} -> {ms:.3f} ms")
            if best_s is None or ms < best_s[0]:
                best_s = (ms, sb)
        if best_s is not None:
            best = (best_s[0], dict(best[1], subcell_bits=best_s[1]))
    if save:
        cache = load_cache()
        cache[key] = {"config": best[1], "ms": best[0]}
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    return best[1]
