#!/usr/bin/env python
"""Throughput of the all-agents neighbourhood query on one MI355X.

Headline workload (the configuration the metric is quoted on): N = 1,048,576
points uniform in a clipped 128^3 lattice (cell edge 2^16 fixed-point
units); every point queries its own radius, uniform in [0.5, 4] cells in
steps of 1/64 cell.  One step is the whole hot path on that input:

    lattice rebuild (cell histogram, exclusive scan, scatter)
    count pass (sphere-table walk, per-row sizes) + exclusive scan -> row_ptr
    write pass (walk again, compact hits, sort each row by (dist2, id))

with inputs resident in HBM, the sphere tables built once beforehand (the
paper precomputes them at start-up) and the output buffer sized once from
the first count.  The persistent launch uses the autotuned configuration;
the plain per-query-set launch and the bin-lattice cube scan are timed on
the same GPU and reported beside it.  The CPU oracle is timed on the host
cores on the same workload and its result checks the GPU output.

Further legs, reported under their own keys of the same JSON line:

    knn        4,194,304 clustered points in a cyclic 256^3 lattice, K = 16,
               cap 8 cells (sphere tables vs the cube scan on a subsample)
    timestep   8,388,608 moving agents in a cyclic 256^3 lattice, radius 3
               cells, 100 steps replayed from one captured HIP graph
    serving    16,777,216 points in a cyclic 512^3 lattice; Poisson batches
               of log-uniform size mixing radius and K-NN queries; p50/p99
               latency of continuous batching vs one plain launch per batch

Prints one JSON line.  `--copy-bytes B` instead times a plain device copy of
B bytes (the calibration run for the HBM byte counters).
"""
from __future__ import annotations

import argparse
import dataclasses
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "all-agents neighbor queries/sec and HBM GB/s at 1 GPU; p99 latency vs plain launch"
HBM_PEAK_GBS = 8000.0
LEGS = ("c2", "knn", "timestep", "serving", "sweep", "tables")
DEFAULT_LEGS = ("c2", "knn", "timestep", "serving")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sample_rows(rp, ids_dev, rows):
    """(row_ptr, ids) of the given rows, gathered from device ids."""
    import numpy as np
    import torch
    lens = rp[rows + 1] - rp[rows]
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows]) if len(rows) else np.zeros(0, np.int64)
    got = ids_dev[torch.from_numpy(idx).to(ids_dev.device)].cpu().numpy().view(np.uint32)
    srp = np.zeros(len(rows) + 1, dtype=np.int64)
    srp[1:] = np.cumsum(lens)
    return srp, got


def same_rows(srp, sids, ref):
    import numpy as np
    return bool(np.array_equal(srp, ref.row_ptr) and np.array_equal(sids, ref.ids))


def sample_of(n, count, seed):
    from paper_cs_0608108_amd import synth
    import numpy as np
    if n <= count:
        return np.arange(n, dtype=np.int64)
    return np.unique(synth.uniform_int(seed, 44, np.arange(count, dtype=np.uint64), 0, n - 1))


# ---------------------------------------------------------------------------
# Headline: batched uneven-radius all-agents query

def leg_c2(args, out):
    import numpy as np
    import torch

    from paper_cs_0608108_amd import autotune, sphidx, synth

    w = synth.radius_uneven_clipped()
    n = w.n
    log(f"workload {w.name}: n={n}")
    lat = sphidx.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, n)
    dev = [sphidx.to_dev_u32(a) for a in w.pts]
    rad = sphidx.to_dev_u32(w.r_fx)
    rmax = 4 * w.lat.edge
    tab = sphidx.Tables(lat, 2, rmax)
    q = sphidx.make_queries(n, None, rad, None, sphidx.MODE_RADIUS, 0)
    buf = sphidx.QueryBuffers(n, 0, want_dist2=False)
    lat.build(*dev)
    sphidx.count(lat, tab, q, buf)
    total = int(buf.row_ptr[-1].item())
    buf.grow(total)
    # workspace room for the count pass to keep every sorted row, so that
    # the write pass copies rows instead of walking the tables again
    buf.reserve_stash(total)
    log(f"pairs per step: {total}")

    def step(ln):
        lat.build(*dev)
        sphidx.count(lat, tab, q, buf, ln)
        sphidx.write(lat, tab, q, buf, ln)

    shape = dict(workload=w.name, n=n)
    if args.no_tune:
        cache = autotune.load_cache()
        ver = autotune.kernel_version()
        cfg = next((v["config"] for k, v in cache.items() if ver in k and f"workload={w.name}" in k
                    and "method=0" in k and "schedule=1" in k), {})
    else:
        cfg = autotune.tune(shape, lambda ln: (lambda: step(ln)), log=log)
    tuned = sphidx.LaunchConfig(method=sphidx.METHOD_SPHERE, schedule=sphidx.SCHED_PERSISTENT, **cfg)
    log(f"launch config: {cfg}")

    def timed(ln, steps, warmup):
        """Wall ms/step, mean phase ms (rebuild, count pass, write pass) and
        mean ms of the count and write kernels alone (events the library
        records around them on the launch stream)."""
        for _ in range(warmup):
            step(ln)
        torch.cuda.synchronize()
        E = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
        ev = [[E() for _ in range(4)] for _ in range(steps)]
        kev = [[E() for _ in range(4)] for _ in range(steps)]
        lc = [dataclasses.replace(ln, events=(k[0], k[1])) for k in kev]
        lw = [dataclasses.replace(ln, events=(k[2], k[3])) for k in kev]
        t0 = time.perf_counter()
        for s in range(steps):
            e = ev[s]
            e[0].record()
            lat.build(*dev)
            e[1].record()
            sphidx.count(lat, tab, q, buf, lc[s])
            e[2].record()
            sphidx.write(lat, tab, q, buf, lw[s])
            e[3].record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ph = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(3)] for e in ev])
        kk = np.array([[k[0].elapsed_time(k[1]), k[2].elapsed_time(k[3])] for k in kev])
        timed.per_step = ph.sum(axis=1)
        return (t1 - t0) * 1e3 / steps, ph.mean(axis=0), kk.mean(axis=0)

    ms, phases, kern = timed(tuned, args.steps, args.warmup)
    # the paper's protocol beside the contract's mean (Section IV.A: repeat,
    # drop the slowest quarter, average the rest), from the per-step events
    per = np.sort(timed.per_step)
    kept = per[: max(1, len(per) - len(per) // 4)]
    out["paper_protocol"] = {"steps": int(len(per)), "dropped_slowest": int(len(per) - len(kept)),
                             "mean_ms": round(float(kept.mean()), 4), "median_ms": round(float(np.median(per)), 4),
                             "queries_per_s": round(n / (float(kept.mean()) * 1e-3), 1)}
    code, flags = lat.status()
    assert code == sphidx.OK, (code, flags)
    rp = buf.row_ptr.cpu().numpy()
    ids = buf.ids[: int(rp[-1])].cpu().numpy().view(np.uint32)
    log(f"persistent: {ms:.3f} ms/step; build {phases[0]:.3f} count {phases[1]:.3f} write {phases[2]:.3f} ms; "
        f"count kernel {kern[0]:.3f} write kernel {kern[1]:.3f} ms")

    # cells and candidate objects per query, sphere tables against the
    # bin-lattice cube: the per-query statistics of one count pass each
    # (untimed; the rows found above are kept on the host)
    cells = {}
    for name, meth in (("sphere", sphidx.METHOD_SPHERE), ("cube", sphidx.METHOD_CUBE)):
        st = torch.zeros(4 * n, dtype=torch.int32, device="cuda")
        sphidx.count(lat, tab, q, buf, sphidx.LaunchConfig(method=meth, stats=st))
        a = st.cpu().numpy().view(np.uint32).reshape(n, 4).astype(np.float64)
        cells[name] = {"rows_walked": round(float(a[:, 0].mean()), 3), "cells_kept": round(float(a[:, 1].mean()), 3),
                       "candidates": round(float(a[:, 2].mean()), 3)}
        del st
    cells["cube_cells"] = cells["cube"]["cells_kept"]
    cells["hits"] = round(total / n, 3)
    cells["kept_over_cube"] = round(cells["sphere"]["cells_kept"] / cells["cube"]["cells_kept"], 4)
    cells["candidates_over_cube"] = round(cells["sphere"]["candidates"] / cells["cube"]["candidates"], 4)
    out["cells_per_query"] = cells
    log(f"per query: sphere {cells['sphere']}, cube {cells['cube']}, hits {cells['hits']}")

    if not args.no_baselines:
        k2 = max(3, args.steps // 2)
        two_walks = dataclasses.replace(tuned, no_stash=1)
        ms_tw, ph_tw, k_tw = timed(two_walks, k2, 1)
        out["without_stash"] = {"ms_per_step": round(ms_tw, 4), "count_kernel_ms": round(float(k_tw[0]), 4),
                                "write_kernels_ms": round(float(k_tw[1]), 4)}
        log(f"without stash: {ms_tw:.3f} ms/step (count {k_tw[0]:.3f}, write {k_tw[1]:.3f})")
        plain = sphidx.LaunchConfig(method=sphidx.METHOD_SPHERE, schedule=sphidx.SCHED_PLAIN)
        ms_plain, ph_plain, _ = timed(plain, k2, 1)
        cube = sphidx.LaunchConfig(method=sphidx.METHOD_CUBE, schedule=sphidx.SCHED_PERSISTENT, **cfg)
        ms_cube, ph_cube, _ = timed(cube, k2, 1)
        rp_c = buf.row_ptr.cpu().numpy()
        ids_c = buf.ids[: int(rp_c[-1])].cpu().numpy().view(np.uint32)
        same = bool(np.array_equal(rp_c, rp) and np.array_equal(ids_c, ids))
        out.update({
            "plain_launch": {"ms_per_step": round(ms_plain, 4), "queries_per_s": n / (ms_plain * 1e-3),
                             "query_ms": round(float(ph_plain[1] + ph_plain[2]), 4)},
            "cube_scan": {"ms_per_step": round(ms_cube, 4), "queries_per_s": n / (ms_cube * 1e-3),
                          "query_ms": round(float(ph_cube[1] + ph_cube[2]), 4), "same_result": same},
            "speedup_vs_plain": round(ms_plain / ms, 3),
            "speedup_vs_cube": round(ms_cube / ms, 3),
        })
        log(f"plain: {ms_plain:.3f} ms/step; cube: {ms_cube:.3f} ms/step; cube result identical: {same}")
        # the per-query choice (Section III.B/C) with the tuned launch, by
        # cells (the paper's volumes) and by estimated lane work; the
        # non-empty cell list is kept (and rebuilt) only here
        lat.attach_cell_list()
        # one discarded run first: the first timing after attaching has read
        # up to 2 ms more per rebuild on the GPU machine, once only
        timed(dataclasses.replace(tuned, method=sphidx.METHOD_AUTO), 3, 2)
        for model, tag in ((0, "auto_choice"), (1, "auto_work")):
            mo = torch.empty(n, dtype=torch.int32, device="cuda")
            auto = dataclasses.replace(tuned, method=sphidx.METHOD_AUTO, method_out=mo, select_model=model)
            ms_auto, ph_auto, k_auto = timed(auto, k2, 3)
            rp_a = buf.row_ptr.cpu().numpy()
            ids_a = buf.ids[: int(rp_a[-1])].cpu().numpy().view(np.uint32)
            used = torch.bincount(mo.long(), minlength=4).cpu().tolist()
            out[tag] = {"ms_per_step": round(ms_auto, 4), "query_ms": round(float(ph_auto[1] + ph_auto[2]), 4),
                        "rebuild_ms": round(float(ph_auto[0]), 4), "count_kernel_ms": round(float(k_auto[0]), 4),
                        "chose": {"sphere": used[sphidx.METHOD_SPHERE], "cube": used[sphidx.METHOD_CUBE],
                                  "list": used[sphidx.METHOD_LIST]},
                        "same_result": bool(np.array_equal(rp_a, rp) and np.array_equal(ids_a, ids))}
            log(f"{tag}: {ms_auto:.3f} ms/step (query {ph_auto[1] + ph_auto[2]:.3f} ms, count kernel "
                f"{k_auto[0]:.3f}), chose {out[tag]['chose']}")
        lat.attach_cell_list(False)

    # roofline of the dominant kernel, the count kernel (it walks the tables,
    # tests candidates, sorts each row and keeps it in the stash):
    # algorithmic bytes = point records 16 B/pt + cell_start 4 B/cell +
    # descriptors 64 B/query + row size 8 B/query + stash offset 4 B/query +
    # stashed ids 4 B/pair, over its own event-timed duration on the launch
    # stream.  The write pass only copies the rows: stash offset 4 B/query,
    # point record 16 B/query (the row's id), row_ptr 16 B/query (two entries
    # of a random row) and 4 B/pair in and out.
    ncells = lat.ncells
    count_bytes = 16 * n + 4 * (ncells + 2) + 64 * n + 8 * n + 4 * n + 4 * total
    gather_bytes = 4 * n + 16 * n + 16 * n + 4 * total + 4 * total
    achieved = count_bytes / (kern[0] * 1e-3) / 1e9
    traffic = _stored_traffic()
    # what bounds it instead: the share of the SIMDs' cycles spent issuing
    # VALU instructions (SQ counters, same source hash), or None
    valu = _stored_counters().get("count_kernel_valu_busy_frac")
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "valu_busy_frac": valu,
                "kernel": ("group_count_kernel" if cfg.get("grouped") else "count_kernel")
                + " (walk, test, sort, stash)",
                "algorithmic_bytes": count_bytes, "kernel_ms": round(float(kern[0]), 4),
                "write_pass": {"kernels": "gather_kernel + write_kernel (rows not stashed)",
                               "ms": round(float(kern[1]), 4), "algorithmic_bytes": gather_bytes,
                               "GBps": round(gather_bytes / (kern[1] * 1e-3) / 1e9, 2)}}

    cpu = None
    exact = None
    if not args.no_cpu:
        import oracle
        L = oracle.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask)
        reps, spent, ref = 0, 0.0, None
        while reps < 8 and spent < 10.0:
            t0 = time.perf_counter()
            g = oracle.Grid(L, w.pts)
            ref = g.radius(w.r_fx)
            spent += time.perf_counter() - t0
            g.close()
            reps += 1
        cpu = {"value": round(n * reps / spent, 1), "unit": "queries/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"full workload ({n} queries, grid build + radius + row sort) x{reps}, {spent:.1f} s"}
        exact = bool(np.array_equal(ref.row_ptr, rp) and np.array_equal(ref.ids, ids))
        log(f"cpu oracle: {cpu['value']:.0f} queries/s on {cpu['cores']} threads; GPU bit-exact: {exact}")

    out.update({
        "metric": METRIC,
        "value": round(n / (ms * 1e-3), 1),
        "unit": "queries/s",
        "ms_per_step": round(ms, 4),
        "config": {"workload": w.name, "points": n, "lattice": "128^3 clipped, cell edge 2^16 units",
                   "radius": "per point, uniform [0.5, 4] cells, 1/64-cell steps", "subcell_bits": 2,
                   "launch": dict(cfg, schedule="persistent")},
        "pairs_per_step": total,
        "pairs_per_s": round(total / (ms * 1e-3), 1),
        "phase_ms": {"rebuild": round(float(phases[0]), 4), "count": round(float(phases[1]), 4),
                     "write": round(float(phases[2]), 4)},
        "bit_exact_vs_oracle": exact,
        "roofline": roofline,
        "cpu_baseline": cpu,
    })
    del buf, lat, tab, dev, rad
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# K-NN under heavy load

def leg_knn(args, out):
    import numpy as np
    import torch

    from paper_cs_0608108_amd import autotune, sphidx, synth

    w = synth.knn_clustered()
    n, K = w.n, int(w.k[0])
    cap = int(w.r_fx[0])
    log(f"workload {w.name}: n={n} K={K} cap={cap}")
    lat = sphidx.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, n)
    dev = [sphidx.to_dev_u32(a) for a in w.pts]
    tab = sphidx.Tables(lat, 2, cap)
    lat.build(*dev)
    q = sphidx.make_queries(n, None, cap, K, sphidx.MODE_KNN, 0)
    # rows are at most K long: with stash room the count pass searches each
    # row once and keeps it, and the write pass only copies.  Rows searched
    # in groups as radius rows keep their whole radius row (about 1.7K pairs)
    buf = sphidx.QueryBuffers(n, n * K, want_dist2=False, stash_pairs=3 * n * K)

    def step_with(launch):
        def run():
            lat.build(*dev)
            sphidx.query(lat, tab, q, buf, launch)
        return run

    # the tuned launch for this workload (grouped: the K-NN rows are searched
    # as radius rows at a first radius, several queries per wavefront)
    shape = dict(workload=w.name, n=n, k=K)
    if args.no_tune:
        cache = autotune.load_cache()
        ver = autotune.kernel_version()
        cfg = next((v["config"] for k, v in cache.items() if ver in k and f"workload={w.name}" in k
                    and "method=0" in k and "schedule=1" in k), {})
    else:
        cfg = autotune.tune(shape, step_with, log=log)
    ln = sphidx.LaunchConfig(**cfg)
    log(f"knn launch config: {cfg}")
    step = step_with(ln)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    rp = buf.row_ptr.cpu().numpy()
    log(f"knn sphere: {ms:.3f} ms/step, pairs {int(rp[-1])}")

    # sphere vs cube on the same subsample of query centres (the cube scan
    # looks at every object of the 17^3-cell cap cube, so all N would take long)
    rows = sample_of(n, 65536, 3)
    cen = tuple(sphidx.to_dev_u32(np.asarray(a)[rows]) for a in w.pts)
    qs = sphidx.make_queries(len(rows), cen, cap, K, sphidx.MODE_KNN, 0)
    bs = sphidx.QueryBuffers(len(rows), len(rows) * K, want_dist2=False, stash_pairs=3 * len(rows) * K)
    sub = {}
    for name, meth in (("sphere", sphidx.METHOD_SPHERE), ("cube", sphidx.METHOD_CUBE)):
        lq = sphidx.LaunchConfig(method=meth, **cfg)
        sphidx.query(lat, tab, qs, bs, lq)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            sphidx.query(lat, tab, qs, bs, lq)
        torch.cuda.synchronize()
        sub[name] = (time.perf_counter() - t0) * 1e3 / 3
        sub[name + "_rows"] = bs.host()[:2]
    same_sub = bool(np.array_equal(sub["sphere_rows"][0], sub["cube_rows"][0])
                    and np.array_equal(sub["sphere_rows"][1], sub["cube_rows"][1]))
    srp, sids = sample_rows(rp, buf.ids, rows)
    exact = None
    if not args.no_cpu:
        import oracle
        L = oracle.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask)
        g = oracle.Grid(L, w.pts)
        ref = g.knn(K, cap, queries=tuple(np.asarray(a)[rows] for a in w.pts))
        g.close()
        exact = same_rows(srp, sids, ref)
    log(f"knn subsample {len(rows)}: sphere {sub['sphere']:.3f} ms, cube {sub['cube']:.3f} ms, "
        f"same {same_sub}, oracle rows bit-exact {exact}")
    out["knn"] = {"workload": w.name, "ms_per_step": round(ms, 4), "queries_per_s": round(n / (ms * 1e-3), 1),
                  "launch": dict(cfg, schedule="persistent"),
                  "step": "rebuild + K-NN query (top-K rows, sorted by (dist2, id))",
                  "subsample": {"queries": int(len(rows)), "sphere_ms": round(sub["sphere"], 4),
                                "cube_ms": round(sub["cube"], 4),
                                "speedup_vs_cube": round(sub["cube"] / sub["sphere"], 3),
                                "sphere_equals_cube": same_sub},
                  "sampled_rows_bit_exact_vs_oracle": exact}
    del buf, bs, lat, tab, dev, cen
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# Moving-agent timesteps (one captured HIP graph per step)

def leg_timestep(args, out):
    import numpy as np
    import torch

    from paper_cs_0608108_amd import autotune, sphidx, synth, timestep

    w = synth.agents_timestep()
    n, seed, r = w.n, w.extra["seed"], int(w.r_fx[0])
    log(f"workload {w.name}: n={n} r={r}")
    sim = timestep.AgentSim(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, w.pts, r, seed)
    # launch configuration for this workload: tuned on the query passes at the
    # starting positions (no movement), before the step is captured
    shape = dict(workload=w.name, n=n)

    def query_step(ln):
        def run():
            sim.lat.build(*sim.pos)
            sphidx.count(sim.lat, sim.tab, sim.q, sim.buf, ln)
            sphidx.write(sim.lat, sim.tab, sim.q, sim.buf, ln)
        return run

    if args.no_tune:
        cache = autotune.load_cache()
        ver = autotune.kernel_version()
        cfg = next((v["config"] for k, v in cache.items() if ver in k and f"workload={w.name}" in k), {})
    else:
        cfg = autotune.tune(shape, query_step, log=log)
    sim.launch = sphidx.LaunchConfig(method=sphidx.METHOD_SPHERE, schedule=sphidx.SCHED_PERSISTENT, **cfg)
    log(f"timestep launch config: {cfg}")
    sim.step()  # eager first step
    torch.cuda.synchronize()
    sim.capture()
    for _ in range(2):
        sim.replay()
    torch.cuda.synchronize()
    steps = args.timestep_steps
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    for _ in range(steps):
        sim.replay()
    b.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    ms = a.elapsed_time(b) / steps
    code, flags = sim.status()
    rp = sim.buf.row_ptr.cpu().numpy()
    pairs = int(rp[-1])
    total_steps = sim.steps_done
    log(f"timestep: {ms:.3f} ms/step (wall {wall:.3f}), pairs {pairs}, status {code}/{flags}")
    exact = None
    if not args.no_cpu:
        import oracle
        L = oracle.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask)
        cur = w.pts
        for t in range(total_steps):
            cur = oracle.move(L, seed, t, cur)
        got = sim.positions()
        pos_ok = all(np.array_equal(got[k], cur[k]) for k in range(3))
        rows = sample_of(n, 32768, 4)
        srp, sids = sample_rows(rp, sim.buf.ids, rows)
        g = oracle.Grid(L, cur)
        ref = g.radius(r, queries=tuple(np.asarray(c)[rows] for c in cur))
        g.close()
        exact = bool(pos_ok and same_rows(srp, sids, ref))
        log(f"timestep after {total_steps} steps: positions equal {pos_ok}, sampled rows bit-exact {exact}")
    out["timestep"] = {"workload": w.name, "steps": steps, "ms_per_step": round(ms, 4),
                       "wall_ms_per_step": round(wall, 4), "agent_queries_per_s": round(n / (ms * 1e-3), 1),
                       "pairs_per_step": pairs, "pairs_per_s": round(pairs / (ms * 1e-3), 1),
                       "step": "move + rebuild + count + scan + write + checksum, one graph replay",
                       "launch": dict(cfg, schedule="persistent"),
                       "status_ok": code == sphidx.OK and flags == 0,
                       "positions_and_sampled_rows_bit_exact_vs_oracle": exact}

    # incremental maintenance: the same steps with the lattice's own records
    # moved and the lattice rebuilt from them (move + rebuild in one update,
    # no by-id positions read or written); checked against the path above
    res = timestep.AgentSim(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, w.pts, r, seed,
                            launch=sim.launch, resident=True)
    res.step()
    torch.cuda.synchronize()
    res.capture()
    for _ in range(2):
        res.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        res.replay()
    b.record()
    torch.cuda.synchronize()
    ms_res = a.elapsed_time(b) / steps
    rcode, rflags = res.status()
    same = res.steps_done == sim.steps_done and all(
        np.array_equal(u, v) for u, v in zip(res.positions(), sim.positions()))
    same = bool(same and torch.equal(res.buf.row_ptr, sim.buf.row_ptr)
                and torch.equal(res.buf.ids[:pairs], sim.buf.ids[:pairs]))
    log(f"timestep, records moved in place: {ms_res:.3f} ms/step, identical to the rebuild path: {same}")
    out["timestep"]["resident"] = {"ms_per_step": round(ms_res, 4),
                                   "agent_queries_per_s": round(n / (ms_res * 1e-3), 1),
                                   "step": "move the lattice's records + rebuild from them + count + scan + "
                                           "write + checksum, one graph replay",
                                   "status_ok": rcode == sphidx.OK and rflags == 0,
                                   "positions_and_rows_equal_rebuild_path": same}
    del sim, res
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# Serving loop

def leg_serving(args, out):
    import numpy as np
    import torch

    from paper_cs_0608108_amd import serving, sphidx, synth

    w = synth.serving_lattice()
    spec = w.lat
    seed = w.extra["seed"]
    log(f"workload {w.name}: n={w.n}")
    lat = sphidx.Lattice(spec.log2_cells, spec.frac_bits, spec.cyclic_mask, w.n)
    dev = [sphidx.to_dev_u32(a) for a in w.pts]
    lat.build(*dev)
    tab = sphidx.Tables(lat, 2, 16 * spec.edge)
    nb = args.serving_batches
    sizes = synth.serving_batch_sizes(seed, nb, 65536)
    qs = [synth.serving_batch(spec, seed, i, int(s)) for i, s in enumerate(sizes)]
    pool = 4 << 30

    def make(arrivals):
        return [serving.Batch(i, float(arrivals[i]), q, r, k) for i, (q, r, k) in enumerate(qs)]

    fast = serving.GpuExecutor(lat, tab, args.serving_slots, int(sizes.max()), pool)
    plain = serving.GpuExecutor(lat, tab, 1, int(sizes.max()), pool,
                                launch=sphidx.LaunchConfig(schedule=sphidx.SCHED_PLAIN))
    # warm-up (first launches, table upload) on a few batches
    serving.run_admission_model(make(np.zeros(nb))[:4], fast, args.serving_slots, pool)
    serving.run_admission_model(make(np.zeros(nb))[:4], plain, 1, pool)
    torch.cuda.synchronize()
    # capacity: every batch queued at t = 0
    res = {}
    for name, ex, slots in (("continuous", fast, args.serving_slots), ("plain_per_batch", plain, 1)):
        bs = make(np.zeros(nb))
        serving.run_admission_model(bs, ex, slots, pool)
        res[name + "_saturated"] = serving.latency_stats(bs)
    # offered load: Poisson batches at fractions of the continuous path's
    # saturated batch rate, the same arrival sequence for both paths
    sat_rate = res["continuous_saturated"]["queries_per_s"] / float(sizes.mean())
    loads = {}
    for frac in (0.5, 0.8, 0.95):
        rate = frac * sat_rate
        arr = np.cumsum(synth.serving_interarrivals(seed, nb, rate))
        row = {"batches_per_s": round(rate, 2)}
        for name, ex, slots in (("continuous", fast, args.serving_slots), ("plain_per_batch", plain, 1)):
            bs = make(arr)
            adm = serving.run_admission_model(bs, ex, slots, pool)
            st = serving.latency_stats(bs)
            st["pool_peak_bytes"] = adm.pool.peak
            st["rejected"] = sum(b.rejected for b in bs)
            row[name] = st
        row["p99_speedup_vs_plain"] = round(row["plain_per_batch"]["p99_ms"] / row["continuous"]["p99_ms"], 3)
        loads[f"{frac:.2f}"] = row
    res["poisson"] = loads
    pairs = sum(b.pairs for b in bs)
    exact = None
    if not args.no_cpu:
        # the last run's rows of a few batches against the oracle
        import oracle
        L = oracle.Lattice(spec.log2_cells, spec.frac_bits, spec.cyclic_mask)
        g = oracle.Grid(L, w.pts)
        small = [i for i in np.argsort(sizes)[: max(3, nb // 10)]]
        chk = make(np.zeros(nb))
        chk = [chk[i] for i in small]
        serving.run_admission_model(chk, fast, args.serving_slots, pool, keep=True)
        exact = True
        for b in chk:
            ref = g.mixed(b.k, b.radius, queries=b.centres)
            rp, ids = b.result
            exact &= bool(np.array_equal(rp, ref.row_ptr) and np.array_equal(ids, ref.ids))
        g.close()
    for k, row in loads.items():
        log(f"serving load {k}: continuous p50 {row['continuous']['p50_ms']:.2f} p99 "
            f"{row['continuous']['p99_ms']:.2f} ms; plain p50 {row['plain_per_batch']['p50_ms']:.2f} p99 "
            f"{row['plain_per_batch']['p99_ms']:.2f} ms")
    log(f"serving capacity {res['continuous_saturated']['queries_per_s']:.0f} vs "
        f"{res['plain_per_batch_saturated']['queries_per_s']:.0f} q/s; oracle {exact}")
    out["serving"] = {"workload": w.name, "batches": nb, "slots": args.serving_slots,
                      "mean_batch": float(sizes.mean()), "median_batch": float(np.median(sizes)),
                      "load": "Poisson arrivals at 0.5 / 0.8 / 0.95 of the continuous path's saturated batch rate",
                      "pairs_last_run": int(pairs), **res,
                      "p99_speedup_vs_plain_at_0.8": loads["0.80"]["p99_speedup_vs_plain"],
                      "sampled_batches_bit_exact_vs_oracle": exact}
    del fast, plain, lat, tab, dev
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# Section IV sweep: sphere tables against the bin-lattice cube scan

def leg_sweep(args, out):
    """All neighbours and the nearest neighbour for random centres, by world
    (16^3, 32^3), boundary (wrapping, clipped), load and query distance (cell
    units, up to 3/4 of the world), the shapes of the paper's Figs. 5-10.
    Each point times the same queries with both methods (count + write, the
    write touching every neighbour's id; 5 runs, the 2 slowest dropped) and
    checks that their rows agree.
    All-neighbour points also time the per-query choice by volume (sphere,
    cube or non-empty cell list, Section III.B/C) and count what it chose."""
    import numpy as np
    import torch

    from paper_cs_0608108_amd import sphidx, synth

    radii = (0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 7.5, 8.0, 10.0, 12.0)
    rows = []
    mismatches = 0

    def timed_query(lat, tab, q, ln, reps=5, drop=2):
        """Mean ms of count + write over `reps` runs, the `drop` slowest left
        out (the paper's protocol, Section IV.A, in small)."""
        buf = sphidx.QueryBuffers(q.count, 0, want_dist2=False)
        sphidx.count(lat, tab, q, buf, ln)
        total = int(buf.row_ptr[-1].item())
        buf.grow(max(total, 1))
        buf.reserve_stash(max(total, 1))

        def run():
            sphidx.count(lat, tab, q, buf, ln)
            sphidx.write(lat, tab, q, buf, ln)
        run()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            run()
            b.record()
        torch.cuda.synchronize()
        t = sorted(a.elapsed_time(b) for a, b in ev)[: reps - drop]
        return sum(t) / len(t), buf

    for log2 in (4, 5):
        for mask in (7, 0):
            for load in (0.625, 1.0, 5.0, 10.0, 20.0):
                w = synth.sweep_world(log2, mask, load)
                L = 1 << log2
                lat = sphidx.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, max(w.n, 1))
                lat.attach_cell_list()
                dev = [sphidx.to_dev_u32(a) for a in w.pts]
                lat.build(*dev)
                n_list = lat.cell_list_host()[0]
                tab = sphidx.Tables(lat, 2, int(0.75 * L * w.lat.edge))
                for rc in radii:
                    if rc > 0.75 * L:
                        continue
                    r = int(rc * w.lat.edge)
                    # enough queries to fill the GPU, few enough to bound the output
                    vol = min(4.19 * rc ** 3, float(L ** 3))
                    Q = int(min(16384, max(512, 3e7 / max(load * vol, 1.0))))
                    cen = [sphidx.to_dev_u32(a) for a in synth.sweep_centres(w.lat, 6, Q)]
                    point = {"world": f"{L}^3", "wrap": mask == 7, "load": load, "r": rc, "queries": Q,
                             "nonempty_cells": n_list}
                    for mode, k, key in ((sphidx.MODE_RADIUS, 0, "all"), (sphidx.MODE_KNN, 1, "nearest")):
                        q = sphidx.make_queries(Q, tuple(cen), r, k, mode, 0)
                        t_s, b_s = timed_query(lat, tab, q, sphidx.LaunchConfig())
                        t_c, b_c = timed_query(lat, tab, q, sphidx.LaunchConfig(method=sphidx.METHOD_CUBE))
                        n_s = int(b_s.row_ptr[-1].item())
                        same = bool(torch.equal(b_s.row_ptr, b_c.row_ptr) and torch.equal(b_s.ids[:n_s], b_c.ids[:n_s]))
                        mismatches += 0 if same else 1
                        point[key] = {"sphere_ms": round(t_s, 4), "cube_ms": round(t_c, 4),
                                      "ratio": round(t_c / t_s, 3), "pairs": n_s, "same": same}
                        if mode == sphidx.MODE_RADIUS:
                            # the choice by cells (model 0, the paper's) and by
                            # estimated lane work (model 1)
                            for model, tag in ((0, "auto"), (1, "work")):
                                mo = torch.empty(Q, dtype=torch.int32, device="cuda")
                                ln_a = sphidx.LaunchConfig(method=sphidx.METHOD_AUTO, method_out=mo,
                                                           select_model=model)
                                t_a, b_a = timed_query(lat, tab, q, ln_a)
                                same_a = bool(torch.equal(b_s.row_ptr, b_a.row_ptr) and
                                              torch.equal(b_s.ids[:n_s], b_a.ids[:n_s]))
                                mismatches += 0 if same_a else 1
                                used = torch.bincount(mo.long(), minlength=4).cpu().tolist()
                                point[key].update({f"{tag}_ms": round(t_a, 4), f"ratio_{tag}": round(t_c / t_a, 3),
                                                   f"{tag}_chose": {"sphere": used[sphidx.METHOD_SPHERE],
                                                                    "cube": used[sphidx.METHOD_CUBE],
                                                                    "list": used[sphidx.METHOD_LIST]},
                                                   f"same_{tag}": same_a})
                                del b_a
                        del b_s, b_c
                    rows.append(point)
                    log(f"sweep {point['world']} wrap={point['wrap']} load={load} r={rc}: all x{point['all']['ratio']}"
                        f" auto x{point['all']['ratio_auto']} {point['all']['auto_chose']}"
                        f" work x{point['all']['ratio_work']} {point['all']['work_chose']}"
                        f" nearest x{point['nearest']['ratio']}")
                del lat, tab, dev
                torch.cuda.empty_cache()
    out["section_iv_sweep"] = {
        "ratio": "cube ms / sphere ms (above 1: the sphere tables are faster); ratio_auto, ratio_work: "
                 "cube ms / ms of the per-query choice by cells (the paper's volumes) and by estimated work",
        "step": "count + write on random centres; rows compared between the methods",
        "all_points_identical": mismatches == 0, "points": rows}


# ---------------------------------------------------------------------------
# Table designs compared (host only, no GPU)

def leg_tables(args, out):
    """Cells walked per query under each table design (Section II.A, III.A)
    for random positions in the home cell, by radius, and the ball/cube ratio
    of the sub-cell tables in 2, 3 and 4 dimensions (Sections I and V)."""
    import numpy as np

    from paper_cs_0608108_amd import sphidx

    F = 16
    e = 1 << F
    tab = sphidx.Tables(sphidx.desc_of((8, 8, 8), F, 7), 2, 16 * e)
    rng = np.random.default_rng(31)
    rows = []
    for rc in (0.5, 1.0, 2.0, 4.0, 8.0, 16.0):
        n = 4000
        f = [rng.integers(0, e, n).astype(np.uint32) for _ in range(3)]
        r = np.full(n, int(rc * e), dtype=np.uint32)
        c = sphidx.table_census(tab, f, r)
        row = {"r_cells": rc, "queries": n}
        row.update({k: round(float(v.mean()), 1) for k, v in c.items()})
        rows.append(row)
        log(f"tables r={rc}: " + " ".join(f"{k} {row[k]}" for k in sphidx.CENSUS_FIELDS))
    nd = []
    for dims in (2, 3, 4):
        for rc in (4, 8, 16):
            sph, cube, _ = sphidx.table_census_nd(dims, 8, 1, rc << 8)
            nd.append({"dims": dims, "r_cells": rc, "sphere_cells": round(sph, 1), "cube_cells": round(cube, 1),
                       "ratio": round(sph / cube, 4)})
    out["table_census"] = {
        "designs": "cells walked per query: bin-lattice cube, unshaved table, the paper's 64 specialised tables, "
                   "those after the Eq. 1 run-time test, this library's sub-cell class tables (s = 2), exact; "
                   "dropped = exact cells a design leaves out (must be 0)",
        "by_radius": rows, "ball_to_cube": nd}


def copy_calibration(nbytes):
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 5
    print(json.dumps({"copy_bytes": nbytes, "ms": ms, "GBps_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--legs", default=",".join(DEFAULT_LEGS), help="comma list of " + ",".join(LEGS))
    ap.add_argument("--no-tune", action="store_true", help="use the cached/default launch configuration")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs (profiling runs)")
    ap.add_argument("--no-baselines", action="store_true", help="skip the plain-launch and cube-scan legs")
    ap.add_argument("--timestep-steps", type=int, default=100)
    ap.add_argument("--serving-batches", type=int, default=200)
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--copy-bytes", type=int, default=0, help="only time a plain device copy of this size")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    legs = [x for x in args.legs.split(",") if x]
    if legs != ["tables"] or args.copy_bytes:
        torch.cuda.set_device(0)
    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
        return
    for x in legs:
        if x not in LEGS:
            sys.exit(f"unknown leg {x}")
    out = {"metric": METRIC, "value": None, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic"}
    # no cyclic garbage collection inside the timed regions: a collection
    # pass while the GPU waits for the next launch lands in the events of
    # that phase (one 35 ms pause showed up as 1.7 ms on a 20-step mean);
    # garbage is collected between the legs instead
    gc.disable()
    for x in legs:
        log(f"== leg {x}")
        {"c2": leg_c2, "knn": leg_knn, "timestep": leg_timestep, "serving": leg_serving,
         "sweep": leg_sweep, "tables": leg_tables}[x](args, out)
        gc.collect()
    print(json.dumps(out))


def _stored_counters():
    """Counter figures of the count kernel from committed rocprofv3 runs
    (profiles/traffic.json), used only while the kernel source still has the
    hash recorded with them; {} otherwise."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return {}
    with open(p) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_cs_0608108_amd", "csrc", "query.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return rec if rec.get("query_hip_sha256_16") == h else {}


def _stored_traffic():
    """HBM bytes per launch of the count kernel (FETCH_SIZE + WRITE_SIZE)."""
    return _stored_counters().get("count_kernel_bytes")


if __name__ == "__main__":
    main()
