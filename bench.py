#!/usr/bin/env python
"""Throughput of the all-agents neighbourhood query on one MI355X.

Headline workload: the largest all-agents configuration, N = 8,388,608
moving agents uniform at the start in a cyclic 256^3 lattice (cell edge
2^16 fixed-point units), radius 3 cells.  One step is the whole hot path on
that input, captured once as a HIP graph and replayed:

    move every agent (counter-hash displacement in [-1/4, 1/4] cell per axis,
        applied to the lattice's own records, keyed by agent id)
    lattice rebuild from those records (cell histogram, exclusive scan,
        scatter)
    count pass (sphere-table walk, rows sorted and kept) + scan -> row_ptr
    write pass (kept rows copied into place) + neighbour-count checksum

with inputs resident in HBM and the sphere tables built once beforehand
(the paper precomputes them at start-up).  `--steps K` graph replays are
timed between device synchronisations after `--warmup W`; the run then
continues to the workload's 100 steps and checks positions, the
neighbour-count checksum over all rows and sampled rows against the CPU
oracle's replay.  The bin-lattice cube scan, the plain launch, the step
that moves by-id coordinate arrays and rebuilds from them, and the
incremental lattice update run the same steps beside it.

Further workloads, each under its own key of the same JSON line with its
own roofline and oracle baseline:

    c1       4,096 points uniform in a cyclic 32^3 lattice, r = 2.5 cells,
             full CSR against brute force
    c2       1,048,576 points uniform in a clipped 128^3 lattice, per-point
             radius in [0.5, 4] cells; persistent launch vs plain launch vs
             cube scan
    knn      4,194,304 clustered points in a cyclic 256^3 lattice, K = 16,
             cap 8 cells (sphere tables vs the cube scan on a subsample)
    serving  16,777,216 points in a cyclic 512^3 lattice; Poisson batches of
             log-uniform size mixing radius and K-NN queries; p50/p99
             latency of continuous batching vs one plain launch per batch

Roofline: the algorithmic bytes of a query are each input array read once
and each output written once, 16 B per point record + 4 B per cell_start
entry + 8 B per row_ptr entry + 4 B per output id; the library's own
intermediates (query descriptors, stash offsets, stashed rows) are reported
beside them as overhead, not counted.  Prints one JSON line.
`--copy-bytes B` instead times a plain device copy of B bytes (the
calibration run for the HBM byte counters).
"""
from __future__ import annotations

import argparse
import dataclasses
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "all-agents neighbor queries/sec and HBM GB/s at 1 GPU; p99 latency vs plain launch"
HBM_PEAK_GBS = 8000.0
LEGS = ("timestep", "c1", "c2", "knn", "serving", "sweep", "tables")
DEFAULT_LEGS = ("timestep", "c1", "c2", "knn", "serving")


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
# Algorithmic bytes (what the method must move once) and the roofline

def query_bytes(n, ncells, Q, pairs, dist2=False):
    """All-agents query: every point record (16 B), every cell_start entry
    (4 B, the region cells and the outside cell's two bounds), every row_ptr
    entry (8 B) and every output id (4 B, +8 B with dist^2) once."""
    return 16 * n + 4 * (ncells + 2) + 8 * (Q + 1) + (12 if dist2 else 4) * pairs


def resident_update_bytes(n, ncells):
    """The lattice kept from its own records: the move reads and writes every
    record (16 + 16 B); the rebuild reads them in the histogram and the
    scatter (16 + 16 B) and writes them (16 B); the counts are zeroed,
    incremented, scanned (read + write) and read as cursors (4 + 4 + 8 + 4 B
    per cell)."""
    return {"move": 32 * n, "rebuild": n * (16 + 16 + 16) + ncells * (4 + 4 + 8 + 4)}


def overhead_bytes(Q, pairs):
    """The library's own intermediates: 64-byte query descriptors written by
    the setup kernel and read by the count kernel, stash offsets written and
    read (4 + 4 B), stashed rows written and read back (4 + 4 B per id)."""
    return {"descriptors": 128 * Q, "stash_offsets": 8 * Q, "stash_rows": 8 * pairs}


def stored_counters(workload):
    """HBM bytes and SQ figures of a workload's dominant kernel from committed
    rocprofv3 runs (profiles/traffic.json), used only while the library's
    sources still hash to what was profiled; {} otherwise."""
    from paper_cs_0608108_amd import autotune
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return {}
    with open(p) as f:
        rec = json.load(f)
    if rec.get("source_hash") != autotune.kernel_version():
        return {}
    return rec.get("kernels", {}).get(workload, {})


def roofline(workload, kernel, alg_bytes, kernel_ms, copy_gbps, extra=None):
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    rec = stored_counters(workload)
    d = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": rec.get("bytes"),
         "kernel": kernel, "kernel_ms": round(kernel_ms, 4), "algorithmic_bytes": int(alg_bytes),
         "copy_GBps": round(copy_gbps, 1) if copy_gbps else None,
         "frac_of_copy": round(achieved / copy_gbps, 5) if copy_gbps else None}
    if rec.get("valu_busy_frac") is not None:
        d["valu_busy_frac"] = rec["valu_busy_frac"]
    if extra:
        d.update(extra)
    return d


def copy_bandwidth(nbytes=1 << 30):
    """Achievable device-copy bandwidth (read + write GB/s) of a plain
    device-to-device copy, timed with HIP events."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(10):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 10
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def tuned_config(args, shape, make_runner, method=None, schedule=None, subcell_runner=None):
    """(launch fields, sub-cell bits of the tables): tuned on the device, or
    from the cache with --no-tune (2 sub-cell bits when none was tuned)."""
    from paper_cs_0608108_amd import autotune, sphidx
    method = sphidx.METHOD_SPHERE if method is None else method
    schedule = sphidx.SCHED_PERSISTENT if schedule is None else schedule
    if args.no_tune:
        cfg = autotune.cached(shape, method, schedule)
    else:
        cfg = autotune.tune(shape, make_runner, method=method, schedule=schedule, log=log,
                            subcell_runner=subcell_runner)
    cfg = dict(cfg)
    return cfg, int(cfg.pop("subcell_bits", 2))


def event_pairs(k):
    import torch
    return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]


def mean_ms(pairs):
    import numpy as np
    return float(np.mean([a.elapsed_time(b) for a, b in pairs]))


# ---------------------------------------------------------------------------
# Headline: moving-agent timesteps (one captured HIP graph per step)

def leg_timestep(args, out):
    import numpy as np
    import torch

    from paper_cs_0608108_amd import sphidx, synth, timestep

    w = synth.agents_timestep()
    spec = w.lat
    n, seed, r = w.n, w.extra["seed"], int(w.r_fx[0])
    ncells = 1 << sum(spec.log2_cells)
    K = args.steps
    log(f"workload {w.name}: n={n} r={r}")
    # the lattice is kept from its own records (moved in place, rebuilt from
    # them); the step that moves by-id coordinate arrays and rebuilds from
    # them is timed beside it
    sim = timestep.AgentSim(spec.log2_cells, spec.frac_bits, spec.cyclic_mask, w.pts, r, seed, resident=True)
    shape = dict(workload=w.name, n=n)

    def query_step(ln):
        def run():
            sim.lat.build(*sim.pos)
            sphidx.count(sim.lat, sim.tab, sim.q, sim.buf, ln)
            sphidx.write(sim.lat, sim.tab, sim.q, sim.buf, ln)
        return run

    tabs = {2: sim.tab}

    def subcell_step(ln, sb):
        if sb not in tabs:
            tabs[sb] = sphidx.Tables(sim.lat, sb, r)

        def run():
            sim.lat.build(*sim.pos)
            sphidx.count(sim.lat, tabs[sb], sim.q, sim.buf, ln)
            sphidx.write(sim.lat, tabs[sb], sim.q, sim.buf, ln)
        return run

    cfg, sbits = tuned_config(args, shape, query_step, subcell_runner=subcell_step)
    sim.tab = tabs[sbits] if sbits in tabs else sphidx.Tables(sim.lat, sbits, r)
    tabs.clear()
    sim.launch = sphidx.LaunchConfig(method=sphidx.METHOD_SPHERE, schedule=sphidx.SCHED_PERSISTENT, **cfg)
    log(f"timestep launch config: {cfg}, sub-cell bits {sbits}")
    # the dominant kernel's duration: eager steps (the same kernels and
    # arguments the graph replays) with HIP events the library records
    # around the count kernel on the launch stream
    kev = event_pairs(max(3, min(K, 20)))
    for e in kev:
        sim.step(count_events=e)
    torch.cuda.synchronize()
    kern_ms = mean_ms(kev)
    sim.capture()
    for _ in range(args.warmup):
        sim.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    for _ in range(K):
        sim.replay()
    b.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / K
    ms = a.elapsed_time(b) / K
    # the rest of the workload's 100 steps; at step 50 the row sizes of
    # sampled agents are kept (device copies in stream order, no sync)
    rows = sample_of(n, 65536, 4)
    rows_d = torch.from_numpy(rows).cuda()
    mid = {}
    while sim.steps_done < 100:
        sim.replay()
        if sim.steps_done == 50:
            rp_d = sim.buf.row_ptr
            mid[50] = (rp_d[rows_d + 1] - rp_d[rows_d]).clone()
    torch.cuda.synchronize()
    final = sim.steps_done
    code, flags = sim.status()
    rp = sim.buf.row_ptr.cpu().numpy()
    pairs = int(rp[-1])
    log(f"timestep: {ms:.3f} ms/step (wall {wall:.3f}), count kernel {kern_ms:.3f} ms, pairs {pairs}, "
        f"status {code}/{flags}")

    # the same steps with the bin-lattice cube scan, the plain launch, the
    # by-id rebuild and the incremental lattice update; each runs to the same
    # final step and is compared with the path above
    def other(tag, launch, resident=True, incremental=False):
        o = timestep.AgentSim(spec.log2_cells, spec.frac_bits, spec.cyclic_mask, w.pts, r, seed, launch=launch,
                              resident=resident, incremental=incremental, subcell_bits=sbits)
        o.step()
        torch.cuda.synchronize()
        o.capture()
        for _ in range(2):
            o.replay()
        torch.cuda.synchronize()
        reps = max(3, min(K, 20))
        ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ea.record()
        for _ in range(reps):
            o.replay()
        eb.record()
        torch.cuda.synchronize()
        oms = ea.elapsed_time(eb) / reps
        while o.steps_done < final:
            o.replay()
        torch.cuda.synchronize()
        ocode, oflags = o.status()
        same = o.steps_done == final and all(np.array_equal(u, v) for u, v in zip(o.positions(), sim.positions()))
        same = bool(same and ocode == sphidx.OK and torch.equal(o.buf.row_ptr, sim.buf.row_ptr)
                    and torch.equal(o.buf.ids[:pairs], sim.buf.ids[:pairs]) and o.checksum() == sim.checksum())
        log(f"timestep {tag}: {oms:.3f} ms/step, identical after {final} steps: {same}")
        del o
        torch.cuda.empty_cache()
        return {"ms_per_step": round(oms, 4), "agent_queries_per_s": round(n / (oms * 1e-3), 1),
                "timed_replays": reps, "identical_after_100_steps": same}

    def maintenance_times():
        """The lattice update alone, per step (HIP events, eager, K steps
        each): move the by-id arrays + full counting-sort rebuild; move the
        lattice's records + rebuild from them; the incremental update."""
        lat = sphidx.Lattice(spec.log2_cells, spec.frac_bits, spec.cyclic_mask, n)
        pos = [sphidx.to_dev_u32(c) for c in w.pts]
        desc = sphidx.desc_of(spec.log2_cells, spec.frac_bits, spec.cyclic_mask)
        lat.build(*pos)
        rec = torch.empty(4 * n, dtype=torch.int32, device="cuda")
        inc = torch.empty(sphidx.move_incremental_scratch_bytes(lat) // 4 + 1, dtype=torch.int32, device="cuda")
        res = {}
        reps = max(5, min(K, 20))
        for tag, fn in (("rebuild", lambda t: (sphidx.move_agents(desc, seed, t, *pos), lat.build(*pos))),
                        ("resident", lambda t: sphidx.move_resident(lat, seed, rec, step=t)),
                        ("incremental", lambda t: sphidx.move_incremental(lat, seed, inc, step=t))):
            for t in range(3):
                fn(t)
            ev = event_pairs(reps)
            for t, (e0, e1) in enumerate(ev):
                e0.record()
                fn(3 + t)
                e1.record()
            torch.cuda.synchronize()
            res[tag] = round(mean_ms(ev), 4)
        code_m, _ = lat.status()
        res["status_ok"] = code_m == sphidx.OK
        log(f"lattice update per step: {res}")
        del lat, pos, rec, inc
        torch.cuda.empty_cache()
        return res

    base = {}
    if not args.no_baselines:
        base["cube_scan"] = other("cube", dataclasses.replace(sim.launch, method=sphidx.METHOD_CUBE))
        base["plain_launch"] = other("plain", sphidx.LaunchConfig(method=sphidx.METHOD_SPHERE,
                                                                   schedule=sphidx.SCHED_PLAIN))
        base["paper64"] = other("paper64", sphidx.LaunchConfig(method=sphidx.METHOD_PAPER64))
        base["paper64"]["step"] = ("the same step with the paper's 64 specialised cell tables and the Eq. 1 "
                                   "run-time test (one query per wavefront)")
        base["rebuild_by_id"] = other("rebuild by id", sim.launch, resident=False)
        base["rebuild_by_id"]["step"] = ("move the by-id coordinate arrays + counting-sort rebuild from them + "
                                         "count + scan + write + checksum, one graph replay")
        base["incremental"] = other("incremental", sim.launch, resident=False, incremental=True)
        base["incremental"]["step"] = ("move the lattice's records + place again only the agents that changed "
                                       "cell (stayers keep their order) + count + scan + write + checksum")
        base["maintenance_ms"] = maintenance_times()

    exact, cpu, checks = None, None, {}
    if not args.no_cpu:
        import oracle
        L = oracle.Lattice(spec.log2_cells, spec.frac_bits, spec.cyclic_mask)
        # the oracle doing one step's work: move and grid build over every
        # agent, sorted radius rows of a sample, scaled to all agents
        samp = sample_of(n, 1 << 19, 5)
        t0 = time.perf_counter()
        moved = oracle.move(L, seed, 0, w.pts)
        t1 = time.perf_counter()
        g = oracle.Grid(L, moved)
        t2 = time.perf_counter()
        g.radius(r, queries=tuple(np.asarray(c)[samp] for c in moved))
        t3 = time.perf_counter()
        g.close()
        step_s = (t1 - t0) + (t2 - t1) + (t3 - t2) * n / len(samp)
        cpu = {"value": round(n / step_s, 1), "unit": "queries/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"one step: move + grid build of all {n} agents ({t2 - t0:.2f} s) and the sorted radius "
                         f"rows of {len(samp)} sampled agents ({t3 - t2:.2f} s), scaled to all agents",
               **host_info()}
        # the replay: row sizes of the sampled agents at step 50; at the final
        # step every position, the count checksum over all rows and the rows
        # of 32,768 sampled agents
        cur = w.pts
        for t in range(final):
            cur = oracle.move(L, seed, t, cur)
            if t + 1 in mid:
                g = oracle.Grid(L, cur)
                cnt = g.radius_counts(r, queries=tuple(np.asarray(c)[rows] for c in cur))
                g.close()
                checks[f"step_{t + 1}_sampled_row_sizes"] = bool(np.array_equal(cnt, mid[t + 1].cpu().numpy()))
        pos_ok = all(np.array_equal(u, v) for u, v in zip(sim.positions(), cur))
        g = oracle.Grid(L, cur)
        counts = g.radius_counts(r)
        orp = np.zeros(n + 1, np.int64)
        orp[1:] = np.cumsum(counts)
        checks[f"step_{final}_positions"] = pos_ok
        checks[f"step_{final}_count_checksum_all_rows"] = sim.checksum() == oracle.count_checksum(orp)
        checks[f"step_{final}_row_sizes_all_rows"] = bool(np.array_equal(rp, orp))
        srows = sample_of(n, 32768, 6)
        srp, sids = sample_rows(rp, sim.buf.ids, srows)
        ref = g.radius(r, queries=tuple(np.asarray(c)[srows] for c in cur))
        g.close()
        checks[f"step_{final}_sampled_rows"] = same_rows(srp, sids, ref)
        exact = all(checks.values())
        log(f"timestep oracle checks: {checks}")
        log(f"cpu oracle: {cpu['value']:.0f} agent-queries/s on {cpu['cores']} threads")

    alg = query_bytes(n, ncells, n, pairs)
    upd = resident_update_bytes(n, ncells)
    step_alg = upd["move"] + upd["rebuild"] + alg
    rl = roofline(w.name, ("group_count_kernel" if cfg.get("grouped") else "count_kernel")
                  + " (walk, test, sort, keep rows)", alg, kern_ms, out.get("hbm_copy_GBps"),
                  {"step": {"algorithmic_bytes": int(step_alg), "ms": round(ms, 4),
                            "achieved": round(step_alg / (ms * 1e-3) / 1e9, 2),
                            "frac": round(step_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                            "bytes": {**upd, "query": alg}},
                   "library_overhead_bytes": overhead_bytes(n, pairs)})
    out.update({
        "metric": METRIC,
        "value": round(n / (ms * 1e-3), 1),
        "unit": "queries/s",
        "ms_per_step": round(ms, 4),
        "config": {"workload": w.name, "agents": n, "lattice": "256^3 cyclic, cell edge 2^16 units",
                   "radius": "3 cells", "steps": 100,
                   "step": "move the lattice's records + rebuild it from them + count + scan + write + "
                           "checksum, one graph replay",
                   "subcell_bits": sbits, "launch": dict(cfg, schedule="persistent")},
        "pairs_per_step": pairs,
        "pairs_per_s": round(pairs / (ms * 1e-3), 1),
        "wall_ms_per_step": round(wall, 4),
        "count_kernel_ms": round(kern_ms, 4),
        "status_ok": code == sphidx.OK and flags == 0,
        "bit_exact_vs_oracle": exact,
        "oracle_checks": checks,
        "roofline": rl,
        "cpu_baseline": cpu,
    })
    if base:
        out.update(base)
        out["speedup_vs_cube"] = round(base["cube_scan"]["ms_per_step"] / ms, 3)
        out["speedup_vs_plain"] = round(base["plain_launch"]["ms_per_step"] / ms, 3)
    del sim
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# Plain radius query at CPU scale (4,096 points)

def leg_c1(args, out):
    import numpy as np
    import torch

    from paper_cs_0608108_amd import sphidx, synth

    w = synth.radius_uniform_cyclic()
    spec, n, r = w.lat, w.n, int(w.r_fx[0])
    ncells = 1 << sum(spec.log2_cells)
    log(f"workload {w.name}: n={n}")
    lat = sphidx.Lattice(spec.log2_cells, spec.frac_bits, spec.cyclic_mask, n)
    dev = [sphidx.to_dev_u32(a) for a in w.pts]
    tab = sphidx.Tables(lat, 2, r)
    q = sphidx.make_queries(n, None, r)
    buf = sphidx.QueryBuffers(n, 0, want_dist2=True)
    lat.build(*dev)
    sphidx.count(lat, tab, q, buf)
    total = int(buf.row_ptr[-1].item())
    buf.grow(total)
    buf.reserve_stash(total)
    ln = sphidx.LaunchConfig()
    K = max(args.steps, 10)
    for _ in range(3):
        lat.build(*dev)
        sphidx.count(lat, tab, q, buf, ln)
        sphidx.write(lat, tab, q, buf, ln)
    torch.cuda.synchronize()
    kev = event_pairs(K)
    lc = [dataclasses.replace(ln, events=e) for e in kev]
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for s in range(K):
        lat.build(*dev)
        sphidx.count(lat, tab, q, buf, lc[s])
        sphidx.write(lat, tab, q, buf, ln)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / K
    kern_ms = mean_ms(kev)
    rp, ids, d2 = buf.host()
    exact, cpu = None, None
    if not args.no_cpu:
        import oracle
        L = oracle.Lattice(spec.log2_cells, spec.frac_bits, spec.cyclic_mask)
        times = {}
        ref = None
        for threads in (oracle.num_threads(), 1):
            nthr = oracle.num_threads()
            oracle.set_num_threads(threads)
            reps, spent = 0, 0.0
            while reps < 20 and spent < 2.0:
                t0 = time.perf_counter()
                ref = oracle.radius_brute(L, w.pts, w.r_fx)
                spent += time.perf_counter() - t0
                reps += 1
            times[threads] = spent / reps
            oracle.set_num_threads(nthr)
        exact = bool(np.array_equal(ref.row_ptr, rp) and np.array_equal(ref.ids, ids)
                     and np.array_equal(ref.dist2, d2))
        thr = max(times)
        cpu = {"value": round(n / times[thr], 1), "unit": "queries/s", "cores": thr, "kind": "oracle",
               "sample": "full workload, brute force (every query against every point, sorted rows)",
               "one_thread_queries_per_s": round(n / times[1], 1), **host_info()}
        log(f"c1: {ms:.4f} ms/step; oracle {cpu['value']:.0f} q/s ({thr} threads), "
            f"{cpu['one_thread_queries_per_s']:.0f} q/s (1 thread); bit-exact {exact}")
    alg = query_bytes(n, ncells, n, total, dist2=True)
    out["c1"] = {"workload": w.name, "ms_per_step": round(ms, 4), "queries_per_s": round(n / (ms * 1e-3), 1),
                 "step": "rebuild + count + scan + write (ids and dist2)", "pairs_per_step": total,
                 "bit_exact_vs_oracle": exact,
                 "roofline": roofline(w.name, "count_kernel (walk, test, sort, keep rows)", alg, kern_ms,
                                      out.get("hbm_copy_GBps")),
                 "cpu_baseline": cpu}
    del buf, lat, tab, dev


# ---------------------------------------------------------------------------
# Batched uneven-radius all-agents query

def leg_c2(args, out):
    import numpy as np
    import torch

    from paper_cs_0608108_amd import sphidx, synth

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
    tabs = {2: tab}

    def subcell_step(ln, sb):
        if sb not in tabs:
            tabs[sb] = sphidx.Tables(lat, sb, rmax)

        def run():
            lat.build(*dev)
            sphidx.count(lat, tabs[sb], q, buf, ln)
            sphidx.write(lat, tabs[sb], q, buf, ln)
        return run

    cfg, sbits = tuned_config(args, shape, lambda ln: (lambda: step(ln)), subcell_runner=subcell_step)
    tab = tabs[sbits] if sbits in tabs else sphidx.Tables(lat, sbits, rmax)
    tabs.clear()
    tuned = sphidx.LaunchConfig(method=sphidx.METHOD_SPHERE, schedule=sphidx.SCHED_PERSISTENT, **cfg)
    log(f"launch config: {cfg}, sub-cell bits {sbits}")

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

    K = max(args.steps, 10)
    ms, phases, kern = timed(tuned, K, args.warmup)
    # the paper's protocol beside the mean (Section IV.A: repeat, drop the
    # slowest quarter, average the rest), from the per-step events
    per = np.sort(timed.per_step)
    kept = per[: max(1, len(per) - len(per) // 4)]
    res = {"paper_protocol": {"steps": int(len(per)), "dropped_slowest": int(len(per) - len(kept)),
                              "mean_ms": round(float(kept.mean()), 4), "median_ms": round(float(np.median(per)), 4),
                              "queries_per_s": round(n / (float(kept.mean()) * 1e-3), 1)}}
    code, flags = lat.status()
    assert code == sphidx.OK, (code, flags)
    rp = buf.row_ptr.cpu().numpy()
    ids = buf.ids[: int(rp[-1])].cpu().numpy().view(np.uint32)
    log(f"c2 persistent: {ms:.3f} ms/step; build {phases[0]:.3f} count {phases[1]:.3f} write {phases[2]:.3f} ms; "
        f"count kernel {kern[0]:.3f} write kernels {kern[1]:.3f} ms")

    # cells and candidate objects per query, sphere tables against the
    # bin-lattice cube: the per-query statistics of one count pass each
    # (untimed; the rows found above are kept on the host)
    cells = {}
    for name, meth in (("sphere", sphidx.METHOD_SPHERE), ("cube", sphidx.METHOD_CUBE),
                       ("paper64", sphidx.METHOD_PAPER64)):
        st = torch.zeros(4 * n, dtype=torch.int32, device="cuda")
        sphidx.count(lat, tab, q, buf, sphidx.LaunchConfig(method=meth, stats=st))
        a = st.cpu().numpy().view(np.uint32).reshape(n, 4).astype(np.float64)
        cells[name] = {"rows_walked": round(float(a[:, 0].mean()), 3), "cells_kept": round(float(a[:, 1].mean()), 3),
                       "candidates": round(float(a[:, 2].mean()), 3)}
        del st
    cells["hits"] = round(total / n, 3)
    cells["kept_over_cube"] = round(cells["sphere"]["cells_kept"] / cells["cube"]["cells_kept"], 4)
    cells["candidates_over_cube"] = round(cells["sphere"]["candidates"] / cells["cube"]["candidates"], 4)
    res["cells_per_query"] = cells
    log(f"per query: sphere {cells['sphere']}, cube {cells['cube']}, hits {cells['hits']}")

    if not args.no_baselines:
        k2 = max(3, K // 2)
        ms_tw, ph_tw, k_tw = timed(dataclasses.replace(tuned, no_stash=1), k2, 1)
        res["without_stash"] = {"ms_per_step": round(ms_tw, 4), "count_kernel_ms": round(float(k_tw[0]), 4),
                                "write_kernels_ms": round(float(k_tw[1]), 4)}
        plain = sphidx.LaunchConfig(method=sphidx.METHOD_SPHERE, schedule=sphidx.SCHED_PLAIN)
        ms_plain, ph_plain, _ = timed(plain, k2, 1)
        cube = sphidx.LaunchConfig(method=sphidx.METHOD_CUBE, schedule=sphidx.SCHED_PERSISTENT, **cfg)
        ms_cube, ph_cube, k_cube = timed(cube, K, 2)
        rp_c = buf.row_ptr.cpu().numpy()
        ids_c = buf.ids[: int(rp_c[-1])].cpu().numpy().view(np.uint32)
        same = bool(np.array_equal(rp_c, rp) and np.array_equal(ids_c, ids))
        res.update({
            "plain_launch": {"ms_per_step": round(ms_plain, 4), "queries_per_s": n / (ms_plain * 1e-3),
                             "query_ms": round(float(ph_plain[1] + ph_plain[2]), 4)},
            "cube_scan": {"ms_per_step": round(ms_cube, 4), "queries_per_s": n / (ms_cube * 1e-3),
                          "query_ms": round(float(ph_cube[1] + ph_cube[2]), 4),
                          "count_kernel_ms": round(float(k_cube[0]), 4), "same_result": same},
            "speedup_vs_plain": round(ms_plain / ms, 3),
            "speedup_vs_cube": round(ms_cube / ms, 3),
        })
        log(f"without stash {ms_tw:.3f}; plain {ms_plain:.3f}; cube {ms_cube:.3f} ms/step (count kernel "
            f"{k_cube[0]:.3f}); cube result identical: {same}")
        # the paper's own table design (64 specialised cell tables, Eq. 1
        # run-time test), one query per wavefront, against the row tables in
        # the same launch shape
        one = dataclasses.replace(tuned, grouped=0)
        ms_one, _, k_one = timed(one, k2, 1)
        ms_p64, _, k_p64 = timed(sphidx.LaunchConfig(method=sphidx.METHOD_PAPER64, schedule=sphidx.SCHED_PERSISTENT,
                                                     **{k_: v for k_, v in cfg.items()
                                                        if k_ not in ("grouped", "table_in_lds")}), k2, 1)
        rp_p = buf.row_ptr.cpu().numpy()
        ids_p = buf.ids[: int(rp_p[-1])].cpu().numpy().view(np.uint32)
        res["paper64"] = {"ms_per_step": round(ms_p64, 4), "count_kernel_ms": round(float(k_p64[0]), 4),
                          "row_tables_one_query_per_wave_ms_per_step": round(ms_one, 4),
                          "row_tables_one_query_per_wave_count_kernel_ms": round(float(k_one[0]), 4),
                          "same_result": bool(np.array_equal(rp_p, rp) and np.array_equal(ids_p, ids))}
        log(f"paper64: {ms_p64:.3f} ms/step (count kernel {k_p64[0]:.3f}); row tables one query per wave "
            f"{ms_one:.3f} (count kernel {k_one[0]:.3f}); same {res['paper64']['same_result']}")
        # the row table staged in LDS, whole and in per-class chunks, against
        # the tuned launch that reads it from device memory
        lds = {"table_bytes": int(tab.info().total_entries) * 16, "device_memory_ms_per_step": round(ms, 4),
               "device_memory_count_kernel_ms": round(float(kern[0]), 4)}
        for mode, tag in ((1, "whole"), (2, "chunked")):
            try:
                ms_l, _, k_l = timed(dataclasses.replace(tuned, table_in_lds=mode), k2, 1)
            except sphidx.SphidxError as e:
                lds[tag] = {"refused": str(e)}
                continue
            rp_l = buf.row_ptr.cpu().numpy()
            ids_l = buf.ids[: int(rp_l[-1])].cpu().numpy().view(np.uint32)
            lds[tag] = {"ms_per_step": round(ms_l, 4), "count_kernel_ms": round(float(k_l[0]), 4),
                        "same_result": bool(np.array_equal(rp_l, rp) and np.array_equal(ids_l, ids))}
        res["table_in_lds"] = lds
        log(f"row table in LDS: {lds}")
        # the per-query choice (Section III.B/C) with the tuned launch, by
        # cells (the paper's volumes) and by estimated lane work; the
        # non-empty cell list is kept (and rebuilt) only here
        lat.attach_cell_list()
        timed(dataclasses.replace(tuned, method=sphidx.METHOD_AUTO), 3, 2)
        for model, tag in ((0, "auto_choice"), (1, "auto_work")):
            mo = torch.empty(n, dtype=torch.int32, device="cuda")
            auto = dataclasses.replace(tuned, method=sphidx.METHOD_AUTO, method_out=mo, select_model=model)
            ms_auto, ph_auto, k_auto = timed(auto, k2, 3)
            rp_a = buf.row_ptr.cpu().numpy()
            ids_a = buf.ids[: int(rp_a[-1])].cpu().numpy().view(np.uint32)
            used = torch.bincount(mo.long(), minlength=4).cpu().tolist()
            res[tag] = {"ms_per_step": round(ms_auto, 4), "query_ms": round(float(ph_auto[1] + ph_auto[2]), 4),
                        "rebuild_ms": round(float(ph_auto[0]), 4), "count_kernel_ms": round(float(k_auto[0]), 4),
                        "chose": {"sphere": used[sphidx.METHOD_SPHERE], "cube": used[sphidx.METHOD_CUBE],
                                  "list": used[sphidx.METHOD_LIST]},
                        "same_result": bool(np.array_equal(rp_a, rp) and np.array_equal(ids_a, ids))}
            log(f"{tag}: {ms_auto:.3f} ms/step, chose {res[tag]['chose']}")
        lat.attach_cell_list(False)

    cpu, exact = None, None
    if not args.no_cpu:
        import oracle
        L = oracle.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask)
        reps, spent, ref = 0, 0.0, None
        while reps < 8 and spent < 8.0:
            t0 = time.perf_counter()
            g = oracle.Grid(L, w.pts)
            ref = g.radius(w.r_fx)
            spent += time.perf_counter() - t0
            g.close()
            reps += 1
        exact = bool(np.array_equal(ref.row_ptr, rp) and np.array_equal(ref.ids, ids))
        # one thread, on the first 131,072 queries of the same workload
        nthr = oracle.num_threads()
        oracle.set_num_threads(1)
        sub = 1 << 17
        t0 = time.perf_counter()
        g = oracle.Grid(L, w.pts)
        t1 = time.perf_counter()
        g.radius(w.r_fx[:sub], queries=tuple(np.asarray(c)[:sub] for c in w.pts))
        t2 = time.perf_counter()
        g.close()
        oracle.set_num_threads(nthr)
        one = n / ((t1 - t0) + (t2 - t1) * n / sub)
        cpu = {"value": round(n * reps / spent, 1), "unit": "queries/s", "cores": nthr, "kind": "oracle",
               "sample": f"full workload ({n} queries: grid build + radius + row sort) x{reps}, {spent:.1f} s",
               "one_thread_queries_per_s": round(one, 1),
               "one_thread_sample": f"grid build + the first {sub} queries, scaled to {n}", **host_info()}
        log(f"cpu oracle: {cpu['value']:.0f} queries/s on {nthr} threads, {one:.0f} on 1; GPU bit-exact: {exact}")

    alg = query_bytes(n, lat.ncells, n, total)
    res.update({
        "workload": w.name, "ms_per_step": round(ms, 4), "queries_per_s": round(n / (ms * 1e-3), 1),
        "pairs_per_step": total, "pairs_per_s": round(total / (ms * 1e-3), 1),
        "config": {"points": n, "lattice": "128^3 clipped, cell edge 2^16 units",
                   "radius": "per point, uniform [0.5, 4] cells, 1/64-cell steps", "subcell_bits": sbits,
                   "launch": dict(cfg, schedule="persistent")},
        "step": "rebuild + count + scan + write",
        "phase_ms": {"rebuild": round(float(phases[0]), 4), "count": round(float(phases[1]), 4),
                     "write": round(float(phases[2]), 4)},
        "bit_exact_vs_oracle": exact,
        "roofline": roofline(w.name, ("group_count_kernel" if cfg.get("grouped") else "count_kernel")
                             + " (walk, test, sort, keep rows)", alg, float(kern[0]), out.get("hbm_copy_GBps"),
                             {"write_pass_ms": round(float(kern[1]), 4),
                              "library_overhead_bytes": overhead_bytes(n, total)}),
        "cpu_baseline": cpu,
    })
    out["c2"] = res
    del buf, lat, tab, dev, rad
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# K-NN under heavy load

def leg_knn(args, out):
    import numpy as np
    import torch

    from paper_cs_0608108_amd import sphidx, synth

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
    # row once and keeps it, and the write pass only copies (rows searched in
    # groups as radius rows keep their first K; the rest of the room absorbs
    # the regions' unused chunk tails)
    buf = sphidx.QueryBuffers(n, n * K, want_dist2=False, stash_pairs=3 * n * K)

    def step_with(launch, count_launch=None):
        def run():
            lat.build(*dev)
            sphidx.count(lat, tab, q, buf, count_launch or launch)
            sphidx.write(lat, tab, q, buf, launch)
        return run

    shape = dict(workload=w.name, n=n, k=K)
    tabs = {2: tab}

    def subcell_step(ln_, sb):
        if sb not in tabs:
            tabs[sb] = sphidx.Tables(lat, sb, cap)

        def run():
            lat.build(*dev)
            sphidx.count(lat, tabs[sb], q, buf, ln_)
            sphidx.write(lat, tabs[sb], q, buf, ln_)
        return run

    cfg, sbits = tuned_config(args, shape, step_with, subcell_runner=subcell_step)
    tab = tabs[sbits] if sbits in tabs else sphidx.Tables(lat, sbits, cap)
    tabs.clear()
    ln = sphidx.LaunchConfig(**cfg)
    log(f"knn launch config: {cfg}, sub-cell bits {sbits}")
    # the order of the objects inside a cell: the counting sort's, or by x
    # (rows over dense cells then narrowed to the sphere's x-slab); the
    # faster of the two, each over a few steps
    order_ms = {}
    for order in (sphidx.ORDER_ANY, sphidx.ORDER_X):
        lat.set_cell_order(order)
        for _ in range(2):
            step_with(ln)()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            step_with(ln)()
        e1.record()
        torch.cuda.synchronize()
        order_ms["x" if order == sphidx.ORDER_X else "any"] = round(e0.elapsed_time(e1) / 5, 4)
    order = sphidx.ORDER_X if order_ms["x"] < order_ms["any"] else sphidx.ORDER_ANY
    lat.set_cell_order(order)
    log(f"knn cell order: {order_ms} ms/step -> {'x' if order else 'any'}")
    for _ in range(2):
        step_with(ln)()
    torch.cuda.synchronize()
    reps = max(5, min(args.steps, 20))
    kev = event_pairs(reps)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for e in kev:
        step_with(ln, dataclasses.replace(ln, events=e))()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    kern_ms = mean_ms(kev)
    rp = buf.row_ptr.cpu().numpy()
    pairs = int(rp[-1])
    log(f"knn sphere: {ms:.3f} ms/step, count kernel {kern_ms:.3f} ms, pairs {pairs}")
    res = {}
    rows = sample_of(n, 65536, 3)
    if not args.no_baselines:
        # sphere vs cube on the same subsample of query centres (the cube scan
        # looks at every object of the 17^3-cell cap cube, so all N would
        # take long)
        cen = tuple(sphidx.to_dev_u32(np.asarray(c)[rows]) for c in w.pts)
        qs = sphidx.make_queries(len(rows), cen, cap, K, sphidx.MODE_KNN, 0)
        bs = sphidx.QueryBuffers(len(rows), len(rows) * K, want_dist2=False, stash_pairs=3 * len(rows) * K)
        sub = {}
        for name, meth in (("sphere", sphidx.METHOD_SPHERE), ("cube", sphidx.METHOD_CUBE)):
            lq = sphidx.LaunchConfig(**dict(cfg, method=meth))
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
        res["subsample"] = {"queries": int(len(rows)), "sphere_ms": round(sub["sphere"], 4),
                            "cube_ms": round(sub["cube"], 4), "speedup_vs_cube": round(sub["cube"] / sub["sphere"], 3),
                            "sphere_equals_cube": same_sub}
        log(f"knn subsample {len(rows)}: sphere {sub['sphere']:.3f} ms, cube {sub['cube']:.3f} ms, same {same_sub}")
        del bs, cen
    exact, cpu = None, None
    if not args.no_cpu:
        import oracle
        L = oracle.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask)
        t0 = time.perf_counter()
        g = oracle.Grid(L, w.pts)
        t1 = time.perf_counter()
        ref = g.knn(K, cap, queries=tuple(np.asarray(c)[rows] for c in w.pts))
        t2 = time.perf_counter()
        g.close()
        srp, sids = sample_rows(rp, buf.ids, rows)
        exact = same_rows(srp, sids, ref)
        cpu = {"value": round(n / ((t1 - t0) + (t2 - t1) * n / len(rows)), 1), "unit": "queries/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"grid build ({t1 - t0:.2f} s) + the K nearest of {len(rows)} sampled points "
                         f"({t2 - t1:.2f} s), scaled to all {n}", **host_info()}
        log(f"knn oracle: {cpu['value']:.0f} q/s; sampled rows bit-exact {exact}")
    alg = query_bytes(n, lat.ncells, n, pairs)
    res.update({"workload": w.name, "ms_per_step": round(ms, 4), "queries_per_s": round(n / (ms * 1e-3), 1),
                "launch": dict(cfg, schedule="persistent"), "subcell_bits": sbits,
                "cell_order": "x" if order else "any", "ms_per_step_by_cell_order": order_ms,
                "step": "rebuild + K-NN count + scan + write (top-K rows, sorted by (dist2, id))",
                "pairs_per_step": pairs,
                "sampled_rows_bit_exact_vs_oracle": exact,
                "roofline": roofline(w.name, ("group_count_kernel" if cfg.get("grouped") else "count_kernel")
                                     + " (K-NN rows searched, sorted and kept)", alg, kern_ms,
                                     out.get("hbm_copy_GBps"),
                                     {"library_overhead_bytes": overhead_bytes(n, pairs)}),
                "cpu_baseline": cpu})
    out["knn"] = res
    del buf, lat, tab, dev
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
    warm = 16
    sizes = synth.serving_batch_sizes(seed, nb + warm, 65536)
    qs = [synth.serving_batch(spec, seed, i, int(s)) for i, s in enumerate(sizes)]
    sizes, wq = sizes[warm:], qs[:warm]
    qs = qs[warm:]
    pool = 4 << 30
    slots = args.serving_slots

    def make(arrivals, src=qs):
        return [serving.Batch(i, float(arrivals[i]), q, r, k) for i, (q, r, k) in enumerate(src)]

    # the launch for the serving mix: tuned on one 16,384-query batch of it
    tq, tr, tk = synth.serving_batch(spec, seed, 1 << 14, 16384)
    tdev = (tuple(sphidx.to_dev_u32(c) for c in tq), sphidx.to_dev_u32(tr), sphidx.to_dev_u32(tk))
    tqq = sphidx.make_queries(16384, tdev[0], tdev[1], tdev[2], sphidx.MODE_MIXED)
    tbuf = sphidx.QueryBuffers(16384, 0, want_dist2=False)
    sphidx.count(lat, tab, tqq, tbuf)
    tt = int(tbuf.row_ptr[-1].item())
    tbuf.grow(tt)
    tbuf.reserve_stash(tt)

    def tstep(ln):
        def run():
            sphidx.count(lat, tab, tqq, tbuf, ln)
            sphidx.write(lat, tab, tqq, tbuf, ln)
        return run

    tabs = {2: tab}

    def subcell_step(ln_, sb):
        if sb not in tabs:
            tabs[sb] = sphidx.Tables(lat, sb, 16 * spec.edge)

        def run():
            sphidx.count(lat, tabs[sb], tqq, tbuf, ln_)
            sphidx.write(lat, tabs[sb], tqq, tbuf, ln_)
        return run

    cfg, sbits = tuned_config(args, dict(workload=w.name, batch="mix16384"), tstep, subcell_runner=subcell_step)
    tab = tabs[sbits] if sbits in tabs else sphidx.Tables(lat, sbits, 16 * spec.edge)
    tabs.clear()
    fast_ln = sphidx.LaunchConfig(**cfg)
    log(f"serving launch config: {cfg}, sub-cell bits {sbits}")

    # roofline of the query passes on one full-size batch of the mix: the
    # bytes a random-centre query must touch (centre, radius or K, the
    # cell_start entries of its kept cells, its candidate records, its row,
    # its row_ptr entry), from the count pass's per-query statistics
    bq, br, bk = synth.serving_batch(spec, seed, 1 << 15, 65536)
    bdev = (tuple(sphidx.to_dev_u32(c) for c in bq), sphidx.to_dev_u32(br), sphidx.to_dev_u32(bk))
    bqq = sphidx.make_queries(65536, bdev[0], bdev[1], bdev[2], sphidx.MODE_MIXED)
    bbuf = sphidx.QueryBuffers(65536, 0, want_dist2=False)
    st = torch.zeros(4 * 65536, dtype=torch.int32, device="cuda")
    sphidx.count(lat, tab, bqq, bbuf, sphidx.LaunchConfig(stats=st))
    bt = int(bbuf.row_ptr[-1].item())
    sa = st.cpu().numpy().view(np.uint32).reshape(65536, 4).astype(np.int64)
    b_alg = int((12 + 4 + 8) * 65536 + 4 * sa[:, 1].sum() + 16 * sa[:, 2].sum() + 4 * bt)
    bbuf.grow(bt)
    bbuf.reserve_stash(bt)
    for _ in range(2):
        tstep(fast_ln)()
        sphidx.count(lat, tab, bqq, bbuf, fast_ln)
        sphidx.write(lat, tab, bqq, bbuf, fast_ln)
    torch.cuda.synchronize()
    pev = event_pairs(5)
    for e0, e1 in pev:
        e0.record()
        sphidx.count(lat, tab, bqq, bbuf, fast_ln)
        sphidx.write(lat, tab, bqq, bbuf, fast_ln)
        e1.record()
    torch.cuda.synchronize()
    batch_ms = mean_ms(pev)
    del st, tbuf, bbuf

    # both paths are the library's serving loop (sphidx_server_*): the
    # continuous one with `slots` streams and the tuned persistent launch,
    # the baseline with one slot and the plain schedule (count, size, write,
    # then the next batch)
    torch.cuda.synchronize()
    fast = sphidx.Server(lat, tab, slots, int(sizes.max()), pool, stash_pairs=1 << 25, launch=fast_ln)
    plain = sphidx.Server(lat, tab, 1, int(sizes.max()), pool, stash_pairs=1 << 25,
                          launch=sphidx.LaunchConfig(schedule=sphidx.SCHED_PLAIN))
    paths = (("continuous", fast, slots), ("plain_per_batch", plain, 1))
    for _, ex, sl in paths:
        serving.run_on_server(ex, make(np.zeros(warm), wq))
    # capacity: every batch queued at t = 0
    res = {}
    for name, ex, sl in paths:
        bs = make(np.zeros(nb))
        serving.run_on_server(ex, bs)
        res[name + "_saturated"] = serving.latency_stats(bs)
        log(f"serving {name} saturated: {res[name + '_saturated']['queries_per_s']:.0f} q/s")
    mean_batch = float(sizes.mean())
    sat = {name: res[name + "_saturated"]["queries_per_s"] / mean_batch for name, _, _ in paths}

    def offered(name, ex, sl, rate, tag):
        arr = np.cumsum(synth.serving_interarrivals(seed + tag, nb, rate))
        bs = make(arr)
        peak = serving.run_on_server(ex, bs)
        s = serving.latency_stats(bs)
        s.update({"batches_per_s": round(rate, 2), "pool_peak_bytes": peak,
                  "rejected": sum(b.rejected for b in bs)})
        return s

    # Poisson arrivals at fractions of each path's own saturated batch rate
    # (both stable), then at one absolute rate both sustain -- 0.8 of the
    # plain path's capacity -- twice, with two arrival sequences, for the
    # p99 comparison and its run-to-run spread
    own = {}
    for frac in (0.5, 0.8, 0.95):
        own[f"{frac:.2f}"] = {name: offered(name, ex, sl, frac * sat[name], 0) for name, ex, sl in paths}
        log(f"serving own-rate {frac}: " + ", ".join(
            f"{k} p50 {v['p50_ms']:.2f} p99 {v['p99_ms']:.2f} ms" for k, v in own[f"{frac:.2f}"].items()))
    common_rate = 0.8 * sat["plain_per_batch"]
    common = []
    for tag in (100, 200):
        row = {name: offered(name, ex, sl, common_rate, tag) for name, ex, sl in paths}
        row["p99_speedup_vs_plain"] = round(row["plain_per_batch"]["p99_ms"] / row["continuous"]["p99_ms"], 3)
        common.append(row)
        log(f"serving common rate {common_rate:.1f}/s (arrivals {tag}): continuous p99 "
            f"{row['continuous']['p99_ms']:.2f}, plain p99 {row['plain_per_batch']['p99_ms']:.2f} ms")
    p99s = [r["p99_speedup_vs_plain"] for r in common]

    exact, cpu = None, None
    if not args.no_cpu:
        # a stratified sample of batches, the two largest among them, through
        # the continuous path, every row against the oracle
        import oracle
        order = np.argsort(sizes)
        pick = sorted(set(order[-2:].tolist()) | {int(order[int(f * (nb - 1))]) for f in np.linspace(0, 0.97, 10)})
        chk = make(np.zeros(nb))
        chk = [chk[i] for i in pick]
        serving.run_on_server(fast, chk, keep=True)
        L = oracle.Lattice(spec.log2_cells, spec.frac_bits, spec.cyclic_mask)
        g = oracle.Grid(L, w.pts)
        exact = True
        t_or, nq = 0.0, 0
        for b in chk:
            t0 = time.perf_counter()
            ref = g.mixed(b.k, b.radius, queries=b.centres)
            t_or += time.perf_counter() - t0
            nq += b.size
            rp, ids = b.result
            exact &= bool(np.array_equal(rp, ref.row_ptr) and np.array_equal(ids, ref.ids))
        g.close()
        cpu = {"value": round(nq / t_or, 1), "unit": "queries/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{len(chk)} batches ({nq} queries, sizes {sorted(int(b.size) for b in chk)}), "
                         f"the rows of each mixed batch on a plain grid", **host_info()}
        log(f"serving oracle: {cpu['value']:.0f} q/s; {len(chk)} batches bit-exact {exact}")
    out["serving"] = {
        "workload": w.name, "batches": nb, "warmup_batches": warm, "slots": slots,
        "loop": "the library's serving loop (sphidx_server_run) for both paths",
        "launch": dict(cfg, schedule="persistent"), "subcell_bits": sbits,
        "mean_batch": mean_batch, "median_batch": float(np.median(sizes)), **res,
        "load_own_rate": own,
        "load_own_rate_note": "Poisson arrivals at 0.5 / 0.8 / 0.95 of each path's own saturated batch rate",
        "common_rate": {"batches_per_s": round(common_rate, 2),
                        "note": "0.8 of the plain path's saturated batch rate, both paths, two arrival sequences",
                        "runs": common},
        "p99_speedup_vs_plain": round(float(np.mean(p99s)), 3),
        "p99_speedup_vs_plain_runs": p99s,
        "capacity_ratio_vs_plain": round(sat["continuous"] / sat["plain_per_batch"], 3),
        "stratified_batches_bit_exact_vs_oracle": exact,
        "roofline": roofline(w.name, "count + write passes of one 65,536-query batch of the mix", b_alg,
                             batch_ms, out.get("hbm_copy_GBps"),
                             {"bytes_per_query": round(b_alg / 65536, 1), "pairs": bt}),
        "cpu_baseline": cpu,
    }
    fast.close()
    plain.close()
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
                        # the paper's own table design (64 specialised cell
                        # tables, Eq. 1 run-time test)
                        t_p, b_p = timed_query(lat, tab, q, sphidx.LaunchConfig(method=sphidx.METHOD_PAPER64))
                        same_p = bool(torch.equal(b_s.row_ptr, b_p.row_ptr) and
                                      torch.equal(b_s.ids[:n_s], b_p.ids[:n_s]))
                        mismatches += 0 if same_p else 1
                        point[key].update({"paper64_ms": round(t_p, 4), "ratio_paper64": round(t_c / t_p, 3),
                                           "same_paper64": same_p})
                        del b_p
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
                        f" nearest x{point['nearest']['ratio']} paper64 x{point['all']['ratio_paper64']}")
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
    ap.add_argument("--serving-batches", type=int, default=2000)
    # slots of the continuous serving path: capacity on the serving mix grew
    # with slots up to about 8 (1: 14.9, 2: 24.6, 4: 31.5, 8: 36.9, 12: 37.3,
    # 16: 37.1 M queries/s over 1,000 batches), most batches being too small
    # to fill the GPU alone
    ap.add_argument("--serving-slots", type=int, default=8)
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
    if legs != ["tables"]:
        out["hbm_copy_GBps"] = round(copy_bandwidth(), 1)
        log(f"device copy: {out['hbm_copy_GBps']} GB/s (read + write)")
    # no cyclic garbage collection inside the timed regions: a collection
    # pass while the GPU waits for the next launch lands in the events of
    # that phase; garbage is collected between the legs instead
    gc.disable()
    for x in legs:
        log(f"== leg {x}")
        {"timestep": leg_timestep, "c1": leg_c1, "c2": leg_c2, "knn": leg_knn, "serving": leg_serving,
         "sweep": leg_sweep, "tables": leg_tables}[x](args, out)
        gc.collect()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
