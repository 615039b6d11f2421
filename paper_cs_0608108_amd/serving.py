"""Serving loop: query batches against a device-resident lattice.

Batches arrive over time (for instance a Poisson stream).  The server keeps
up to `slots` batches in flight, each on its own HIP stream (default
priority), so their kernels overlap on the device:

    admit   a slot is free -> copy the batch's centres, radii and K to the
            device and run the count pass (row sizes + scan)
    size    when the count is done, the exact output size is known; the
            batch is admitted to the write pass only when that many bytes
            fit in the output pool (admission by memory), else it waits
    write   run the write pass into its reserved pool range
    done    record the latency (completion - arrival), release the slot and
            the pool range (after handing the result to the caller)

The loop runs in the library (sphidx_server_*, driven here by
`run_on_server`); with one slot and the plain schedule the same loop is one
launch per batch: count, size, write, then the next batch.
`run_admission_model` is the same policy in Python over an abstract
executor, so the policy's invariants (slots, first-fit pool, arrival-order
admission, rejection) are tested without a device.  `one_launch_per_batch`
runs each batch alone through the plain query calls (a check of the
server's rows).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass

import numpy as np

ALIGN = 256


class MemoryPool:
    """First-fit allocator over [0, size) with coalescing free list."""

    def __init__(self, size: int):
        self.size = int(size)
        self.free = [(0, self.size)]  # sorted (offset, length)
        self.used = 0
        self.peak = 0

    def alloc(self, nbytes: int):
        n = max(ALIGN, (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN)
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, ln - n)
                self.used += n
                self.peak = max(self.peak, self.used)
                return off, n
        return None

    def release(self, off: int, n: int):
        self.used -= n
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged


class Admission:
    """Slot and memory admission (host logic)."""

    def __init__(self, slots: int, pool_bytes: int):
        self.slots = int(slots)
        self.in_flight = 0
        self.pool = MemoryPool(pool_bytes)

    def can_start(self):
        return self.in_flight < self.slots

    def start(self):
        assert self.can_start()
        self.in_flight += 1

    def reserve(self, nbytes):
        return self.pool.alloc(nbytes)

    def finish(self, reservation):
        if reservation is not None:
            self.pool.release(*reservation)
        self.in_flight -= 1


@dataclass
class Batch:
    index: int
    arrival: float                # seconds after the run starts
    centres: tuple                # host uint32 arrays
    radius: np.ndarray            # host uint32 (K-NN rows: the search cap)
    k: np.ndarray                 # host uint32 (0 = radius query)
    t_start: float = 0.0
    t_done: float = 0.0
    pairs: int = 0
    rejected: bool = False        # its output alone exceeds the whole pool
    result: tuple | None = None   # (row_ptr, ids) when kept

    @property
    def size(self):
        return len(self.radius)


def run_admission_model(batches, executor, slots, pool_bytes, keep=False, clock=time.perf_counter, poll=None):
    """Drive `executor` (GPU or fake) through the batches in arrival order.

    Executor interface: start(batch) -> token (launches the count pass);
    counted(token) -> exact pair total, or None while the count runs;
    output_bytes(pairs) -> bytes the write pass needs; write(token,
    (offset, bytes)) launches the write pass into that pool range;
    done(token) -> bool; collect(token) -> result; release(token) frees the
    slot.  A batch whose output alone exceeds the pool is marked rejected
    (the caller splits it).  Returns the Admission object (pool statistics)."""
    adm = Admission(slots, pool_bytes)
    order = sorted(batches, key=lambda b: b.arrival)
    pending = collections.deque(order)
    counting, waiting, writing = [], collections.deque(), []
    t0 = clock()
    remaining = len(order)
    while remaining:
        now = clock() - t0
        progressed = False
        while pending and pending[0].arrival <= now and adm.can_start():
            b = pending.popleft()
            adm.start()
            b.t_start = now
            counting.append((b, executor.start(b)))
            progressed = True
        still = []
        for b, tok in counting:
            tot = executor.counted(tok)
            if tot is None:
                still.append((b, tok))
            else:
                b.pairs = tot
                waiting.append((b, tok))
                progressed = True
        counting = still
        while waiting:
            b, tok = waiting[0]
            need = executor.output_bytes(b.pairs)
            if need > adm.pool.size:
                waiting.popleft()
                b.rejected = True
                b.t_done = clock() - t0
                executor.release(tok)
                adm.finish(None)
                remaining -= 1
                progressed = True
                continue
            res = adm.reserve(need)
            if res is None:
                break
            waiting.popleft()
            executor.write(tok, res)
            writing.append((b, tok, res))
            progressed = True
        still = []
        for b, tok, res in writing:
            if executor.done(tok):
                b.t_done = clock() - t0
                if keep:
                    b.result = executor.collect(tok)
                executor.release(tok)
                adm.finish(res)
                remaining -= 1
                progressed = True
            else:
                still.append((b, tok, res))
        writing = still
        if not progressed and poll:
            poll()
    return adm


def run_on_server(server, batches, keep=False):
    """Replay `batches` (Batch objects) on a library server (sphidx.Server):
    the loop above, in native code, on the GPU.  Fills each batch's start
    and completion times, pairs and rejection (and result with keep).
    Returns the peak pool bytes reserved at once."""
    order = sorted(batches, key=lambda b: b.arrival)
    res, rows = server.run([b.arrival for b in order], [b.centres for b in order], [b.radius for b in order],
                           [b.k for b in order], keep=keep)
    for i, b in enumerate(order):
        b.t_start, b.t_done = float(res["start_s"][i]), float(res["done_s"][i])
        b.pairs, b.rejected = int(res["pairs"][i]), bool(res["rejected"][i])
        if keep:
            b.result = rows[i]
    return int(res["pool_in_use"].max()) if len(order) else 0


def one_launch_per_batch(batches, lat, tab, launch=None, keep=False):
    """Baseline: one stream, each batch counted, sized and written in turn."""
    from . import sphidx
    t0 = time.perf_counter()
    for b in sorted(batches, key=lambda x: x.arrival):
        while time.perf_counter() - t0 < b.arrival:
            pass
        b.t_start = time.perf_counter() - t0
        cen = tuple(sphidx.to_dev_u32(a) for a in b.centres)
        rad = sphidx.to_dev_u32(b.radius)
        kk = sphidx.to_dev_u32(b.k)
        q = sphidx.make_queries(b.size, cen, rad, kk, sphidx.MODE_MIXED)
        rp, ids, _ = sphidx.run(lat, tab, q, launch, want_dist2=False)
        b.t_done = time.perf_counter() - t0
        b.pairs = int(rp[-1])
        if keep:
            b.result = (rp, ids)


def latency_stats(batches):
    lat = np.array([b.t_done - b.arrival for b in batches])
    q = sum(b.size for b in batches)
    span = max(b.t_done for b in batches) - min(b.arrival for b in batches)
    return {"batches": len(batches), "queries": q, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "queries_per_s": q / span if span > 0 else None, "span_s": span}
