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

`MemoryPool` and `Admission` are plain host logic (no GPU), so their
invariants are tested without a device.  `one_launch_per_batch` is the
baseline: one stream, each batch counted, sized and written before the next
one starts.
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


class GpuExecutor:
    """Runs batches on the device: one stream, workspace and input buffers per slot."""

    def __init__(self, lat, tab, slots, max_batch, pool_bytes, launch=None, stash_pairs=1 << 25):
        import torch

        from . import sphidx
        self.sx, self.torch = sphidx, torch
        self.lat, self.tab = lat, tab
        self.launch = launch or sphidx.LaunchConfig()
        self.pool = torch.empty(int(pool_bytes) + ALIGN, dtype=torch.uint8, device="cuda")
        self.pool_base = self.pool.data_ptr() + ((-self.pool.data_ptr()) % ALIGN)
        self.free_slots = list(range(slots))
        self.slot = []
        for _ in range(slots):
            s = dict(stream=torch.cuda.Stream(),
                     buf=sphidx.QueryBuffers(max_batch, 0, want_dist2=False, stash_pairs=stash_pairs),
                     inp=torch.empty((5, max_batch), dtype=torch.int32, device="cuda"),
                     host=torch.empty((5, max_batch), dtype=torch.int32, pin_memory=True),
                     total=torch.empty(1, dtype=torch.int64, pin_memory=True))
            self.slot.append(s)

    def output_bytes(self, pairs):
        return 4 * max(pairs, 1)

    def start(self, b):
        sx, torch = self.sx, self.torch
        si = self.free_slots.pop()
        s = self.slot[si]
        n = b.size
        h = s["host"].numpy().view(np.uint32)
        for a in range(3):
            h[a, :n] = b.centres[a]
        h[3, :n] = b.radius
        h[4, :n] = b.k
        with torch.cuda.stream(s["stream"]):
            s["inp"][:, :n].copy_(s["host"][:, :n], non_blocking=True)
            inp = s["inp"]
            q = sx.make_queries(n, (inp[0], inp[1], inp[2]), inp[3], inp[4], sx.MODE_MIXED)
            buf = s["buf"]
            cs = buf.c()
            cs.capacity = 0
            sx.check(sx.load().sphidx_count(self.lat.handle, self.tab.handle, sx.ctypes.byref(q),
                                            sx.ctypes.byref(cs), sx.ctypes.byref(self.launch.c()),
                                            sx._stream(s["stream"])), "count")
            s["total"].copy_(buf.row_ptr[n:n + 1], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s["stream"])
        return dict(si=si, q=q, n=n, ev=ev, done=None)

    def counted(self, tok):
        if not tok["ev"].query():
            return None
        return int(self.slot[tok["si"]]["total"][0])

    def write(self, tok, res):
        sx, torch = self.sx, self.torch
        s = self.slot[tok["si"]]
        off, nb = res
        cs = s["buf"].c()
        cs.ids_dev = self.pool_base + off
        cs.dist2_dev = None
        cs.capacity = nb // 4
        with torch.cuda.stream(s["stream"]):
            sx.check(sx.load().sphidx_write(self.lat.handle, self.tab.handle, sx.ctypes.byref(tok["q"]),
                                            sx.ctypes.byref(cs), sx.ctypes.byref(self.launch.c()),
                                            sx._stream(s["stream"])), "write")
            ev = torch.cuda.Event()
            ev.record(s["stream"])
        tok["done"] = ev
        tok["res"] = res

    def done(self, tok):
        return tok["done"].query()

    def collect(self, tok):
        s = self.slot[tok["si"]]
        n = tok["n"]
        rp = s["buf"].row_ptr[: n + 1].cpu().numpy()
        off, nb = tok["res"]
        tot = int(rp[-1])
        ids = self.pool[off + ((-self.pool.data_ptr()) % ALIGN):][: 4 * tot].view(self.torch.int32)
        return rp, ids.cpu().numpy().view(np.uint32)

    def release(self, tok):
        self.free_slots.append(tok["si"])


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
