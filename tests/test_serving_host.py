"""Serving loop host logic (no GPU): the output pool allocator and the
slot/memory admission, driven by a simulated executor on a simulated clock.

Invariants checked: never more batches in flight than slots, never more
pool bytes reserved than the pool holds, live reservations never overlap,
every batch completes exactly once, a batch is written only after its count
finished, write admission is first-come-first-served, and a batch whose
output alone exceeds the pool is rejected instead of blocking the loop."""
import numpy as np
import pytest

from paper_cs_0608108_amd import serving, synth


def test_pool_first_fit_and_coalescing():
    p = serving.MemoryPool(4096)
    a = p.alloc(1)
    b = p.alloc(300)
    c = p.alloc(1000)
    assert a == (0, 256) and b == (256, 512) and c == (768, 1024)
    assert p.used == 1792 and p.alloc(4096) is None
    p.release(*b)
    assert p.alloc(600) == (1792, 768)       # the 512-byte hole is too small
    assert p.alloc(500) == (256, 512)        # first fit takes the hole
    p.release(*a)
    p.release(256, 512)
    p.release(*c)
    p.release(1792, 768)
    assert p.free == [(0, 4096)] and p.used == 0 and p.peak == 2560


def test_pool_random_alloc_release_never_overlaps():
    rng = np.random.default_rng(3)
    p = serving.MemoryPool(1 << 20)
    live = []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            p.release(*live.pop(int(rng.integers(len(live)))))
        else:
            r = p.alloc(int(rng.integers(1, 40000)))
            if r is not None:
                live.append(r)
        spans = sorted(live)
        for (o1, n1), (o2, _) in zip(spans, spans[1:]):
            assert o1 + n1 <= o2
        assert all(o % serving.ALIGN == 0 and o + n <= p.size for o, n in live)
        assert p.used == sum(n for _, n in live)
        assert p.used + sum(n for _, n in p.free) == p.size


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def tick(self):
        self.t += 1e-4


class FakeExecutor:
    """Count takes 2 us per query, write 3 us per query; pairs = 37 per query."""

    def __init__(self, clock, slots, pool):
        self.clock, self.slots, self.pool = clock, slots, pool
        self.live = {}
        self.in_flight = 0
        self.started, self.written = [], []

    def output_bytes(self, pairs):
        return 4 * max(pairs, 1)

    def start(self, b):
        self.in_flight += 1
        assert self.in_flight <= self.slots
        self.started.append(b.index)
        return dict(b=b, t_count=self.clock() + 2e-6 * b.size, t_write=None)

    def counted(self, tok):
        return 37 * tok["b"].size if self.clock() >= tok["t_count"] else None

    def write(self, tok, res):
        assert self.clock() >= tok["t_count"]
        off, n = res
        assert n >= self.output_bytes(37 * tok["b"].size) and off + n <= self.pool
        for o2, n2 in self.live.values():
            assert off + n <= o2 or o2 + n2 <= off, "overlapping reservations"
        self.live[tok["b"].index] = res
        self.max_live = max(getattr(self, "max_live", 0), len(self.live))
        self.written.append(tok["b"].index)
        tok["t_write"] = self.clock() + 3e-6 * tok["b"].size

    def done(self, tok):
        return self.clock() >= tok["t_write"]

    def collect(self, tok):
        return tok["b"].index

    def release(self, tok):
        self.live.pop(tok["b"].index, None)
        self.in_flight -= 1


def _batches(count, seed, rate, max_size=4096):
    sizes = synth.serving_batch_sizes(seed, count, max_size)
    gaps = synth.serving_interarrivals(seed, count, rate)
    t = np.cumsum(gaps)
    out = []
    for i in range(count):
        n = int(sizes[i])
        out.append(serving.Batch(i, float(t[i]), (np.zeros(n, np.uint32),) * 3, np.ones(n, np.uint32),
                                 np.zeros(n, np.uint32)))
    return out


@pytest.mark.parametrize("slots,pool,rate", [(1, 1 << 22, 500.0), (3, 1 << 20, 2000.0), (8, 600_000, 5000.0)])
def test_admission_invariants(slots, pool, rate):
    clock = FakeClock()
    bs = _batches(120, 9, rate)
    ex = FakeExecutor(clock, slots, pool)
    adm = serving.run_admission_model(bs, ex, slots, pool, keep=True, clock=clock, poll=clock.tick)
    assert adm.in_flight == 0 and adm.pool.used == 0 and adm.pool.peak <= pool
    assert ex.in_flight == 0 and not ex.live
    order = sorted(range(len(bs)), key=lambda i: bs[i].arrival)
    assert ex.started == order                       # admitted in arrival order
    for b in bs:
        if b.rejected:
            assert 4 * 37 * b.size > pool and b.result is None
        else:
            assert b.result == b.index and b.pairs == 37 * b.size
            assert b.arrival <= b.t_start <= b.t_done
    assert len(ex.written) == len(set(ex.written)) == sum(not b.rejected for b in bs)
    st = serving.latency_stats([b for b in bs if not b.rejected])
    assert 0 < st["p50_ms"] <= st["p99_ms"]


def test_oversized_batch_is_rejected_not_blocking():
    clock = FakeClock()
    bs = _batches(10, 4, 1000.0)
    big = bs[3]
    pool = 4 * 37 * big.size - 1 if big.size > 1 else 100
    for b in bs:  # everything but the big one fits
        if b is not big and 4 * 37 * b.size > pool:
            b.radius = b.radius[:1]
            b.centres = (b.centres[0][:1],) * 3
            b.k = b.k[:1]
    ex = FakeExecutor(clock, 2, pool)
    serving.run_admission_model(bs, ex, 2, pool, keep=True, clock=clock, poll=clock.tick)
    assert big.rejected
    assert all(not b.rejected and b.result == b.index for b in bs if b is not big)


def test_memory_admission_serialises_when_pool_is_tight():
    """With room for one batch's output only, writes never overlap in time."""
    clock = FakeClock()
    bs = _batches(30, 5, 1e6, max_size=64)
    for b in bs:  # equal sizes, all arrive at once
        b.radius = np.ones(64, np.uint32)
        b.centres = (np.zeros(64, np.uint32),) * 3
        b.k = np.zeros(64, np.uint32)
    pool = 4 * 37 * 64 + 200
    ex = FakeExecutor(clock, 4, pool)
    serving.run_admission_model(bs, ex, 4, pool, keep=True, clock=clock, poll=clock.tick)
    assert ex.max_live == 1
    assert all(not b.rejected and b.result == b.index for b in bs)
