"""Moving-agent timesteps (dynamic objects, Section I of the paper).

One step = move every agent (seeded counter-hash displacement, read from a
device step counter) -> rebuild the lattice -> all-agents radius query
(count pass, scan, write pass) -> checksum of the per-row counts.  With
`resident=True` the first two are one incremental update instead: the
lattice's own sorted records are moved and the lattice is rebuilt from them,
and the by-id positions are written only when asked for; with
`incremental=True` only the agents that change cell are placed again by
atomics, the others keeping their order.  Every
call is a stream-ordered kernel launch with no host synchronisation, no
device allocation and no memset, so the whole step is captured once as a
HIP graph and replayed.  The output buffers are sized once from the first
step's count with headroom; a step whose pairs exceed them sets the
capacity flag and writes no ids.  `ensure_capacity()`, called after a step
or a replay, finds that flag, grows the buffers to the step's own count
(with the same headroom), runs that step's query again on the current
lattice (the agents are not moved twice) and captures the graph again.
"""
from __future__ import annotations

import dataclasses

import torch

from . import sphidx


class AgentSim:
    def __init__(self, log2_cells, frac_bits, cyclic_mask, pts, r_fx, seed, subcell_bits=2, headroom=1.25,
                 launch: sphidx.LaunchConfig | None = None, flags=0, cell_list=False, resident=False,
                 incremental=False):
        self.n = len(pts[0])
        self.desc = sphidx.desc_of(log2_cells, frac_bits, cyclic_mask)
        self.lat = sphidx.Lattice(log2_cells, frac_bits, cyclic_mask, self.n)
        self.pos = [sphidx.to_dev_u32(a) for a in pts]
        self.seed = int(seed)
        self.r_fx = int(r_fx)
        self.headroom = float(headroom)
        self.tab = sphidx.Tables(self.lat, subcell_bits, self.r_fx)
        self.launch = launch or sphidx.LaunchConfig()
        self.q = sphidx.make_queries(self.n, None, self.r_fx, None, sphidx.MODE_RADIUS, flags)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.chk = torch.zeros(2, dtype=torch.int64, device="cuda")
        if cell_list:  # rebuilt with the lattice, inside the captured step too
            self.lat.attach_cell_list()
        # size the outputs from the pairs at the starting positions
        self.lat.build(*self.pos)
        probe = sphidx.QueryBuffers(self.n, 0, want_dist2=False)
        sphidx.count(self.lat, self.tab, self.q, probe, self.launch)
        cap = int(int(probe.row_ptr[-1].item()) * headroom) + 1024
        # the stash lets the count pass keep the sorted rows: the write pass
        # then copies them instead of walking the tables a second time
        self.buf = sphidx.QueryBuffers(self.n, cap, want_dist2=False, stash_pairs=cap)
        self.resident = bool(resident)
        self.incremental = bool(incremental)
        # moved records of the update from records (16 bytes per agent), or
        # the incremental update's scratch
        nbytes = 16 * self.n if resident else sphidx.move_incremental_scratch_bytes(self.lat) if incremental else 0
        self.scratch = torch.empty((nbytes + 3) // 4, dtype=torch.int32, device="cuda")
        self.graph = None
        self.steps_done = 0

    def _query_kernels(self, count_launch=None):
        sphidx.count(self.lat, self.tab, self.q, self.buf, count_launch or self.launch)
        sphidx.write(self.lat, self.tab, self.q, self.buf, self.launch)
        sphidx.count_checksum(self.buf.row_ptr, self.n, self.chk)

    def _step_kernels(self, count_launch=None):
        if self.incremental:
            sphidx.move_incremental(self.lat, self.seed, self.scratch, step_dev=self.step_dev)
        elif self.resident:
            sphidx.move_resident(self.lat, self.seed, self.scratch, step_dev=self.step_dev)
        else:
            sphidx.move_agents_counted(self.desc, self.seed, self.step_dev, *self.pos)
            self.lat.build(*self.pos)
        self._query_kernels(count_launch)

    def step(self, count_events=None):
        """One step launched eagerly; count_events = (begin, end) torch events
        that the library records around the count kernel."""
        ln = dataclasses.replace(self.launch, events=count_events) if count_events else None
        self._step_kernels(ln)
        self.steps_done += 1

    def ensure_capacity(self):
        """Check the status word after a step or replay (synchronises).  When
        the step's pairs exceeded the output buffers, grow them to its count
        times the headroom, run its query again on the current lattice and
        capture the graph again.  Returns (grew, flags), the flags being
        those the step set."""
        code, flags = self.lat.status()
        if not flags & sphidx.FLAG_CAPACITY:
            return False, flags
        total = int(self.buf.row_ptr[-1].item())
        cap = max(total, int(total * self.headroom)) + 1024
        self.buf = None
        self.buf = sphidx.QueryBuffers(self.n, cap, want_dist2=False, stash_pairs=cap)
        self._query_kernels()
        torch.cuda.synchronize()
        if self.graph is not None:
            self.capture()
        return True, flags

    def capture(self):
        """Capture one step as a HIP graph (the capture itself runs nothing)."""
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._step_kernels()
        self.graph = g

    def replay(self):
        self.graph.replay()
        self.steps_done += 1

    def status(self):
        return self.lat.status()

    def checksum(self):
        c = self.chk.cpu().numpy().view("uint64")
        return int(c[0]), int(c[1])

    def positions(self):
        if self.resident or self.incremental:
            sphidx.lattice_positions(self.lat, *self.pos)
        return tuple(sphidx.to_host_u32(p) for p in self.pos)

    def csr(self):
        return self.buf.host()
