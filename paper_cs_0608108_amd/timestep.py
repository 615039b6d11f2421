"""Moving-agent timesteps (dynamic objects, Section I of the paper).

One step = move every agent (seeded counter-hash displacement, read from a
device step counter) -> rebuild the lattice -> all-agents radius query
(count pass, scan, write pass) -> checksum of the per-row counts.  With
`resident=True` the first two are one incremental update instead: the
lattice's own sorted records are moved and the lattice is rebuilt from them,
and the by-id positions are written only when asked for.  Every
call is a stream-ordered kernel launch with no host synchronisation, no
device allocation and no memset, so the whole step is captured once as a
HIP graph and replayed.  The output buffers are sized once from the first
step's count with headroom; a step whose pairs exceed them sets the
capacity flag (checked with `status()`), and `step()` can redo it eagerly
with larger buffers.
"""
from __future__ import annotations

import torch

from . import sphidx


class AgentSim:
    def __init__(self, log2_cells, frac_bits, cyclic_mask, pts, r_fx, seed, subcell_bits=2, headroom=1.25,
                 launch: sphidx.LaunchConfig | None = None, flags=0, cell_list=False, resident=False):
        self.n = len(pts[0])
        self.desc = sphidx.desc_of(log2_cells, frac_bits, cyclic_mask)
        self.lat = sphidx.Lattice(log2_cells, frac_bits, cyclic_mask, self.n)
        self.pos = [sphidx.to_dev_u32(a) for a in pts]
        self.seed = int(seed)
        self.r_fx = int(r_fx)
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
        # moved records of the incremental update (16 bytes per agent)
        self.scratch = torch.empty(4 * self.n if resident else 0, dtype=torch.int32, device="cuda")
        self.graph = None
        self.steps_done = 0

    def _step_kernels(self):
        if self.resident:
            sphidx.move_resident(self.lat, self.seed, self.scratch, step_dev=self.step_dev)
        else:
            sphidx.move_agents_counted(self.desc, self.seed, self.step_dev, *self.pos)
            self.lat.build(*self.pos)
        sphidx.count(self.lat, self.tab, self.q, self.buf, self.launch)
        sphidx.write(self.lat, self.tab, self.q, self.buf, self.launch)
        sphidx.count_checksum(self.buf.row_ptr, self.n, self.chk)

    def step(self):
        """One step launched eagerly."""
        self._step_kernels()
        self.steps_done += 1

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
        if self.resident:
            sphidx.lattice_positions(self.lat, *self.pos)
        return tuple(sphidx.to_host_u32(p) for p in self.pos)

    def csr(self):
        return self.buf.host()
