"""Moving-agent timesteps on the GPU: eager steps and HIP-graph replays
against the oracle's movement replay and grid radius query, bit for bit.

Each step moves every agent with the counter-hash displacement, rebuilds the
lattice and answers the all-agents radius query.  The checksum of per-row
counts is compared at every step, positions at every step, and the whole
CSR at sampled steps.  Between graph replays the program does unrelated
eager device work and synchronises, as a simulation loop would."""
import numpy as np
import pytest

from gpu_util import assert_same, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_cs_0608108_amd import sphidx
    sphidx.load()
    return sphidx


@pytest.mark.parametrize("mask,log2,n,seed,launch", [
    (7, (5, 5, 5), 32768, 11, {}),
    (5, (5, 4, 6), 20000, 12, {}),
    (7, (5, 5, 5), 32768, 13, {"sort_cap": 128, "table_in_lds": 1}),
    (5, (5, 4, 6), 20000, 14, {"grouped": 1, "waves_per_block": 2}),
    # the non-empty cell list, rebuilt inside the captured step: chosen by
    # volume at 150 agents in 32^3 cells, or forced for every query
    (7, (5, 5, 5), 150, 15, {"method": 2, "cell_list": True}),
    (5, (5, 4, 6), 3000, 16, {"method": 3, "cell_list": True}),
    # incremental maintenance: the lattice's own records are moved and the
    # lattice rebuilt from them (by-id positions only when read)
    (7, (5, 5, 5), 32768, 17, {"resident": True}),
    (5, (5, 4, 6), 20000, 18, {"resident": True, "grouped": 1, "waves_per_block": 2}),
])
def test_timestep_graph_replays_match_oracle(sx, orc, mask, log2, n, seed, launch):
    import torch

    from paper_cs_0608108_amd import synth, timestep
    F = 16
    spec = synth.LatticeSpec(log2, F, mask)
    pts = synth.uniform_points(spec, n, seed)
    r = 3 * (1 << F)
    say(f"timestep mask={mask} log2={log2} n={n} seed={seed} launch={launch}")
    launch = dict(launch)
    cell_list = launch.pop("cell_list", False)
    resident = launch.pop("resident", False)
    sim = timestep.AgentSim(log2, F, mask, pts, r, seed, launch=sx.LaunchConfig(**launch), cell_list=cell_list,
                            resident=resident)
    L = orc.Lattice(log2, F, mask)
    cur = tuple(np.asarray(a, dtype=np.uint32) for a in pts)

    def check(step, full):
        nonlocal cur
        cur = orc.move(L, seed, step, cur)
        got = sim.positions()
        for a in range(3):
            assert np.array_equal(got[a], cur[a]), f"positions axis {a} after step {step}"
        g = orc.Grid(L, cur)
        ref = g.radius(r)
        g.close()
        assert sim.checksum() == orc.count_checksum(ref.row_ptr), f"checksum after step {step}"
        if full:
            rp, ids, _ = sim.csr()
            assert_same((rp, ids, None), ref, f"CSR after step {step}")
        code, flags = sim.status()
        assert code == sx.OK and flags == 0, (step, code, flags)

    step = 0
    for _ in range(2):  # eager
        sim.step()
        torch.cuda.synchronize()
        check(step, full=True)
        step += 1
    sim.capture()
    junk = torch.arange(1 << 16, device="cuda")
    for i in range(6):  # replays with eager work between them
        sim.replay()
        torch.cuda.synchronize()
        check(step, full=i in (0, 5))
        step += 1
        junk = (junk * 3 + 1) % 1000003
        torch.cuda.synchronize()
    sim.step()  # eager again after the graph: same counter, same buffers
    torch.cuda.synchronize()
    check(step, full=True)
    assert sim.steps_done == step + 1


def _cells_sorted(h):
    """(cell, id) order of a lattice's records with their coordinates: the
    order inside a cell is the build's own, so compare cell by cell."""
    cs = h["cell_start"]
    pos = np.arange(len(h["ids"]))
    cell = np.searchsorted(cs, pos, side="right") - 1
    o = np.lexsort((h["ids"], cell))
    return cell[o], h["ids"][o], h["xs"][o], h["ys"][o], h["zs"][o]


@pytest.mark.parametrize("mask", [7, 0, 5])
def test_resident_move_equals_move_then_build(sx, mask):
    """Incremental maintenance (Section I): moving the lattice's records and
    rebuilding from them gives the cell starts, cell contents and positions
    of moving the by-id arrays and building again, step after step; objects
    outside a clipped region and unusable coordinates included."""
    import torch

    from gpu_util import tiny_points
    rng = np.random.default_rng(170 + mask)
    log2, F, seed = (5, 4, 5), 10, 23
    pts = tiny_points(rng, log2, F, mask, 6000, outside=(mask != 7), invalid=(mask == 0))
    n = len(pts[0])
    desc = sx.desc_of(log2, F, mask)
    dev_a = [sx.to_dev_u32(a) for a in pts]
    dev_b = [sx.to_dev_u32(a) for a in pts]
    lat_a = sx.Lattice(log2, F, mask, n)
    lat_b = sx.Lattice(log2, F, mask, n)
    lat_a.build(*dev_a)
    lat_b.build(*dev_b)
    step_a = torch.zeros(1, dtype=torch.int32, device="cuda")
    step_b = torch.zeros(1, dtype=torch.int32, device="cuda")
    scratch = torch.empty(4 * n, dtype=torch.int32, device="cuda")
    out = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(3)]
    for step in range(4):
        say(f"resident mask={mask} step={step}")
        if step < 3:
            sx.move_agents_counted(desc, seed, step_a, *dev_a)
            sx.move_resident(lat_b, seed, scratch, step_dev=step_b)
        else:  # the host-step form
            sx.move_agents(desc, seed, 40, *dev_a)
            sx.move_resident(lat_b, seed, scratch, step=40)
        lat_a.build(*dev_a)
        ha, hb = lat_a.host_arrays(), lat_b.host_arrays()
        assert np.array_equal(ha["cell_start"], hb["cell_start"]), step
        for u, v in zip(_cells_sorted(ha), _cells_sorted(hb)):
            assert np.array_equal(u, v), step
        sx.lattice_positions(lat_b, *out)
        for a in range(3):
            assert np.array_equal(sx.to_host_u32(out[a]), sx.to_host_u32(dev_a[a])), (step, a)
    assert int(step_b.item()) == 3
    # scratch smaller than 16 bytes per object, or misaligned
    with pytest.raises(sx.SphidxError):
        sx.move_resident(lat_b, seed, scratch[: 4 * n - 1])
    with pytest.raises(sx.SphidxError):
        sx.move_resident(lat_b, seed, scratch[1:])


@pytest.mark.parametrize("mask", [7, 0, 5])
def test_incremental_move_equals_move_then_build(sx, mask):
    """Incremental maintenance restricted to the objects that change cell:
    cell starts, cell contents and positions equal those of moving the by-id
    arrays and building again, step after step (objects outside a clipped
    region and unusable coordinates included); inside every cell the objects
    that stayed keep their previous order and come first."""
    import torch

    from gpu_util import tiny_points
    rng = np.random.default_rng(190 + mask)
    log2, F, seed = (5, 4, 5), 10, 29
    pts = tiny_points(rng, log2, F, mask, 6000, outside=(mask != 7), invalid=(mask == 0))
    n = len(pts[0])
    desc = sx.desc_of(log2, F, mask)
    dev_a = [sx.to_dev_u32(a) for a in pts]
    dev_b = [sx.to_dev_u32(a) for a in pts]
    lat_a = sx.Lattice(log2, F, mask, n)
    lat_b = sx.Lattice(log2, F, mask, n)
    lat_a.build(*dev_a)
    lat_b.build(*dev_b)
    step_a = torch.zeros(1, dtype=torch.int32, device="cuda")
    step_b = torch.zeros(1, dtype=torch.int32, device="cuda")
    scratch = torch.empty(sx.move_incremental_scratch_bytes(lat_b) // 4 + 1, dtype=torch.int32, device="cuda")
    out = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(3)]
    for step in range(5):
        say(f"incremental mask={mask} step={step}")
        before = lat_b.host_arrays()
        if step < 4:
            sx.move_agents_counted(desc, seed, step_a, *dev_a)
            sx.move_incremental(lat_b, seed, scratch, step_dev=step_b)
        else:  # the host-step form
            sx.move_agents(desc, seed, 40, *dev_a)
            sx.move_incremental(lat_b, seed, scratch, step=40)
        lat_a.build(*dev_a)
        ha, hb = lat_a.host_arrays(), lat_b.host_arrays()
        assert np.array_equal(ha["cell_start"], hb["cell_start"]), step
        for u, v in zip(_cells_sorted(ha), _cells_sorted(hb)):
            assert np.array_equal(u, v), step
        sx.lattice_positions(lat_b, *out)
        for a in range(3):
            assert np.array_equal(sx.to_host_u32(out[a]), sx.to_host_u32(dev_a[a])), (step, a)
        # stayers first, in their previous order
        cs0, cs1 = before["cell_start"], hb["cell_start"]
        ncell = len(cs1) - 1
        old_cell = np.empty(n, np.int64)
        old_rank = np.empty(n, np.int64)
        pos = np.arange(n)
        oc = np.searchsorted(cs0, pos, side="right") - 1
        old_cell[before["ids"]] = oc
        old_rank[before["ids"]] = pos
        nc = np.searchsorted(cs1, pos, side="right") - 1
        ids1 = hb["ids"]
        stay = old_cell[ids1] == nc
        for c in np.unique(nc[stay])[:200]:
            sel = np.nonzero(nc == c)[0]
            st = stay[sel]
            k = int(st.sum())
            assert st[:k].all(), (step, c)
            assert np.all(np.diff(old_rank[ids1[sel[:k]]]) > 0), (step, c)
        assert ncell > 0
    assert int(step_b.item()) == 4
    with pytest.raises(sx.SphidxError):
        sx.move_incremental(lat_b, seed, scratch[:16])


def test_resident_move_on_an_empty_lattice(sx):
    import torch
    lat = sx.Lattice((4, 4, 4), 8, 7, 16)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    lat.build(e, e, e)
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    sx.move_resident(lat, 5, e, step_dev=step)
    sx.lattice_positions(lat, e, e, e)
    inc = torch.empty(sx.move_incremental_scratch_bytes(lat) // 4 + 1, dtype=torch.int32, device="cuda")
    sx.move_incremental(lat, 5, inc, step_dev=step)
    h = lat.host_arrays()
    assert len(h["ids"]) == 0 and (h["cell_start"] == 0).all()
    assert int(step.item()) == 2
    code, flags = lat.status()
    assert code == sx.OK and flags == 0


def test_capacity_overflow_grows_the_buffers_and_redoes_the_query(sx, orc):
    """Output buffers sized below the first step's pairs: the step sets the
    capacity flag and writes no ids; ensure_capacity() grows the buffers,
    runs the step's query again without moving the agents a second time and
    captures the graph again, and the rows then equal the oracle's."""
    import torch

    from paper_cs_0608108_amd import synth, timestep
    spec = synth.LatticeSpec((5, 5, 5), 16, 7)
    n, seed, r = 20000, 23, 2 << 16
    pts = synth.uniform_points(spec, n, seed)
    sim = timestep.AgentSim(spec.log2_cells, spec.frac_bits, spec.cyclic_mask, pts, r, seed, headroom=0.5)
    L = orc.Lattice(spec.log2_cells, spec.frac_bits, spec.cyclic_mask)
    sim.step()
    grew, flags = sim.ensure_capacity()
    assert grew and flags & sx.FLAG_CAPACITY
    assert sim.ensure_capacity() == (False, 0)
    cur = pts
    for t in range(sim.steps_done):
        cur = orc.move(L, seed, t, cur)
    ref = orc.Grid(L, cur).radius(r)
    rp, ids, _ = sim.csr()
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ids, ref.ids), "after the eager step"
    sim.capture()
    for _ in range(3):
        sim.replay()
        sim.ensure_capacity()
    torch.cuda.synchronize()
    cur = pts
    for t in range(sim.steps_done):
        cur = orc.move(L, seed, t, cur)
    ref = orc.Grid(L, cur).radius(r)
    rp, ids, _ = sim.csr()
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(ids, ref.ids), "after the replays"
    assert sim.checksum() == orc.count_checksum(ref.row_ptr)


@pytest.mark.parametrize("resident", [False, True, "incremental"])
def test_full_size_timestep_in_the_benchmark_launch(sx, orc, resident):
    """The moving-agent workload at full size (8,388,608 agents in a cyclic
    256^3 lattice, r = 3 cells) in the launch the benchmark times (groups of
    queries, rows kept in the count pass): one eager step and three graph
    replays, then every position, the neighbour-count checksum over all
    8,388,608 rows and 20,000 sampled rows against the oracle's replay; with
    `resident` the records are moved in place instead of the lattice being
    rebuilt from positions."""
    import torch

    from paper_cs_0608108_amd import synth, timestep
    w = synth.agents_timestep()
    n, seed, r = w.n, w.extra["seed"], int(w.r_fx[0])
    ln = sx.LaunchConfig(method=sx.METHOD_SPHERE, schedule=sx.SCHED_PERSISTENT, grouped=1, interior=1,
                         sort_cap=256, waves_per_block=4, tile=64, blocks_per_cu=8)
    sim = timestep.AgentSim(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, w.pts, r, seed, launch=ln,
                            resident=resident is True, incremental=resident == "incremental")
    say(f"8,388,608-agent timestep, full size, resident={resident}")
    sim.step()
    torch.cuda.synchronize()
    sim.capture()
    for _ in range(3):
        sim.replay()
        torch.cuda.synchronize()
    code, flags = sim.status()
    assert code == sx.OK and flags == 0
    L = orc.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask)
    cur = w.pts
    for t in range(sim.steps_done):
        cur = orc.move(L, seed, t, cur)
    got = sim.positions()
    for a in range(3):
        assert np.array_equal(got[a], cur[a]), f"axis {a} after {sim.steps_done} steps"
    rp = sim.buf.row_ptr.cpu().numpy()
    rows = np.unique(np.random.default_rng(41).integers(0, n, 20000))
    idx = np.concatenate([np.arange(rp[i], rp[i + 1]) for i in rows])
    ids = sim.buf.ids[torch.from_numpy(idx).to(sim.buf.ids.device)].cpu().numpy().view(np.uint32)
    g = orc.Grid(L, cur)
    ref = g.radius(r, queries=tuple(np.asarray(c)[rows] for c in cur))
    counts = g.radius_counts(r)
    g.close()
    orp = np.zeros(n + 1, np.int64)
    orp[1:] = np.cumsum(counts)
    assert sim.checksum() == orc.count_checksum(orp), "count checksum over all rows"
    assert np.array_equal(rp, orp), "every row length"
    srp = np.zeros(len(rows) + 1, np.int64)
    srp[1:] = np.cumsum(rp[rows + 1] - rp[rows])
    assert np.array_equal(srp, ref.row_ptr), "row lengths"
    assert np.array_equal(ids, ref.ids), "sampled rows"
    if resident is True:
        # the benchmark's headline path: every row in full (about 483 M
        # ids), against the oracle's rows of all agents at this step
        del ids, idx
        say("every row of the 8,388,608-agent step against the oracle")
        g = orc.Grid(L, cur)
        full = g.radius(r)
        g.close()
        assert np.array_equal(full.row_ptr, rp), "every row length (full oracle)"
        all_ids = sim.buf.ids[: int(rp[-1])].cpu().numpy().view(np.uint32)
        first_bad = np.flatnonzero(all_ids != full.ids)
        assert first_bad.size == 0, f"{first_bad.size} ids differ, first at pair {first_bad[:1]}"
        say("every row identical:", int(rp[-1]), "pairs")
