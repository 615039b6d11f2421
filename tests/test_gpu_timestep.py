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
    sim = timestep.AgentSim(log2, F, mask, pts, r, seed, launch=sx.LaunchConfig(**launch), cell_list=cell_list)
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
