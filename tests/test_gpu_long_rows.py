"""Long radius rows in the write pass: rows longer than the wavefront's LDS
row buffer taken by one block of 2, 4 or 8 waves (walked once, ordered by a
block-wide bucket sort), rows beyond the block's 3,072 pairs and K-NN rows
left to the windowed top-M kernel; bit for bit against the oracle, with
every walk (sphere tables, cube, per-query choice, the paper's tables)."""
import numpy as np
import pytest

from gpu_util import assert_same, lattice, run, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_cs_0608108_amd import sphidx
    sphidx.load()
    return sphidx


@pytest.mark.parametrize("mask", [7, 0])
def test_long_rows_by_block_match_oracle(sx, orc, mask):
    rng = np.random.default_rng(500 + mask)
    log2, F = (5, 5, 5), 10
    E = 1 << F
    W = 32 << F
    n = 60000  # about 1.8 objects per cell
    pts = tuple(rng.integers(0, W, n).astype(np.uint32) for _ in range(3))
    lat = lattice(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 8 * E)
    Qn = 3000
    cen = tuple(rng.integers(0, W, Qn).astype(np.uint32) for _ in range(3))
    # radii from short rows (sort_cap) to rows past the block's 3,072 pairs
    r = rng.integers(0, 8 * E, Qn).astype(np.uint32)
    r[:100] = 8 * E
    k = np.where(rng.random(Qn) < 0.2, rng.integers(65, 300, Qn), 0).astype(np.uint32)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    ref = g.radius(r, queries=cen)
    refm = g.mixed(k, r, queries=cen)
    g.close()
    lens = np.diff(ref.row_ptr)
    assert (lens > 256).sum() > 300 and (lens > 3072).sum() > 20
    for lw in (1, 2, 4, 8):
        for method in (sx.METHOD_SPHERE, sx.METHOD_CUBE, sx.METHOD_AUTO, sx.METHOD_PAPER64):
            for stash in (False, True):
                say(f"long rows mask={mask} waves={lw} method={method} stash={stash}")
                ln = sx.LaunchConfig(method=method, long_row_waves=lw)
                assert_same(run(sx, lat, tab, r, queries=cen, launch=ln, stash=stash), ref,
                            f"radius, waves {lw}, method {method}")
        ln = sx.LaunchConfig(long_row_waves=lw, sort_cap=128)
        assert_same(run(sx, lat, tab, r, k=k, mode=sx.MODE_MIXED, queries=cen, launch=ln), refm,
                    f"mixed, waves {lw}")
    code, flags = lat.status()
    assert code == sx.OK, (code, flags)
