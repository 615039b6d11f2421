"""Section IV worlds on the GPU against the oracle: a 16^3 world at 10
objects per cell, wrapping and clipped, random centres, query distances from
a quarter cell to 3/4 of the world (past the half-world point where the
wrapping sphere walk hands over to the whole-world cube scan), all
neighbours and the nearest neighbour, with both methods, bit for bit."""
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


@pytest.mark.parametrize("mask", [7, 0])
def test_section_iv_world_matches_oracle(sx, orc, mask):
    from paper_cs_0608108_amd import synth
    w = synth.sweep_world(4, mask, 10.0)
    lat = sx.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, w.n)
    dev = [sx.to_dev_u32(a) for a in w.pts]
    lat.build(*dev)
    e = w.lat.edge
    tab = sx.Tables(lat, 2, 12 * e)
    cen = synth.sweep_centres(w.lat, 6, 256)
    cen_dev = tuple(sx.to_dev_u32(a) for a in cen)
    g = orc.Grid(orc.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask), w.pts)
    for rc in (0.25, 1.5, 7.5, 12.0):
        r = int(rc * e)
        ref_all = g.radius(r, queries=cen)
        ref_nn = g.knn(1, r, queries=cen)
        for name, ln in (("sphere", sx.LaunchConfig()), ("cube", sx.LaunchConfig(method=sx.METHOD_CUBE))):
            say(f"section IV mask={mask} r={rc} {name}")
            q = sx.make_queries(256, cen_dev, r, 0, sx.MODE_RADIUS, 0)
            assert_same(sx.run(lat, tab, q, ln, stash=True), ref_all, f"all r={rc} {name}")
            q = sx.make_queries(256, cen_dev, r, 1, sx.MODE_KNN, 0)
            assert_same(sx.run(lat, tab, q, ln), ref_nn, f"nearest r={rc} {name}")
    g.close()
    del cen_dev, dev
