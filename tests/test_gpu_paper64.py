"""The paper's own table design on the device (METHOD_PAPER64: per-cell
entries sorted by b^2, the 64 tables specialised on the six flags
[frac(d) < zeta], the run-time test of Eq. 1 from d - 1 on) against the
oracle, bit for bit, and its cells walked and kept against the host census
of the same design."""
import numpy as np
import pytest

from gpu_util import assert_same, lattice, run, say, tiny_points

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_cs_0608108_amd import sphidx
    sphidx.load()
    return sphidx


def _paper(sx, **kw):
    return sx.LaunchConfig(method=sx.METHOD_PAPER64, **kw)


@pytest.mark.parametrize("mask", [7, 0, 3, 5])
def test_paper_tables_radius_and_knn_match_oracle(sx, orc, mask):
    rng = np.random.default_rng(300 + mask)
    log2, F = (4, 5, 4), 10
    pts = tiny_points(rng, log2, F, mask, 20000, outside=(mask != 7))
    lat = lattice(sx, log2, F, mask, pts, cell_list=False)
    E = 1 << F
    tab = sx.Tables(lat, 2, 3 * E)  # larger radii take the cube scan
    L = orc.Lattice(log2, F, mask)
    g = orc.Grid(L, pts)
    r = rng.integers(0, 4 * E, size=len(pts[0])).astype(np.uint32)
    r[:50] = 0
    r[50:100] = E
    ref = g.radius(r)
    for launch, stash in ((_paper(sx), False), (_paper(sx), True), (_paper(sx, schedule=sx.SCHED_PLAIN), False),
                          (_paper(sx, grouped=1), True)):
        say(f"paper64 radius mask={mask} schedule={launch.schedule} stash={stash}")
        assert_same(run(sx, lat, tab, r, launch=launch, stash=stash), ref, f"paper64 radius mask {mask}")
    # explicit centres, K nearest and a mixed batch
    W = [(1 << (log2[a] + F)) for a in range(3)]
    Qn = 4000
    cen = tuple(rng.integers(0, W[a] + (0 if (mask >> a) & 1 else W[a] // 8), size=Qn).astype(np.uint32)
                for a in range(3))
    k = rng.integers(1, 40, size=Qn).astype(np.uint32)
    cap = rng.integers(0, 4 * E, size=Qn).astype(np.uint32)
    refk = g.knn(k, cap, queries=cen)
    kk = np.where(rng.random(Qn) < 0.5, k, 0).astype(np.uint32)
    refm = g.mixed(kk, cap, queries=cen)
    g.close()
    for stash in (False, True):
        say(f"paper64 knn/mixed mask={mask} stash={stash}")
        assert_same(run(sx, lat, tab, cap, k=k, mode=sx.MODE_KNN, queries=cen, launch=_paper(sx), stash=stash),
                    refk, f"paper64 knn mask {mask}")
        assert_same(run(sx, lat, tab, cap, k=kk, mode=sx.MODE_MIXED, queries=cen, launch=_paper(sx), stash=stash),
                    refm, f"paper64 mixed mask {mask}")
    code, flags = lat.status()
    assert code == sx.OK, (code, flags)


def test_paper_tables_cells_match_the_host_census(sx, orc):
    """Cells walked (entries of the unshaved and specialised tables) and kept
    (after the Eq. 1 test) per query, from the count pass's statistics, equal
    the host census of the same design; kept covers the exact set."""
    import torch
    rng = np.random.default_rng(31)
    log2, F, mask = (5, 5, 5), 12, 7
    E = 1 << F
    pts = tiny_points(rng, log2, F, mask, 3000)
    lat = lattice(sx, log2, F, mask, pts, cell_list=False)
    tab = sx.Tables(lat, 2, 6 * E)
    Qn = 3000
    W = 1 << (log2[0] + F)
    cen = tuple(rng.integers(0, W, size=Qn).astype(np.uint32) for _ in range(3))
    r = rng.integers(0, 6 * E, size=Qn).astype(np.uint32)
    r[:20] = 0
    r[20:40] = rng.integers(0, 4, 20) * E  # whole cells: frac(d) = 0
    keep = (tuple(sx.to_dev_u32(c) for c in cen), sx.to_dev_u32(r))
    q = sx.make_queries(Qn, keep[0], keep[1])
    st = torch.zeros(4 * Qn, dtype=torch.int32, device="cuda")
    buf = sx.QueryBuffers(Qn, 0)
    sx.count(lat, tab, q, buf, _paper(sx, stats=st))
    torch.cuda.synchronize()
    s = st.cpu().numpy().view(np.uint32).reshape(Qn, 4)
    f = [c & (E - 1) for c in cen]
    cen_ = sx.table_census(tab, f, r)
    np.testing.assert_array_equal(s[:, 0], cen_["paper64"])
    np.testing.assert_array_equal(s[:, 1], cen_["paper64_eq1"])
    assert (cen_["dropped"] == 0).all()
    kept, _, _ = orc.cells_touched(orc.Lattice(log2, F, mask), cen, r)
    assert (s[:, 1] >= kept).all()
    say("paper64 mean walked/kept/exact", s[:, 0].mean(), s[:, 1].mean(), kept.mean())
    del keep


def test_paper_tables_need_a_cap_within_their_limit(sx):
    lat = sx.Lattice((6, 6, 6), 8, 7, 16)
    tab = sx.Tables(lat, 1, 40 << 8)  # offsets beyond the paper tables' 32 cells
    q = sx.make_queries(0, None, 1 << 8)
    buf = sx.QueryBuffers(0, 0)
    with pytest.raises(sx.SphidxError) as ei:
        sx.count(lat, tab, q, buf, _paper(sx))
    assert ei.value.code == sx.ERR_RADIUS
