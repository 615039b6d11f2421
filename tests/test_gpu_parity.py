"""GPU parity: the HIP path through the C ABI against the oracle, bit for bit.

Every comparison is exact: row pointers, ids and squared distances are
integers.  Inputs are seeded and synthetic (uniform points, Gaussian
clusters, hand fixtures, degenerate layouts)."""
import numpy as np
import pytest

from goldens import read_hand, read_keyed
from gpu_util import assert_same, lattice, run, say, tiny_points

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_cs_0608108_amd import sphidx
    sphidx.load()
    return sphidx


def _launches(sx):
    L = sx.LaunchConfig
    return {
        "sphere-persistent": L(method=sx.METHOD_SPHERE, schedule=sx.SCHED_PERSISTENT),
        "sphere-grouped": L(method=sx.METHOD_SPHERE, schedule=sx.SCHED_PERSISTENT, grouped=1),
        # grouped with the wholly-inside shortcut off: dense small worlds
        # would otherwise take the one-query-per-wavefront count
        "sphere-grouped-flat": L(method=sx.METHOD_SPHERE, schedule=sx.SCHED_PERSISTENT, grouped=1, interior=1),
        "cube-grouped": L(method=sx.METHOD_CUBE, schedule=sx.SCHED_PERSISTENT, grouped=1),
        "sphere-plain": L(method=sx.METHOD_SPHERE, schedule=sx.SCHED_PLAIN),
        "sphere-small-cap": L(method=sx.METHOD_SPHERE, schedule=sx.SCHED_PERSISTENT, sort_cap=64, tile=1,
                              waves_per_block=2),
        "sphere-lds-table": L(method=sx.METHOD_SPHERE, schedule=sx.SCHED_PLAIN, table_in_lds=1,
                              waves_per_block=1, sort_cap=128),
        "cube": L(method=sx.METHOD_CUBE, schedule=sx.SCHED_PERSISTENT),
        "cube-plain": L(method=sx.METHOD_CUBE, schedule=sx.SCHED_PLAIN, tile=3),
        "auto": L(method=sx.METHOD_AUTO, schedule=sx.SCHED_PERSISTENT),
        "auto-grouped-weighted": L(method=sx.METHOD_AUTO, schedule=sx.SCHED_PERSISTENT, grouped=1,
                                   select_weight=384, reversal_fx=40),
        "list-plain": L(method=sx.METHOD_LIST, schedule=sx.SCHED_PLAIN, tile=2),
    }


# ---------------------------------------------------------------------------
# Lattice rebuild (counting sort)

@pytest.mark.parametrize("mask", [0, 5, 7])
def test_rebuild_is_the_oracle_counting_sort(sx, orc, mask):
    say("rebuild mask", mask)
    rng = np.random.default_rng(40 + mask)
    log2, F = (4, 3, 5), 10
    pts = tiny_points(rng, log2, F, mask, 20000, outside=True, invalid=True)
    lat = lattice(sx, log2, F, mask, pts)
    h = lat.host_arrays()
    cs = h["cell_start"]
    nc = lat.ncells
    grid = orc.Grid(orc.Lattice(log2, F, mask), pts)
    counts = grid.counts()
    np.testing.assert_array_equal(np.diff(cs[: nc + 2]), counts)
    # unusable objects (clipped coordinate >= 2^30) land in the last cell
    L = orc.Lattice(log2, F, mask)
    bad = np.zeros(len(pts[0]), bool)
    for a in range(3):
        if not (mask >> a) & 1:
            bad |= pts[a] >= (1 << 30)
    assert cs[nc + 2] - cs[nc + 1] == bad.sum() and cs[nc + 2] == len(pts[0])
    # the sorted arrays are a permutation of the input, normalised
    ids = h["ids"]
    assert np.array_equal(np.sort(ids), np.arange(len(pts[0])))
    for a, key in enumerate(("xs", "ys", "zs")):
        exp = pts[a][ids].astype(np.uint64)
        if (mask >> a) & 1:
            exp = exp % (((1 << log2[a]) << F))
        np.testing.assert_array_equal(h[key], exp.astype(np.uint32))
    # every object sits in the cell range of its own cell
    cellof = np.zeros(len(ids), np.int64)
    for k in range(nc + 2):
        cellof[cs[k]:cs[k + 1]] = k
    xs, ys, zs = h["xs"], h["ys"], h["zs"]
    inside = np.ones(len(ids), bool)
    for a, v in enumerate((xs, ys, zs)):
        if not (mask >> a) & 1:
            inside &= v < ((1 << log2[a]) << F)
    inside &= ~bad[ids]
    exp_cell = ((zs >> F).astype(np.int64) << (log2[0] + log2[1])) | ((ys >> F).astype(np.int64) << log2[0]) | (xs >> F)
    np.testing.assert_array_equal(cellof[inside], exp_cell[inside])
    assert (cellof[~inside & ~bad[ids]] == nc).all()
    code, flags = lat.status()
    if bad.any():
        assert flags & sx.FLAG_RANGE and code == sx.ERR_RANGE
    else:
        assert flags == 0 and code == sx.OK
    assert lat.status()[1] == 0  # cleared


def test_packed_index_and_outside_cell_follow_the_paper_example(sx):
    g = read_keyed("swar_example.txt")
    log2 = tuple(int(v) for v in g["lattice_log2"])
    F = 4
    c = [int(v) for v in g["center_cell"]]
    r = [int(v) for v in g["result_cell"]]
    e = 1 << F
    # one object in the centre cell, one in the translated cell, one outside
    pts = tuple(np.array([c[a] * e + 3, r[a] * e + 5, (1 << log2[a]) * e + 1 if a == 1 else 0],
                         dtype=np.uint32) for a in range(3))
    lat = lattice(sx, log2, F, 0, pts)
    cs = lat.host_arrays()["cell_start"]
    packed_c = int(g["packed_center"][0].replace("_", ""), 2)
    packed_r = int(g["packed_result"][0].replace("_", ""), 2)
    outside = int(g["outside_index"][0].replace("_", ""), 2)
    assert outside == lat.ncells
    occupied = set(np.nonzero(np.diff(cs))[0].tolist())
    assert occupied == {packed_c, packed_r, outside}
    # the translated cell (offset -5, +4, +3) is found from the centre cell
    off = [int(v) for v in g["offset_cells"]]
    d2 = sum(((r[a] * e + 5) - (c[a] * e + 3)) ** 2 for a in range(3))
    tab = sx.Tables(lat, 2, 8 * e)
    rp, ids, dd = run(sx, lat, tab, int(np.ceil(np.sqrt(d2))), queries=tuple(
        np.array([c[a] * e + 3], dtype=np.uint32) for a in range(3)))
    assert 1 in ids.tolist() and off == [r[a] - c[a] for a in range(3)]


# ---------------------------------------------------------------------------
# Hand fixtures (Section II.A definitions worked by hand)

@pytest.mark.parametrize("name", ["hand_cyclic.txt", "hand_clipped.txt"])
@pytest.mark.parametrize("launch", ["sphere-persistent", "sphere-plain", "cube", "sphere-grouped"])
def test_hand_fixtures(sx, name, launch):
    latd, pts, rows = read_hand(name)
    lat = lattice(sx, latd["log2_cells"], latd["frac_bits"], latd["cyclic_mask"], pts)
    tab = sx.Tables(lat, 1, 64)
    ln = _launches(sx)[launch]
    n = len(pts[0])
    for row in rows:
        r = np.full(n, row["r"], np.uint32)
        if row["kind"] == "radius":
            rp, ids, d2 = run(sx, lat, tab, r, flags=row["flags"], launch=ln)
        else:
            rp, ids, d2 = run(sx, lat, tab, r, k=row["k"], mode=sx.MODE_KNN, flags=row["flags"], launch=ln)
        i = row["q"]
        got = list(zip(d2[rp[i]:rp[i + 1]].tolist(), ids[rp[i]:rp[i + 1]].tolist()))
        assert got == row["exp"], (row, got)


# ---------------------------------------------------------------------------
# Radius queries on random worlds, every method and schedule

WORLDS = [((2, 2, 2), 4), ((3, 3, 3), 6), ((4, 3, 2), 8), ((5, 5, 5), 16), ((3, 4, 5), 2)]


@pytest.mark.parametrize("mask", [0, 3, 6, 7])
@pytest.mark.parametrize("world", WORLDS)
def test_radius_random_worlds(sx, orc, mask, world):
    log2, F = world
    say("radius world", log2, F, mask)
    rng = np.random.default_rng(hash((log2, F, mask)) % 2 ** 32)
    n = 1500
    pts = tiny_points(rng, log2, F, mask, n, outside=True, invalid=True)
    lat = lattice(sx, log2, F, mask, pts)
    e = 1 << F
    L = orc.Lattice(log2, F, mask)
    grid = orc.Grid(L, pts)
    rmax = int(2.5 * e)
    tabs = {s: sx.Tables(lat, s, rmax) for s in range(0, min(F, 3) + 1)}
    r = rng.integers(0, 3 * e, n).astype(np.uint32)  # some beyond the tables' cap -> cube fallback
    r[:20] = 0
    for flags in (0, 1):
        ref = grid.radius(r, flags=flags)
        for name, ln in _launches(sx).items():
            s = int(rng.integers(0, len(tabs)))
            if ln.table_in_lds and tabs[s].info().total_entries * 16 > 60000:
                continue
            assert_same(run(sx, lat, tabs[s], r, flags=flags, launch=ln), ref, f"{name} s={s} flags={flags}")
    # explicit centres, some outside the region / unusable on clipped axes
    qs = tiny_points(rng, log2, F, mask, 300, outside=True, invalid=True)
    rq = rng.integers(0, 3 * e, 300).astype(np.uint32)
    ref = grid.radius(rq, queries=qs)
    for name, ln in _launches(sx).items():
        if ln.table_in_lds:
            continue
        assert_same(run(sx, lat, tabs[min(2, len(tabs) - 1)], rq, queries=qs, launch=ln), ref, f"explicit {name}")


def test_radius_uniform_cyclic_32_full_vs_brute_force(sx, orc):
    from paper_cs_0608108_amd import synth
    w = synth.radius_uniform_cyclic()
    say("uniform cyclic 32^3, 4,096 points", w.name)
    L = orc.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask)
    ref = orc.radius_brute(L, w.pts, w.r_fx)
    lat = lattice(sx, w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, w.pts)
    for s in (0, 2):
        tab = sx.Tables(lat, s, int(w.r_fx[0]))
        for name, ln in _launches(sx).items():
            if ln.table_in_lds and tab.info().total_entries * 16 > 60000:
                continue
            assert_same(run(sx, lat, tab, w.r_fx, launch=ln), ref, f"uniform 4,096 points {name} s={s}")
        # uniform radius passed as a scalar
        assert_same(run(sx, lat, tab, int(w.r_fx[0])), ref, "uniform 4,096 points, scalar radius")


def test_tables_loaded_from_file_answer_queries(sx, orc, tmp_path):
    """Tables written to a file and read back (their row tables rebuilt at
    load) give the same rows as the oracle, with the table in device memory
    and staged in LDS, on a clipped and a cyclic world with uneven radii."""
    from paper_cs_0608108_amd import synth
    rng = np.random.default_rng(2029)
    for mask in (0, 7):
        lat_s = synth.LatticeSpec((4, 4, 4), 10, mask)
        pts = synth.uniform_points(lat_s, 3000, 71 + mask)
        r = rng.integers(lat_s.edge // 2, 3 * lat_s.edge, size=3000, dtype=np.uint32)
        say("loaded tables, mask", mask)
        L = orc.Lattice(lat_s.log2_cells, lat_s.frac_bits, mask)
        ref = orc.radius_brute(L, pts, r)
        lat = lattice(sx, lat_s.log2_cells, lat_s.frac_bits, mask, pts)
        path = tmp_path / f"tables_{mask}.bin"
        sx.Tables(lat, 1, int(2.5 * lat_s.edge)).save(path)  # radii above the cap fall back to the cube
        tab = sx.Tables.load_file(path)
        assert tab.info().total_entries * 16 <= 60000, "the LDS launch needs the whole table in LDS"
        for name in ("sphere-persistent", "sphere-grouped", "sphere-lds-table"):
            assert_same(run(sx, lat, tab, r, launch=_launches(sx)[name]), ref, f"loaded tables {name} mask {mask}")
        assert_same(run(sx, lat, tab, r, launch=_launches(sx)["sphere-grouped"], stash=True), ref,
                    f"loaded tables grouped stash mask {mask}")


def test_radius_uneven_clipped_full_size(sx, orc):
    from paper_cs_0608108_amd import synth
    w = synth.radius_uneven_clipped()
    say("uneven radius, 1,048,576 points", w.name)
    L = orc.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask)
    ref = orc.Grid(L, w.pts).radius(w.r_fx)
    say("uneven radius oracle pairs", int(ref.row_ptr[-1]))
    lat = lattice(sx, w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, w.pts)
    tab = sx.Tables(lat, 2, 4 * 65536)
    for name in ("sphere-persistent", "sphere-plain", "cube"):
        assert_same(run(sx, lat, tab, w.r_fx, launch=_launches(sx)[name]), ref, f"uneven radius {name}")
    # the launches the benchmark times: groups of queries whose rows are
    # sorted and kept in the count pass, grabs of 256 and of 64 queries
    for tile, bpc in ((256, 8), (64, 6)):
        ln = sx.LaunchConfig(method=sx.METHOD_SPHERE, schedule=sx.SCHED_PERSISTENT, grouped=1, interior=1,
                             sort_cap=256, waves_per_block=4, tile=tile, blocks_per_cu=bpc)
        say("uneven radius grouped with the stash", tile, bpc)
        assert_same(run(sx, lat, tab, w.r_fx, launch=ln, stash=True), ref, f"uneven radius grouped stash tile {tile}")


# ---------------------------------------------------------------------------
# K nearest

@pytest.mark.parametrize("K", [1, 4, 16, 70, 300])
def test_knn_clustered(sx, orc, K):
    from paper_cs_0608108_amd import synth
    lat_s = synth.LatticeSpec((5, 5, 5), 12, 7)
    pts = synth.gaussian_cluster_points(lat_s, 30000, 3, 8, 1.5 * lat_s.edge)
    say("knn K", K)
    L = orc.Lattice(lat_s.log2_cells, lat_s.frac_bits, 7)
    grid = orc.Grid(L, pts)
    rmax = 3 * lat_s.edge
    ref = grid.knn(np.full(len(pts[0]), K, np.uint32), np.full(len(pts[0]), rmax, np.uint32))
    lat = lattice(sx, lat_s.log2_cells, lat_s.frac_bits, 7, pts)
    tab = sx.Tables(lat, 2, rmax)
    for name in ("sphere-persistent", "sphere-plain", "sphere-small-cap", "cube", "sphere-grouped"):
        got = run(sx, lat, tab, rmax, k=K, mode=sx.MODE_KNN, launch=_launches(sx)[name])
        assert_same(got, ref, f"knn K={K} {name}")


def test_knn_clustered_full_size_every_row(sx, orc):
    """The clustered K-NN workload at full size (4,194,304 points in 64
    clusters, K = 16, search cap 8 cells) in the launches the benchmark
    times: groups of queries searched as radius rows at a first radius,
    rows kept in the count pass, with the objects inside each cell in the
    counting sort's order and in x order.  Every row (ids and squared
    distances) is checked against the oracle's K nearest of all points."""
    import torch

    from paper_cs_0608108_amd import synth
    w = synth.knn_clustered()
    n, K, cap = w.n, int(w.k[0]), int(w.r_fx[0])
    lat = lattice(sx, w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, w.pts)
    tab = sx.Tables(lat, 2, cap)
    q = sx.make_queries(n, None, cap, K, sx.MODE_KNN, 0)
    say("clustered K-NN oracle: K nearest of all 4,194,304 points")
    g = orc.Grid(orc.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask), w.pts)
    ref = g.knn(K, cap)
    g.close()
    assert int(ref.row_ptr[-1]) == n * K
    for order, tile, bpc in ((sx.ORDER_ANY, 64, 6), (sx.ORDER_ANY, 256, 8), (sx.ORDER_X, 64, 8)):
        lat.set_cell_order(order)
        lat.build(*lat._pts_dev)
        ln = sx.LaunchConfig(method=sx.METHOD_SPHERE, schedule=sx.SCHED_PERSISTENT, grouped=1, interior=1,
                             sort_cap=256, waves_per_block=4, tile=tile, blocks_per_cu=bpc)
        say("clustered K-NN grouped with the stash", order, tile, bpc)
        buf = sx.QueryBuffers(n, n * K, want_dist2=True, stash_pairs=3 * n * K)
        sx.query(lat, tab, q, buf, ln)
        torch.cuda.synchronize()
        assert_same(buf.host(), ref, f"clustered K-NN every row, order {order}, tile {tile}")
        del buf
    code, flags = lat.status()
    assert code == sx.OK and flags == 0


@pytest.mark.parametrize("mask", [0, 7])
def test_knn_random_worlds_and_mixed_batches(sx, orc, mask):
    rng = np.random.default_rng(77 + mask)
    log2, F = (3, 4, 3), 8
    e = 1 << F
    pts = tiny_points(rng, log2, F, mask, 3000, outside=True)
    lat = lattice(sx, log2, F, mask, pts)
    L = orc.Lattice(log2, F, mask)
    grid = orc.Grid(L, pts)
    tab = sx.Tables(lat, 2, 3 * e)
    n = len(pts[0])
    k = rng.integers(0, 40, n).astype(np.uint32)
    rmax = rng.integers(0, 4 * e, n).astype(np.uint32)
    for flags in (0, 1):
        ref = grid.knn(k, rmax, flags=flags)
        for name in ("sphere-persistent", "sphere-small-cap", "cube-plain", "auto", "list-plain",
                     "sphere-grouped-flat"):
            assert_same(run(sx, lat, tab, rmax, k=k, mode=sx.MODE_KNN, flags=flags, launch=_launches(sx)[name]),
                        ref, f"knn {name} flags={flags}")
    # mixed: K-NN where k > 0, radius otherwise; explicit centres
    qs = tiny_points(rng, log2, F, mask, 500, outside=True)
    kk = np.where(rng.random(500) < 0.5, rng.integers(1, 30, 500), 0).astype(np.uint32)
    rr = rng.integers(0, 4 * e, 500).astype(np.uint32)
    ref = grid.mixed(kk, rr, queries=qs)
    for name in ("sphere-persistent", "sphere-plain", "cube", "auto-grouped-weighted", "list-plain",
                 "sphere-grouped-flat"):
        assert_same(run(sx, lat, tab, rr, k=kk, mode=sx.MODE_MIXED, queries=qs, launch=_launches(sx)[name]),
                    ref, f"mixed {name}")


# ---------------------------------------------------------------------------
# Degenerate inputs

def test_edge_cases(sx, orc):
    log2, F, mask = (3, 3, 3), 6, 7
    e = 1 << F
    L = orc.Lattice(log2, F, mask)
    empty = tuple(np.zeros(0, np.uint32) for _ in range(3))
    # N = 0, all agents: Q = 0
    lat = lattice(sx, log2, F, mask, empty)
    tab = sx.Tables(lat, 2, 2 * e)
    rp, ids, d2 = run(sx, lat, tab, e)
    assert rp.tolist() == [0] and len(ids) == 0
    # N = 0 with explicit queries: empty rows
    qs = tuple(np.array([5, 100, 300], np.uint32) for _ in range(3))
    rp, ids, d2 = run(sx, lat, tab, e, queries=qs)
    assert rp.tolist() == [0, 0, 0, 0]
    # N = 1
    one = tuple(np.array([77], np.uint32) for _ in range(3))
    lat = lattice(sx, log2, F, mask, one)
    for flags, exp in ((0, [1]), (1, [0])):
        rp, ids, d2 = run(sx, lat, tab, 0, flags=flags)
        assert np.diff(rp).tolist() == exp
    # K = 0 and K > N
    rp, ids, d2 = run(sx, lat, tab, e, k=0, mode=sx.MODE_KNN)
    assert rp.tolist() == [0, 0]
    rp, ids, d2 = run(sx, lat, tab, e, k=50, mode=sx.MODE_KNN)
    assert rp.tolist() == [0, 1]
    # every object in one cell, radius covering them all: rows longer than
    # the LDS buffer take the windowed path
    rng = np.random.default_rng(5)
    n = 1100
    same = tuple((rng.integers(0, e, n) + 3 * e).astype(np.uint32) for _ in range(3))
    lat = lattice(sx, log2, F, mask, same)
    tab = sx.Tables(lat, 1, 2 * e)
    ref = orc.radius_brute(L, same, np.full(n, 2 * e, np.uint32))
    assert int(np.diff(ref.row_ptr).max()) == n
    for name in ("sphere-persistent", "sphere-small-cap", "cube"):
        assert_same(run(sx, lat, tab, 2 * e, launch=_launches(sx)[name]), ref, f"one cell {name}")
    refk = orc.radius_brute(L, same, np.full(n, 2 * e, np.uint32))
    got = run(sx, lat, tab, 2 * e, k=n + 5, mode=sx.MODE_KNN)
    assert_same(got, refk, "one cell knn K > N")
    # duplicates everywhere, r = 0: rows are the duplicate groups
    dup = tuple(np.repeat(rng.integers(0, 8 * e, 40), 5).astype(np.uint32) for _ in range(3))
    lat = lattice(sx, log2, F, mask, dup)
    ref = orc.radius_brute(L, dup, np.zeros(200, np.uint32))
    assert_same(run(sx, lat, tab, 0), ref, "r = 0 duplicates")
    # grouped, rows sorted in the count pass: every query of a group has
    # r = 0, so every hit has dist^2 0 and a row's order is its ids' alone
    for name in ("sphere-grouped", "sphere-grouped-flat"):
        for stash in (False, True):
            assert_same(run(sx, lat, tab, 0, launch=_launches(sx)[name], stash=stash), ref,
                        f"r = 0 duplicates {name} stash={stash}")
    # positions exactly on cell boundaries and at the world edge
    edge = tuple(np.array([0, e, 2 * e, 8 * e - 1, 4 * e, 4 * e - 1], np.uint32) for _ in range(3))
    lat = lattice(sx, log2, F, mask, edge)
    for r in (0, 1, e, 2 * e - 1, 2 * e):
        ref = orc.radius_brute(L, edge, np.full(6, r, np.uint32))
        assert_same(run(sx, lat, tab, r), ref, f"edges r={r}")
        assert_same(run(sx, lat, tab, r, launch=_launches(sx)["sphere-grouped-flat"], stash=True), ref,
                    f"edges grouped r={r}")


# ---------------------------------------------------------------------------
# Cells touched, error paths, movement, checksum, determinism

@pytest.mark.parametrize("mask", [0, 7])
def test_cells_touched_match_oracle(sx, orc, mask):
    import torch
    log2, F = (5, 5, 5), 16
    e = 1 << F
    rng = np.random.default_rng(8 + mask)
    n = 3000
    pts = tuple(rng.integers(0, 32 * e, n).astype(np.uint32) for _ in range(3))
    lat = lattice(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 4 * e)
    r = rng.integers(0, 4 * e, n).astype(np.uint32)
    stats = torch.zeros(4 * n, dtype=torch.int32, device="cuda")
    run(sx, lat, tab, r, launch=sx.LaunchConfig(stats=stats))
    st = stats.cpu().numpy().view(np.uint32).reshape(n, 4)
    kept, inter, cube = orc.cells_touched(orc.Lattice(log2, F, mask), pts, r)
    # rows are by object id; stats likewise
    np.testing.assert_array_equal(st[:, 1], kept)
    np.testing.assert_array_equal(st[:, 3], cube)
    # the walk visits x-rows of cells: at least one row wherever a cell is kept
    assert ((st[:, 0] > 0) | (st[:, 1] == 0)).all()
    say("mean kept/cube", st[:, 1].mean() / st[:, 3].mean())


def test_capacity_overflow_sets_flag_and_writes_nothing(sx, orc):
    import torch
    log2, F, mask = (4, 4, 4), 8, 0
    rng = np.random.default_rng(3)
    pts = tuple(rng.integers(0, 16 << 8, 4000).astype(np.uint32) for _ in range(3))
    lat = lattice(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 512)
    q = sx.make_queries(4000, None, 512)
    buf = sx.QueryBuffers(4000, 100)
    buf.ids.fill_(-7)
    sx.query(lat, tab, q, buf)
    code, flags = lat.status()
    assert code == sx.ERR_CAPACITY and flags & sx.FLAG_CAPACITY
    assert int(buf.row_ptr[-1]) > 100
    assert (buf.ids.cpu() == -7).all()
    # exact capacity works
    tot = int(buf.row_ptr[-1])
    buf2 = sx.QueryBuffers(4000, tot)
    sx.query(lat, tab, q, buf2)
    assert lat.status() == (sx.OK, 0)
    ref = orc.Grid(orc.Lattice(log2, F, mask), pts).radius(np.full(4000, 512, np.uint32))
    torch.cuda.synchronize()
    assert_same(buf2.host(), ref, "exact capacity")


def test_range_flag_for_unusable_query_centres(sx, orc):
    log2, F, mask = (3, 3, 3), 8, 0
    pts = tuple(np.arange(0, 2000, 7, dtype=np.uint32) for _ in range(3))
    lat = lattice(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 600)
    qs = tuple(np.array([10, 1 << 30, 500], np.uint32) for _ in range(3))
    rp, ids, d2 = run(sx, lat, tab, 600, queries=qs)
    code, flags = lat.status()
    assert flags & sx.FLAG_RANGE
    assert rp[2] - rp[1] == 0
    ref = orc.radius_brute(orc.Lattice(log2, F, mask), pts, np.full(3, 600, np.uint32), queries=qs)
    assert_same((rp, ids, d2), ref, "range")


def test_stream_status_and_named_radius_count(sx, orc):
    """sphidx_stream_status reports the flags set by the stream's calls on any
    lattice (then nothing until new work), and sphidx_radius_count gives the
    row sizes of sphidx_count in radius mode."""
    import ctypes

    import torch
    log2, F, mask = (3, 3, 3), 8, 0
    pts = tuple(np.arange(0, 2000, 7, dtype=np.uint32) for _ in range(3))
    lat = lattice(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 600)
    sx.stream_status()  # drain what earlier work on this stream left
    lat.build(*lat._pts_dev)
    assert sx.stream_status() == (sx.OK, 0)
    qs = tuple(sx.to_dev_u32(np.array([10, 1 << 30, 500], np.uint32)) for _ in range(3))
    q = sx.make_queries(3, qs, 600, None, sx.MODE_KNN)  # the named count forces radius mode
    buf = sx.QueryBuffers(3, 0)
    cs = buf.c()
    sx.check(sx.load().sphidx_radius_count(lat.handle, tab.handle, ctypes.byref(q), ctypes.byref(cs),
                                           sx._stream()), "radius_count")
    code, flags = sx.stream_status()
    assert code == sx.ERR_RANGE and flags & sx.FLAG_RANGE
    assert sx.stream_status() == (sx.OK, 0)
    ref = orc.radius_brute(orc.Lattice(log2, F, mask), pts, np.full(3, 600, np.uint32),
                           queries=tuple(q_.cpu().numpy().view(np.uint32) for q_ in qs))
    np.testing.assert_array_equal(buf.row_ptr.cpu().numpy(), ref.row_ptr)
    # a capacity overflow on another lattice, same stream
    lat2 = lattice(sx, log2, F, mask, pts)
    q2 = sx.make_queries(lat2.n, None, 600)
    small = sx.QueryBuffers(lat2.n, 1)
    sx.query(lat2, tab, q2, small)
    code, flags = sx.stream_status()
    assert code == sx.ERR_CAPACITY and flags == sx.FLAG_CAPACITY
    torch.cuda.synchronize()


def test_move_agents_and_checksum_match_oracle(sx, orc):
    import torch
    log2, F, mask = (6, 6, 6), 16, 7
    rng = np.random.default_rng(12)
    n = 50000
    pts = tuple(rng.integers(0, 64 << 16, n).astype(np.uint32) for _ in range(3))
    dev = [sx.to_dev_u32(a) for a in pts]
    desc = sx.desc_of(log2, F, mask)
    L = orc.Lattice(log2, F, mask)
    cur = pts
    for step in range(3):
        sx.move_agents(desc, 99, step, *dev)
        cur = orc.move(L, 99, step, cur)
    torch.cuda.synchronize()
    for a in range(3):
        np.testing.assert_array_equal(sx.to_host_u32(dev[a]), cur[a])
    lat = sx.Lattice(log2, F, mask, n)
    lat.build(*dev)
    tab = sx.Tables(lat, 2, 3 << 16)
    q = sx.make_queries(n, None, 3 << 16)
    buf = sx.QueryBuffers(n, 0)
    sx.count(lat, tab, q, buf)
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    sx.count_checksum(buf.row_ptr, n, out)
    got = out.cpu().numpy().view(np.uint64)
    ref = orc.Grid(L, cur).radius(np.full(n, 3 << 16, np.uint32))
    s, h = orc.count_checksum(ref.row_ptr)
    assert int(got[0]) == s and int(got[1]) == h


def test_runs_are_deterministic(sx):
    from paper_cs_0608108_amd import synth
    w = synth.radius_uneven_clipped(n=1 << 17, log2=6)
    lat = lattice(sx, w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, w.pts)
    tab = sx.Tables(lat, 2, 4 * 65536)
    a = run(sx, lat, tab, w.r_fx)
    lat.build(*lat._pts_dev)
    b = run(sx, lat, tab, w.r_fx)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("mask", [7, 0])
def test_cells_in_x_order_match_oracle(sx, orc, mask):
    """Objects ordered by x inside each cell (SPHIDX_ORDER_X): the build sorts
    every cell of at most 4,096 objects by (x, id), rows of many objects are
    narrowed to the sphere's x-slab by search, and every query result stays
    equal to the oracle's; a cell of more objects stays in the counting
    sort's order and its rows are tested whole."""
    import torch
    from paper_cs_0608108_amd import synth
    rng = np.random.default_rng(700 + mask)
    log2, F = (5, 5, 5), 12
    spec = synth.LatticeSpec(log2, F, mask)
    E = 1 << F
    dense = synth.gaussian_cluster_points(spec, 60000, 91, 8, 1.5 * E)
    W = 32 << F
    flat = [rng.integers(0, W, 8000).astype(np.uint32) for _ in range(3)]
    big = [np.full(5000, (3 << F) + 17 if a else (9 << F) + 5, np.uint32) for a in range(3)]
    big[0] = (9 << F) + rng.integers(0, E, 5000).astype(np.uint32)  # one cell of 5,000 objects
    pts = tuple(np.concatenate([dense[a], flat[a], big[a]]).astype(np.uint32) for a in range(3))
    n = len(pts[0])
    lat = sx.Lattice(log2, F, mask, n)
    lat.set_cell_order(sx.ORDER_X)
    dev = [sx.to_dev_u32(a) for a in pts]
    lat.build(*dev)
    h = lat.host_arrays()
    cs = h["cell_start"]
    sizes = np.diff(cs[: (1 << 15) + 1])
    assert sizes.max() == 5000 and (sizes > 24).sum() > 100
    for c in np.nonzero((sizes > 1) & (sizes <= 4096))[0]:
        xs, ids = h["xs"][cs[c]:cs[c + 1]].astype(np.int64), h["ids"][cs[c]:cs[c + 1]].astype(np.int64)
        key = (xs << 32) | ids
        assert np.all(np.diff(key) > 0), c
    tab = sx.Tables(lat, 2, 3 * E)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    r = rng.integers(0, 3 * E, n).astype(np.uint32)
    ref = g.radius(r)
    K = 12
    refk = g.knn(np.full(n, K, np.uint32), np.full(n, 3 * E, np.uint32))
    for launch, stash in ((sx.LaunchConfig(), True), (sx.LaunchConfig(grouped=1), True),
                          (sx.LaunchConfig(grouped=1, interior=2), False), (sx.LaunchConfig(), False)):
        say(f"x order mask={mask} grouped={launch.grouped} stash={stash}")
        assert_same(run(sx, lat, tab, r, launch=launch, stash=stash), ref, "radius, cells in x order")
        assert_same(run(sx, lat, tab, 3 * E, k=K, mode=sx.MODE_KNN, launch=launch, stash=stash), refk,
                    "K-NN, cells in x order")
    g.close()
    # a records update leaves cells unordered: results still exact
    scratch = torch.empty(4 * n, dtype=torch.int32, device="cuda")
    sx.move_resident(lat, 5, scratch, step=0)
    cur = orc.move(orc.Lattice(log2, F, mask), 5, 0, pts)
    ref2 = orc.Grid(orc.Lattice(log2, F, mask), cur).radius(r)
    assert_same(run(sx, lat, tab, r, launch=sx.LaunchConfig(grouped=1), stash=True), ref2, "after a records update")
    code, flags = lat.status()
    assert code == sx.OK, (code, flags)
