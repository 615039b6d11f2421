"""The count pass's stash (sorted rows kept in the workspace and copied into
place by the write pass) against the oracle, bit for bit: every row stashed,
a stash too small for all rows (the rest walked again), a write asking for
dist^2 after a count that kept none, cube-fallback and K-NN rows in the mix,
and repeated count/write cycles on one workspace."""
import numpy as np
import pytest

from gpu_util import assert_same, say, tiny_points

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_cs_0608108_amd import sphidx
    sphidx.load()
    return sphidx


def _world(sx, log2, F, mask, pts):
    lat = sx.Lattice(log2, F, mask, max(len(pts[0]), 1))
    dev = tuple(sx.to_dev_u32(a) for a in pts)
    lat.build(*dev)
    lat._dev = dev
    return lat


def _cycle(sx, lat, tab, q, launch, want_d2_count, want_d2_write, stash_frac):
    """count (sizing) -> reserve a stash for a fraction of the pairs -> count
    -> write; returns host rows and the number of pairs."""
    buf = sx.QueryBuffers(q.count, 0, want_dist2=want_d2_count)
    sx.count(lat, tab, q, buf, launch)
    total = int(buf.row_ptr[-1].item())
    if stash_frac > 0:
        buf.reserve_stash(max(int(total * stash_frac), 1))
    buf.grow(max(total, 1))
    sx.count(lat, tab, q, buf, launch)
    if want_d2_write and buf.dist2 is None:
        import torch
        buf.dist2 = torch.empty(max(buf.capacity, 1), dtype=torch.int64, device="cuda")
    if not want_d2_write:
        buf.dist2 = None
    sx.write(lat, tab, q, buf, launch)
    import torch
    torch.cuda.synchronize()
    code, flags = lat.status()
    assert code == sx.OK and not (flags & sx.FLAG_CAPACITY), (code, flags)
    return buf.host(), total


@pytest.mark.parametrize("mask", [0, 7])
@pytest.mark.parametrize("stash_frac", [1.0, 0.3, 0.0])
def test_stash_radius_rows_match_oracle(sx, orc, mask, stash_frac):
    rng = np.random.default_rng(100 + mask)
    log2, F = (5, 4, 5), 10
    pts = tiny_points(rng, log2, F, mask, 30000, outside=(mask != 7))
    lat = _world(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 3 << F)
    r = rng.integers(1, 3 << F, size=len(pts[0])).astype(np.uint32)
    r_dev = sx.to_dev_u32(r)  # queries hold raw pointers: keep the tensor alive
    q = sx.make_queries(len(pts[0]), None, r_dev, None, sx.MODE_RADIUS, 0)
    L = orc.Lattice(log2, F, mask)
    g = orc.Grid(L, pts)
    ref = g.radius(r)
    g.close()
    for launch in (sx.LaunchConfig(), sx.LaunchConfig(grouped=1),
                   sx.LaunchConfig(schedule=sx.SCHED_PLAIN, sort_cap=64, tile=2)):
        say(f"stash mask={mask} frac={stash_frac} launch={launch.schedule}/{launch.sort_cap}")
        got, total = _cycle(sx, lat, tab, q, launch, True, True, stash_frac)
        assert_same(got, ref, f"stash frac {stash_frac}")
    del r_dev


def test_stash_without_dist2_then_write_with_dist2(sx, orc):
    rng = np.random.default_rng(7)
    log2, F = (5, 5, 5), 12
    pts = tiny_points(rng, log2, F, 7, 20000)
    lat = _world(sx, log2, F, 7, pts)
    tab = sx.Tables(lat, 2, 2 << F)
    q = sx.make_queries(len(pts[0]), None, 2 << F, None, sx.MODE_RADIUS, sx.EXCLUDE_SELF)
    g = orc.Grid(orc.Lattice(log2, F, 7), pts)
    ref = g.radius(2 << F, flags=orc.EXCLUDE_SELF)
    g.close()
    say("stash ids only, write asks dist2")
    got, _ = _cycle(sx, lat, tab, q, sx.LaunchConfig(), False, True, 1.0)
    assert_same(got, ref, "dist2 requested after an ids-only stash")
    say("stash ids only, write ids only")
    got, _ = _cycle(sx, lat, tab, q, sx.LaunchConfig(), False, False, 1.0)
    assert_same((got[0], got[1], None), ref, "ids-only stash")


def test_stash_with_fallback_and_knn_rows(sx, orc):
    rng = np.random.default_rng(11)
    log2, F = (5, 5, 4), 10
    mask = 1
    pts = tiny_points(rng, log2, F, mask, 25000, outside=True)
    lat = _world(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 2 << F)  # radii above 2 cells fall back to the cube scan
    Qn = 6000
    W = [(1 << (log2[a] + F)) for a in range(3)]
    cen = [rng.integers(0, W[a] + (W[a] // 8 if a else 0), size=Qn).astype(np.uint32) for a in range(3)]
    r = rng.integers(0, 4 << F, size=Qn).astype(np.uint32)
    k = np.where(rng.random(Qn) < 0.3, rng.integers(1, 40, size=Qn), 0).astype(np.uint32)
    keep = (tuple(sx.to_dev_u32(c) for c in cen), sx.to_dev_u32(r), sx.to_dev_u32(k))
    q = sx.make_queries(Qn, keep[0], keep[1], keep[2], sx.MODE_MIXED, 0)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    ref = g.mixed(k, r, queries=tuple(cen))
    g.close()
    for frac, grouped in ((1.0, 0), (0.5, 0), (1.0, 1), (0.5, 1)):
        say(f"mixed stash frac={frac} grouped={grouped}")
        got, _ = _cycle(sx, lat, tab, q, sx.LaunchConfig(grouped=grouped), True, True, frac)
        assert_same(got, ref, f"mixed batch with fallback rows, stash {frac}")
    del keep


def test_ids_only_stash_then_dist2_writes_with_fallback_and_knn_rows(sx, orc):
    """A count that keeps ids only, then two writes that ask for dist^2: rows
    off the sphere tables (radii above the cap, centres outside a clipped
    region) and K-NN rows of a mixed batch are walked again, each once, by
    both writes, in one-query-per-wave and grouped launches."""
    import torch
    rng = np.random.default_rng(12)
    log2, F = (5, 5, 4), 10
    mask = 1
    pts = tiny_points(rng, log2, F, mask, 25000, outside=True)
    lat = _world(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 2 << F)  # radii above 2 cells fall back to the cube scan
    Qn = 6000
    W = [(1 << (log2[a] + F)) for a in range(3)]
    cen = [rng.integers(0, W[a] + (W[a] // 8 if a else 0), size=Qn).astype(np.uint32) for a in range(3)]
    r = rng.integers(0, 4 << F, size=Qn).astype(np.uint32)
    k = np.where(rng.random(Qn) < 0.3, rng.integers(1, 40, size=Qn), 0).astype(np.uint32)
    keep = (tuple(sx.to_dev_u32(c) for c in cen), sx.to_dev_u32(r), sx.to_dev_u32(k))
    q = sx.make_queries(Qn, keep[0], keep[1], keep[2], sx.MODE_MIXED, 0)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    ref = g.mixed(k, r, queries=tuple(cen))
    g.close()
    fb = int(((r > (2 << F)) & (k == 0)).sum())
    assert fb > 100 and int((k > 0).sum()) > 1000
    for grouped in (0, 1):
        say(f"ids-only stash, two dist2 writes, grouped={grouped}")
        launch = sx.LaunchConfig(grouped=grouped)
        buf = sx.QueryBuffers(Qn, 0, want_dist2=False)
        sx.count(lat, tab, q, buf, launch)
        total = int(buf.row_ptr[-1].item())
        buf.grow(max(total, 1))
        buf.reserve_stash(max(total, 1))
        sx.count(lat, tab, q, buf, launch)
        buf.dist2 = torch.empty(max(buf.capacity, 1), dtype=torch.int64, device="cuda")
        for it in range(2):
            buf.ids.fill_(-1)
            buf.dist2.fill_(-1)
            sx.write(lat, tab, q, buf, launch)
            torch.cuda.synchronize()
            code, flags = lat.status()
            assert code == sx.OK and not (flags & sx.FLAG_CAPACITY), (code, flags)
            assert_same(buf.host(), ref, f"grouped {grouped}, write {it}")
    del keep


def test_stash_repeated_cycles_full_size(sx, orc):
    """The uneven-radius workload at full size, three count/write cycles on
    one workspace with the stash sized once."""
    import torch

    from paper_cs_0608108_amd import synth
    w = synth.radius_uneven_clipped()
    lat = _world(sx, w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, w.pts)
    tab = sx.Tables(lat, 2, 4 * w.lat.edge)
    rad = sx.to_dev_u32(w.r_fx)
    q = sx.make_queries(w.n, None, rad, None, sx.MODE_RADIUS, 0)
    buf = sx.QueryBuffers(w.n, 0, want_dist2=False)
    sx.count(lat, tab, q, buf)
    total = int(buf.row_ptr[-1].item())
    buf.grow(total)
    buf.reserve_stash(total)
    g = orc.Grid(orc.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask), w.pts)
    ref = g.radius(w.r_fx)
    g.close()
    for it in range(3):
        say(f"full-size stash cycle {it}")
        lat.build(*lat._dev)
        sx.count(lat, tab, q, buf)
        sx.write(lat, tab, q, buf)
        torch.cuda.synchronize()
        rp, ids, _ = buf.host()
        assert_same((rp, ids, None), ref, f"cycle {it}")
    code, flags = lat.status()
    assert code == sx.OK and flags == 0


@pytest.mark.parametrize("sort_cap", [64, 128, 256])
def test_grouped_count_overflowing_hit_buffer(sx, orc, sort_cap):
    """Dense cells: a group's hits overflow its buffer, so its rows are counted
    exactly but walked again by the write pass."""
    from paper_cs_0608108_amd import synth
    w = synth.sweep_world(4, 0, 20.0)
    lat = _world(sx, w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask, w.pts)
    tab = sx.Tables(lat, 2, 2 * w.lat.edge)
    r = int(1.5 * w.lat.edge)
    q = sx.make_queries(w.n, None, r, None, sx.MODE_RADIUS, 0)
    g = orc.Grid(orc.Lattice(w.lat.log2_cells, w.lat.frac_bits, w.lat.cyclic_mask), w.pts)
    ref = g.radius(r)
    g.close()
    say(f"grouped overflow sort_cap={sort_cap}")
    ln = sx.LaunchConfig(grouped=1, sort_cap=sort_cap, waves_per_block=2)
    got, _ = _cycle(sx, lat, tab, q, ln, False, False, 1.0)
    assert_same((got[0], got[1], None), ref, f"grouped overflow {sort_cap}")


@pytest.mark.parametrize("mask", [7, 0])
@pytest.mark.parametrize("method", ["sphere", "cube"])
def test_grouped_rows_beyond_one_chunk(sx, orc, mask, method):
    """Radii of 3 to 7 cells against sort_cap 64 and 128: one query's rows
    span several chunks of the grouped walk (and several groups' hits
    overflow the buffer), with and without the stash."""
    rng = np.random.default_rng(140 + mask)
    log2, F = (5, 5, 5), 8
    pts = tiny_points(rng, log2, F, mask, 20000, outside=(mask != 7))
    lat = _world(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 7 << F)
    r = rng.integers(3 << F, (7 << F) + 1, size=len(pts[0])).astype(np.uint32)
    r_dev = sx.to_dev_u32(r)
    q = sx.make_queries(len(pts[0]), None, r_dev, None, sx.MODE_RADIUS, 0)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    ref = g.radius(r)
    g.close()
    m = sx.METHOD_SPHERE if method == "sphere" else sx.METHOD_CUBE
    for cap in (64, 128):
        for frac in (1.0, 0.0):
            say(f"grouped chunks mask={mask} method={method} sort_cap={cap} stash={frac}")
            ln = sx.LaunchConfig(method=m, grouped=1, sort_cap=cap, waves_per_block=2)
            got, _ = _cycle(sx, lat, tab, q, ln, True, True, frac)
            assert_same(got, ref, f"grouped chunks {method} cap {cap} stash {frac}")
    del r_dev


@pytest.mark.parametrize("mask", [7, 0])
def test_grouped_knn_radius_rows_match_oracle(sx, orc, mask):
    """K-NN rows searched in groups as radius rows at a first search radius:
    dense clusters (rows kept from a radius that holds K), sparse regions and
    small caps (fewer than K inside: searched again in groups at a larger
    radius, then one query per wavefront, or every object when the radius
    covers the cap), K above half the hit buffer (one query per
    wavefront), buffers that overflow.  Cells holding a tight clump in one
    corner and a lone object in the opposite corner make the home-cell
    density far too high for the lone object's rows, so that they fail both
    grouped rounds."""
    from paper_cs_0608108_amd import synth
    log2, F = (5, 5, 5), 12
    E = 1 << F
    spec = synth.LatticeSpec(log2, F, mask)
    dense = synth.gaussian_cluster_points(spec, 24000, 41 + mask, 8, 1.5 * E)
    sparse = synth.uniform_points(spec, 6000, 43 + mask)
    crng = np.random.default_rng(900 + mask)
    cells = crng.integers(2, 30, (20, 3))
    clump = [np.concatenate([(c[a] << F) + crng.integers(0, E // 16, 300) for c in cells]) for a in range(3)]
    lone = [(cells[:, a] << F) + E - 1 - crng.integers(0, E // 16, 20) for a in range(3)]
    pts = tuple(np.concatenate([dense[a], sparse[a], clump[a], lone[a]]).astype(np.uint32) for a in range(3))
    lat = _world(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 4 << F)
    n = len(pts[0])
    rng = np.random.default_rng(300 + mask)
    k = rng.choice(np.array([1, 4, 16, 40, 70], dtype=np.uint32), n)
    cap = rng.integers(1 << (F - 2), (4 << F) + 1, n).astype(np.uint32)
    keep = (sx.to_dev_u32(k), sx.to_dev_u32(cap))
    q = sx.make_queries(n, None, keep[1], keep[0], sx.MODE_KNN, sx.EXCLUDE_SELF)
    km = np.where(rng.random(n) < 0.5, k, 0).astype(np.uint32)
    keep2 = sx.to_dev_u32(km)
    qm = sx.make_queries(n, None, keep[1], keep2, sx.MODE_MIXED, 0)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    ref = g.knn(k, cap, flags=orc.EXCLUDE_SELF)
    refm = g.mixed(km, cap)
    g.close()
    for cap_lds in (64, 256):
        for frac in (1.0, 0.3, 0.0):
            say(f"grouped knn mask={mask} sort_cap={cap_lds} stash={frac}")
            ln = sx.LaunchConfig(grouped=1, sort_cap=cap_lds, waves_per_block=2)
            got, _ = _cycle(sx, lat, tab, q, ln, True, True, frac)
            assert_same(got, ref, f"grouped knn {cap_lds} {frac}")
            got, _ = _cycle(sx, lat, tab, qm, ln, True, True, frac)
            assert_same(got, refm, f"grouped mixed {cap_lds} {frac}")
    del keep, keep2


@pytest.mark.parametrize("mask", [7, 0])
def test_stash_knn_rows_match_oracle(sx, orc, mask):
    """K-NN rows searched and kept by the count pass (K <= 64) beside rows the
    top-K pass still walks (K > 64, or no stash room), in K-NN and mixed
    batches; ids-only stash with dist^2 asked by the write."""
    rng = np.random.default_rng(200 + mask)
    log2, F = (5, 4, 5), 10
    pts = tiny_points(rng, log2, F, mask, 30000, outside=(mask != 7))
    lat = _world(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 3 << F)
    n = len(pts[0])
    k = rng.integers(1, 90, n).astype(np.uint32)  # some above 64
    k[:50] = 64
    k[50:100] = 65
    cap = rng.integers(0, 3 << F, n).astype(np.uint32)
    keep = (sx.to_dev_u32(k), sx.to_dev_u32(cap))
    q = sx.make_queries(n, None, keep[1], keep[0], sx.MODE_KNN, sx.EXCLUDE_SELF)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    ref = g.knn(k, cap, flags=orc.EXCLUDE_SELF)
    km = np.where(rng.random(n) < 0.5, k, 0).astype(np.uint32)
    keep2 = sx.to_dev_u32(km)
    qm = sx.make_queries(n, None, keep[1], keep2, sx.MODE_MIXED, 0)
    refm = g.mixed(km, cap)
    g.close()
    for frac in (1.0, 0.3):
        for launch in (sx.LaunchConfig(), sx.LaunchConfig(grouped=1)):
            say(f"knn stash mask={mask} frac={frac} grouped={launch.grouped}")
            got, _ = _cycle(sx, lat, tab, q, launch, True, True, frac)
            assert_same(got, ref, f"knn stash {frac}")
            got, _ = _cycle(sx, lat, tab, qm, launch, True, True, frac)
            assert_same(got, refm, f"mixed stash {frac}")
    say("knn stash ids only, write asks dist2")
    got, _ = _cycle(sx, lat, tab, q, sx.LaunchConfig(), False, True, 1.0)
    assert_same(got, ref, "knn ids-only stash, dist2 written")
    del keep, keep2
