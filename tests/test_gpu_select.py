"""The non-empty cell list and the per-query method choice on the GPU
(Section III.B and III.C; weighting factor and reversal distances, Appendix).

* The list a build leaves in the attached buffer against the cells of the
  objects themselves (numpy), after a build, at attachment and after
  rebuilds with other objects.
* Every query forced through the list: radius, K-NN and mixed batches, all
  agents and free centres (some outside the region), against the oracle
  bit for bit.
* METHOD_AUTO: the walk each query used against a host model of the choice
  (sphere cells from the exported tables, cube cells from the centre and
  radius, the list's length), and the rows against the oracle.  Whichever
  walk a query takes, its row is the same: the choice only moves time."""
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


def _region_cells(log2, F, mask, pts):
    """Packed cell of every object inside the region."""
    inside = np.ones(len(pts[0]), dtype=bool)
    c = []
    for a in range(3):
        W = (1 << log2[a]) << F
        v = np.asarray(pts[a], dtype=np.uint64)
        if (mask >> a) & 1:
            v = v % W
        else:
            inside &= v < W
        c.append(v >> F)
    cell = (c[2] << (log2[0] + log2[1])) | (c[1] << log2[0]) | c[0]
    return cell[inside]


def _check_list(lat, log2, F, mask, pts, what):
    cnt, ent = lat.cell_list_host()
    want = np.unique(_region_cells(log2, F, mask, pts)) if len(pts[0]) else np.zeros(0, np.uint64)
    cs = lat.host_arrays()["cell_start"]
    nc = 1 << sum(log2)
    assert cnt == len(want), (what, cnt, len(want))
    assert np.array_equal(ent[:cnt, 0], want.astype(np.uint32)), what
    assert np.array_equal(ent[:cnt, 1], cs[want.astype(np.int64)]), what
    assert ent[cnt, 0] == 0xFFFFFFFF and ent[cnt, 1] == cs[nc], what


@pytest.mark.parametrize("mask", [7, 0, 5])
def test_cell_list_follows_builds(sx, mask):
    rng = np.random.default_rng(40 + mask)
    log2, F = (5, 4, 6), 10
    pts = tiny_points(rng, log2, F, mask, 3000, outside=(mask != 7), invalid=(mask == 0))
    lat = lattice(sx, log2, F, mask, pts, cell_list=False)
    say(f"cell list mask={mask}: attach after a build")
    lat.attach_cell_list()
    _check_list(lat, log2, F, mask, pts, "at attachment")
    for n in (2500, 17, 3000):
        pts2 = tiny_points(rng, log2, F, mask, n, outside=(mask != 7))
        dev = tuple(sx.to_dev_u32(a) for a in pts2)
        lat.build(*dev)
        _check_list(lat, log2, F, mask, pts2, f"rebuild n={n}")
    empty = tuple(sx.to_dev_u32(np.zeros(0, np.uint32)) for _ in range(3))
    lat.build(*empty)
    _check_list(lat, log2, F, mask, (np.zeros(0, np.uint32),) * 3, "empty")
    lat.attach_cell_list(False)
    code, flags = lat.status()  # RANGE: the objects left out on purpose (mask 0)
    assert flags & ~sx.FLAG_RANGE == 0 and code in (sx.OK, sx.ERR_RANGE)


def test_list_method_needs_a_list(sx):
    rng = np.random.default_rng(3)
    log2, F = (4, 4, 4), 8
    pts = tiny_points(rng, log2, F, 7, 500)
    lat = lattice(sx, log2, F, 7, pts, cell_list=False)
    with pytest.raises(sx.SphidxError):
        run(sx, lat, None, 1 << F, launch=sx.LaunchConfig(method=sx.METHOD_LIST))


def test_auto_without_a_list(sx, orc):
    """No list kept: the choice is between the sphere and the cube only."""
    import torch
    rng = np.random.default_rng(5)
    log2, F, mask = (4, 4, 4), 10, 7
    pts = tiny_points(rng, log2, F, mask, 300)
    lat = lattice(sx, log2, F, mask, pts, cell_list=False)
    tab = sx.Tables(lat, 2, 7 << F)
    r = rng.integers(0, 7 << F, 300).astype(np.uint32)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    ref = g.radius(r)
    g.close()
    mo = torch.full((300,), -7, dtype=torch.int32, device="cuda")
    say("auto without a list")
    assert_same(run(sx, lat, tab, r, launch=sx.LaunchConfig(method=sx.METHOD_AUTO, method_out=mo)), ref, "auto")
    used = set(mo.cpu().numpy().tolist())
    assert used <= {sx.METHOD_SPHERE, sx.METHOD_CUBE} and used


def _centres(rng, log2, F, mask, Q, outside_frac=0.1):
    cen = []
    for a in range(3):
        W = (1 << log2[a]) << F
        v = rng.integers(0, W, Q).astype(np.uint64)
        if not (mask >> a) & 1:
            k = int(Q * outside_frac)
            v[:k] = rng.integers(W, W + (3 << F), k)
        cen.append(v.astype(np.uint32))
    return tuple(cen)


@pytest.mark.parametrize("mask", [7, 0, 3])
def test_list_method_matches_oracle(sx, orc, mask):
    rng = np.random.default_rng(50 + mask)
    log2, F = (4, 5, 4), 10
    n = 4000
    pts = tiny_points(rng, log2, F, mask, n, outside=(mask != 7))
    lat = lattice(sx, log2, F, mask, pts)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    r = rng.integers(0, 3 << F, n).astype(np.uint32)
    ref = g.radius(r, flags=orc.EXCLUDE_SELF)
    launches = (sx.LaunchConfig(method=sx.METHOD_LIST), sx.LaunchConfig(method=sx.METHOD_LIST, grouped=1),
                sx.LaunchConfig(method=sx.METHOD_LIST, schedule=sx.SCHED_PLAIN, tile=2, sort_cap=64))
    for ln in launches:
        say(f"list mask={mask} all agents launch={ln.schedule}/{ln.grouped}/{ln.sort_cap}")
        assert_same(run(sx, lat, None, r, flags=sx.EXCLUDE_SELF, launch=ln), ref, "all agents, list")
        rd = sx.to_dev_u32(r)
        q = sx.make_queries(n, None, rd, None, sx.MODE_RADIUS, sx.EXCLUDE_SELF)
        assert_same(sx.run(lat, None, q, ln, stash=True), ref, "all agents, list, stash")
        del rd
    Q = 3000
    cen = _centres(rng, log2, F, mask, Q)
    rq = rng.integers(0, 4 << F, Q).astype(np.uint32)
    k = np.where(rng.random(Q) < 0.4, rng.integers(1, 30, Q), 0).astype(np.uint32)
    ref = g.mixed(k, rq, queries=cen)
    ref_knn = g.knn(12, 3 << F, queries=cen)
    g.close()
    for ln in launches[:2]:
        say(f"list mask={mask} mixed centres grouped={ln.grouped}")
        assert_same(run(sx, lat, None, rq, k, sx.MODE_MIXED, queries=cen, launch=ln), ref, "mixed, list")
        assert_same(run(sx, lat, None, 3 << F, 12, sx.MODE_KNN, queries=cen, launch=ln), ref_knn, "knn, list")


def _choice_model(sx, tab, log2, F, mask, cen, r, k, knn_mode, n_list, weight=256, rev=0, knn_rev=0, model=0,
                  n_obj=0):
    """The walk each query should take (Section III.B/C as the header states
    it), from the exported tables, the centre, the radius and the list.
    Model 1 counts rows (the table's cells with ox = 0 are its rows) plus the
    mean load times the cells tested."""
    info = tab.info()
    s, rmax = info.subcell_bits, info.rmax_fx
    b = max(F - 6, 0)
    e = 1 << F
    exported = [tab.export(c) for c in range(info.nclasses)]
    keys = [kk for _, kk in exported]
    row_keys = [kk[o[:, 0] == 0] for o, kk in exported]  # sorted: a subsequence of sorted keys
    load = min((n_obj << 8) // (1 << sum(log2)), 1 << 24) if model else 0
    out = np.empty(len(cen[0]), dtype=np.int64)
    for i in range(len(cen[0])):
        q = [int(cen[a][i]) for a in range(3)]
        ri = int(r[i])
        knn = knn_mode or int(k[i]) > 0
        inside, cyc_ok, ncube, nn, full = True, True, 1, [], 1
        for a in range(3):
            La = 1 << log2[a]
            lo, hi = (q[a] - ri) >> F, (q[a] + ri) >> F
            full *= min(hi - lo + 1, La) if (mask >> a) & 1 else hi - lo + 1
            if (mask >> a) & 1:
                if La < 4 or ri > (La // 2 - 1) * e:
                    cyc_ok = False
                if hi - lo + 1 >= La:
                    lo, hi = 0, La - 1
            else:
                inside &= q[a] < (La << F)
                lo, hi = max(lo, 0), min(hi, La - 1)
            nn.append(max(hi - lo + 1, 0))
            ncube *= nn[-1]
        sphere = inside and cyc_ok and ri <= rmax
        if knn:
            out[i] = sx.METHOD_SPHERE if sphere and ri >= knn_rev else sx.METHOD_CUBE
            continue
        sphere = sphere and ri >= rev
        wc = nn[1] * nn[2] * 256 + load * ncube if model else ncube
        chosen, tested = wc, ncube
        if sphere:
            cls = sum((((q[a] & (e - 1)) >> (F - s)) << (a * s)) for a in range(3))
            j = -(-ri // (1 << b))
            vs = int(np.searchsorted(keys[cls], (j << b) ** 2, side="right"))
            rows = int(np.searchsorted(row_keys[cls], (j << b) ** 2, side="right"))
            tested = vs * ncube // full
            ws = rows * 256 + load * tested if model else vs
            sphere = ws * weight <= wc * 256
            if sphere:
                chosen = ws
        wl = n_list * 256 + load * tested if model else n_list
        if wl < chosen:
            out[i] = sx.METHOD_LIST
        else:
            out[i] = sx.METHOD_SPHERE if sphere else sx.METHOD_CUBE
    return out


@pytest.mark.parametrize("mask,load", [(7, 0.625), (0, 0.625), (0, 5.0), (6, 1.0)])
def test_auto_choice_matches_model_and_oracle(sx, orc, mask, load):
    import torch
    rng = np.random.default_rng(int(60 + mask + 10 * load))
    log2, F = (4, 4, 4), 12
    n = int(load * (1 << sum(log2)))
    pts = tiny_points(rng, log2, F, mask, n, outside=(mask != 7))
    lat = lattice(sx, log2, F, mask, pts)
    n_list, _ = lat.cell_list_host()
    e = 1 << F
    tab = sx.Tables(lat, 2, 9 * e)
    Q = 1500
    cen = _centres(rng, log2, F, mask, Q, outside_frac=0.05)
    # distances from a tenth of a cell to past the tables' cap
    r = (rng.random(Q) ** 1.5 * 11 * e).astype(np.uint32)
    k = np.where(rng.random(Q) < 0.3, rng.integers(1, 20, Q), 0).astype(np.uint32)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    ref = g.mixed(k, r, queries=cen)
    g.close()
    seen = set()
    for weight, rev, knn_rev, model in ((0, 0, 0, 0), (512, e, 2 * e, 0), (64, 0, 0, 0), (0, 0, 0, 1),
                                        (320, e // 2, 0, 1)):
        mo = torch.full((Q,), -7, dtype=torch.int32, device="cuda")
        for grouped in (0, 1):
            ln = sx.LaunchConfig(method=sx.METHOD_AUTO, select_weight=weight, reversal_fx=rev,
                                 knn_reversal_fx=knn_rev, method_out=mo, grouped=grouped, select_model=model)
            say(f"auto mask={mask} load={load} weight={weight} rev={rev} knn_rev={knn_rev} model={model} "
                f"grouped={grouped}")
            got = run(sx, lat, tab, r, k, sx.MODE_MIXED, queries=cen, launch=ln)
            assert_same(got, ref, "auto choice, mixed")
            want = _choice_model(sx, tab, log2, F, mask, cen, r, k, False, n_list, weight or 256, rev, knn_rev,
                                 model, n)
            used = mo.cpu().numpy().astype(np.int64)
            bad = np.nonzero(used != want)[0]
            assert len(bad) == 0, (f"choice differs at {bad[:5]}: used {used[bad[:5]]} model {want[bad[:5]]} "
                                   f"r {r[bad[:5]]} k {k[bad[:5]]}")
            seen |= set(used.tolist())
    assert {sx.METHOD_SPHERE, sx.METHOD_CUBE} <= seen
    if load < 1:
        assert sx.METHOD_LIST in seen


def test_auto_all_agents_with_stash(sx, orc):
    rng = np.random.default_rng(77)
    log2, F, mask = (5, 5, 5), 12, 5
    n = 20000
    pts = tiny_points(rng, log2, F, mask, n, outside=True)
    lat = lattice(sx, log2, F, mask, pts)
    e = 1 << F
    tab = sx.Tables(lat, 2, 3 * e)
    r = (rng.random(n) * 4 * e).astype(np.uint32)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    ref = g.radius(r)
    g.close()
    rd = sx.to_dev_u32(r)
    q = sx.make_queries(n, None, rd, None, sx.MODE_RADIUS, 0)
    for ln in (sx.LaunchConfig(method=sx.METHOD_AUTO), sx.LaunchConfig(method=sx.METHOD_AUTO, grouped=1),
               sx.LaunchConfig(method=sx.METHOD_AUTO, reversal_fx=e)):
        say(f"auto all agents grouped={ln.grouped} rev={ln.reversal_fx}")
        assert_same(sx.run(lat, tab, q, ln, stash=True), ref, "auto, all agents, stash")
    del rd


@pytest.mark.parametrize("log2,mask", [((1, 1, 2), 7), ((1, 2, 3), 5), ((2, 1, 1), 3)])
def test_list_walk_on_tiny_wrapping_axes(sx, orc, log2, mask):
    """Axes of two and four cells, radii past the whole world: the list walk's
    nearest image (both images equally far at half the axis) and the choice
    between cube and list where no table applies, against brute force."""
    rng = np.random.default_rng(90 + sum(log2) + mask)
    F = 8
    pts = tiny_points(rng, log2, F, mask, 600, outside=(mask != 7))
    lat = lattice(sx, log2, F, mask, pts)
    tab = sx.Tables(lat, 2, 3 << F)
    L = orc.Lattice(log2, F, mask)
    r = rng.integers(0, 6 << F, len(pts[0])).astype(np.uint32)
    ref = orc.radius_brute(L, pts, r)
    for name, ln in (("list", sx.LaunchConfig(method=sx.METHOD_LIST)),
                     ("auto", sx.LaunchConfig(method=sx.METHOD_AUTO)),
                     ("auto-work", sx.LaunchConfig(method=sx.METHOD_AUTO, select_model=1, grouped=1))):
        say(f"tiny world {log2} mask={mask} {name}")
        assert_same(run(sx, lat, tab, r, launch=ln), ref, f"tiny {name}")
    cen = _centres(rng, log2, F, mask, 300)
    k = rng.integers(1, 12, 300).astype(np.uint32)
    rq = rng.integers(0, 6 << F, 300).astype(np.uint32)
    refk = orc.knn_brute(L, pts, k, rq, queries=cen)
    assert_same(run(sx, lat, tab, rq, k, sx.MODE_KNN, queries=cen, launch=sx.LaunchConfig(method=sx.METHOD_LIST)),
                refk, "tiny knn list")
