"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test ties one part of ``oracle/oracle.c`` to something other than the
oracle itself: a value printed in the paper (fixtures under tests/golden/,
each citing its passage), a hand-worked example, a closed form, a theorem,
an exhaustive brute force, or a second tier written independently.
"""
import math

import numpy as np
import pytest

from goldens import read_hand, read_matrix, read_pairs

F16 = 16
E16 = 1 << F16


def lat(orc, log2, F, mask):
    return orc.Lattice(tuple(log2), F, mask)


# ---------------------------------------------------------------------------
# Fig. 2 and the three-dimensional shells (Section II.A)

def test_fig2_base_bound_matches_printed_table(orc):
    fig2 = read_matrix("fig2_min_bound_2d.txt")
    assert fig2.shape == (9, 9)
    for iy, oy in enumerate(range(-4, 5)):
        for ix, ox in enumerate(range(-4, 5)):
            assert orc.base_minbound2([ox, oy]) == fig2[iy, ix], (ox, oy)


def test_fig2_matches_fixed_point_key_of_whole_cell_class(orc):
    # With no sub-cell bits the class box is the whole centre cell; the exact
    # key in units^2, divided by the squared cell edge and floored, must give
    # the printed bound (the +1 unit gap is the paper's 1-ulp remark).
    fig2 = read_matrix("fig2_min_bound_2d.txt")
    for iy, oy in enumerate(range(-4, 5)):
        for ix, ox in enumerate(range(-4, 5)):
            key = orc.table_key(F16, 0, [0, 0, 0], [ox, oy, 0])
            assert key // (E16 * E16) == fig2[iy, ix], (ox, oy)
            # and the key is strictly positive exactly off the 3x3 block
            assert (key == 0) == (abs(ox) <= 0 and abs(oy) <= 0)


def test_shell_counts_3d(orc):
    exp = read_pairs("shell_counts_3d.txt")
    counts = {}
    R = 5
    for z in range(-R, R + 1):
        for y in range(-R, R + 1):
            for x in range(-R, R + 1):
                b2 = orc.base_minbound2([x, y, z])
                counts[b2] = counts.get(b2, 0) + 1
    for b2, c in exp.items():
        assert counts.get(b2, 0) == c, b2


def test_missing_squared_bounds_are_legendre_numbers(orc):
    # Section II.A: some squared distances (7, ...) never occur.  The bound is
    # a sum of three squares of non-negative integers, so by Legendre's
    # three-square theorem the missing values are exactly 4^a (8b + 7).
    seen = set()
    R = 12
    for z in range(0, R + 1):
        for y in range(0, R + 1):
            for x in range(0, R + 1):
                seen.add(orc.base_minbound2([x, y, z]))
    limit = 100
    missing = {n for n in range(limit) if n not in seen}
    legendre = set()
    a = 1
    while a < limit:
        b = 0
        while a * (8 * b + 7) < limit:
            legendre.add(a * (8 * b + 7))
            b += 1
        a *= 4
    assert 7 in missing
    assert missing == legendre


# ---------------------------------------------------------------------------
# Sub-cell specialised table keys (Section III.A, Figs. 3 and 4)

@pytest.mark.parametrize("s", [0, 1, 2, 3])
def test_table_key_closed_form_equals_exhaustive_minimum(orc, s):
    F = 3
    n = 1 << s
    rng = np.random.default_rng(100 + s)
    classes = [(a, b, c) for a in range(n) for b in range(n) for c in range(n)]
    if len(classes) > 27:
        classes = [classes[i] for i in rng.choice(len(classes), 27, replace=False)]
    for cls in classes:
        for oz in range(-3, 4):
            for oy in range(-3, 4):
                for ox in range(-3, 4):
                    o = [ox, oy, oz]
                    assert orc.table_key(F, s, cls, o) == orc.table_key_brute(F, s, cls, o), (cls, o)


def test_table_key_is_a_lower_bound_attained_in_the_class_box(orc):
    # Any position in the class box and any position in cell o are at least
    # sqrt(key) apart (the completeness argument of Section II.A).
    F, s = 4, 2
    e, w = 1 << F, 1 << (F - s)
    rng = np.random.default_rng(7)
    for _ in range(400):
        cls = rng.integers(0, 1 << s, 3)
        o = rng.integers(-4, 5, 3)
        key = orc.table_key(F, s, cls, o)
        q = cls * w + rng.integers(0, w, 3)
        p = o * e + rng.integers(0, e, 3)
        assert int(np.sum((p - q) ** 2)) >= key


def test_unshaved_table_always_holds_27_cells_below_one_cell(orc):
    # Section III.A: below one cell of radius the table built on the whole
    # centre cell always brings in the 27 cells, while the bin-lattice cube
    # holds between 1 and 27 cells depending on the centre.
    # Fixed point keeps the paper's "one unit of least precision" between
    # adjacent cells (Section II.A): the 26 neighbours have keys 1, 2 or 3
    # units^2, so all 27 cells are in from r = 2 units up to one cell.
    for r in [2, 100, E16 // 2, E16 - 1]:
        offs, _ = orc.table_set(F16, 0, [0, 0, 0], r)
        got = sorted(map(tuple, offs.tolist()))
        assert got == sorted((x, y, z) for x in (-1, 0, 1) for y in (-1, 0, 1) for z in (-1, 0, 1))
    offs, keys = orc.table_set(F16, 0, [0, 0, 0], 1)
    assert len(offs) == 7 and sorted(keys.tolist()) == [0] + [1] * 6
    L = lat(orc, (4, 4, 4), F16, 7)
    rng = np.random.default_rng(11)
    counts = set()
    for _ in range(3000):
        q = rng.integers(0, 16 * E16, 3)
        r = int(rng.integers(0, E16))
        counts.add(orc.cube_cells(L, q, r))
    assert min(counts) == 1 and max(counts) == 27
    assert counts <= {1, 2, 3, 4, 6, 8, 9, 12, 18, 27}


# ---------------------------------------------------------------------------
# Cells intersecting the sphere vs the bounding cube (Section I: ~52 %)

def _steiner_kept(r):
    # Expected number of unit cells met by a ball of radius r whose centre is
    # uniform in a cell = volume of (unit cube + ball): Steiner's formula.
    return 1 + 6 * r + 3 * math.pi * r * r + 4.0 / 3.0 * math.pi * r ** 3


@pytest.mark.parametrize("r_cells,nq", [(0.5, 4000), (1.0, 4000), (2.5, 3000), (4.0, 2000), (8.0, 600)])
def test_expected_cells_touched_match_steiner_formula(orc, r_cells, nq):
    L = lat(orc, (6, 6, 6), F16, 7)
    rng = np.random.default_rng(int(r_cells * 10))
    q = [rng.integers(0, 64 * E16, nq).astype(np.uint32) for _ in range(3)]
    r = np.full(nq, int(round(r_cells * E16)), dtype=np.uint32)
    kept, inter, cube = orc.cells_touched(L, q, r)
    assert (kept >= inter).all() and (cube >= kept).all()
    assert abs(kept.mean() / _steiner_kept(r_cells) - 1) < 0.02
    assert abs(cube.mean() / (2 * r_cells + 1) ** 3 - 1) < 0.02


def test_sphere_over_cube_ratio_tends_to_pi_over_six(orc):
    L = lat(orc, (6, 6, 6), F16, 7)
    rng = np.random.default_rng(5)
    nq = 150
    q = [rng.integers(0, 64 * E16, nq).astype(np.uint32) for _ in range(3)]
    r_cells = 16
    kept, _, cube = orc.cells_touched(L, q, np.full(nq, r_cells * E16, dtype=np.uint32))
    ratio = kept.sum() / cube.sum()
    steiner = _steiner_kept(r_cells) / (2 * r_cells + 1) ** 3
    assert abs(ratio - steiner) < 0.01
    # the closed form decreases towards pi/6 (~52 %, Section I)
    seq = [_steiner_kept(x) / (2 * x + 1) ** 3 for x in (1, 4, 16, 64, 1024, 1 << 20)]
    assert all(a > b for a, b in zip(seq, seq[1:]))
    assert abs(seq[-1] - math.pi / 6) < 1e-5


def test_bin_lattice_covers_cyclic_16_world_from_7_5_cells(orc):
    # Section IV.A: in a 16^3 wrapping world the bin-lattice cube covers the
    # whole world for radii above 7.5 cells (span floor(q+r)-floor(q-r)+1 >= 16
    # for every centre iff 2r >= 15).
    L = lat(orc, (4, 4, 4), F16, 7)
    rng = np.random.default_rng(3)
    centres = [rng.integers(0, 16 * E16, 3) for _ in range(500)]
    centres += [np.array([k * E16 + E16 // 2] * 3) for k in range(16)]
    r = int(7.5 * E16)
    assert all(orc.cube_cells(L, q, r) == 4096 for q in centres)
    assert any(orc.cube_cells(L, q, r - 1) < 4096 for q in centres)


# ---------------------------------------------------------------------------
# Hand-worked fixtures: inclusive boundary, minimum image, ties, self, outside

@pytest.mark.parametrize("name", ["hand_cyclic.txt", "hand_clipped.txt"])
def test_hand_fixture_all_tiers(orc, name):
    latd, pts, rows = read_hand(name)
    L = orc.Lattice(latd["log2_cells"], latd["frac_bits"], latd["cyclic_mask"])
    n = len(pts[0])
    grid = orc.Grid(L, pts)
    for row in rows:
        rr = np.zeros(n, dtype=np.uint32)
        rr[:] = row["r"]
        if row["kind"] == "radius":
            outs = [orc.radius_brute(L, pts, rr, flags=row["flags"]),
                    grid.radius(rr, flags=row["flags"])]
            if latd["cyclic_mask"] == 7:
                outs.append(orc.radius_images(L, pts, rr, flags=row["flags"]))
        else:
            kk = np.full(n, row["k"], dtype=np.uint32)
            outs = [orc.knn_brute(L, pts, kk, rr, flags=row["flags"]),
                    grid.knn(kk, rr, flags=row["flags"])]
        for out in outs:
            ids, d2 = out.row(row["q"])
            assert list(zip(d2.tolist(), ids.tolist())) == row["exp"], row


# ---------------------------------------------------------------------------
# Tiers against each other on random tiny worlds

def _tiny(rng, log2, F, mask, n, outside):
    pts = []
    for a in range(3):
        W = (1 << log2[a]) << F
        if (mask >> a) & 1:
            v = rng.integers(0, 1 << 32, n, dtype=np.uint64)          # any value; wraps
            v[: n // 4] = rng.integers(0, W, n // 4)
        else:
            v = rng.integers(0, W, n, dtype=np.uint64)
            if outside:
                k = n // 8
                v[:k] = rng.integers(W, 2 * W + 3, k)                  # outside the region
                v[k:k + 2] = [1 << 30, (1 << 32) - 1]                  # unusable
        pts.append(v.astype(np.uint32))
    # duplicates and cell-boundary positions
    for a in range(3):
        pts[a][-3] = pts[a][-4]
        pts[a][-5] = (pts[a][-5] >> F) << F
    return tuple(pts)


CASES = [((1, 1, 1), 2), ((2, 2, 2), 2), ((3, 2, 1), 3), ((3, 3, 3), 4), ((2, 3, 2), 1)]


@pytest.mark.parametrize("mask", range(8))
@pytest.mark.parametrize("shape", CASES)
def test_min_image_formula_equals_explicit_images(orc, mask, shape):
    log2, F = shape
    rng = np.random.default_rng(1000 + mask * 10 + F)
    L = orc.Lattice(log2, F, mask)
    pts = _tiny(rng, log2, F, mask, 120, outside=False)
    E = 1 << F
    r = rng.integers(0, 3 * E, 120).astype(np.uint32)
    a = orc.radius_brute(L, pts, r)
    b = orc.radius_images(L, pts, r)
    np.testing.assert_array_equal(a.row_ptr, b.row_ptr)
    np.testing.assert_array_equal(a.ids, b.ids)
    np.testing.assert_array_equal(a.dist2, b.dist2)


@pytest.mark.parametrize("mask", range(8))
@pytest.mark.parametrize("shape", CASES)
def test_grid_tier_equals_brute_force(orc, mask, shape):
    log2, F = shape
    rng = np.random.default_rng(2000 + mask * 10 + F)
    L = orc.Lattice(log2, F, mask)
    n = 300
    pts = _tiny(rng, log2, F, mask, n, outside=True)
    E = 1 << F
    for flags in (0, orc.EXCLUDE_SELF):
        r = rng.integers(0, 6 * E, n).astype(np.uint32)
        r[:5] = 0
        a = orc.radius_brute(L, pts, r, flags=flags)
        b = orc.Grid(L, pts).radius(r, flags=flags)
        np.testing.assert_array_equal(a.row_ptr, b.row_ptr)
        np.testing.assert_array_equal(a.ids, b.ids)
        np.testing.assert_array_equal(a.dist2, b.dist2)
    # explicit query centres, some outside the region on clipped axes
    qs = _tiny(rng, log2, F, mask, 64, outside=True)
    r = rng.integers(0, 6 * E, 64).astype(np.uint32)
    a = orc.radius_brute(L, pts, r, queries=qs)
    b = orc.Grid(L, pts).radius(r, queries=qs)
    np.testing.assert_array_equal(a.row_ptr, b.row_ptr)
    np.testing.assert_array_equal(a.ids, b.ids)


def _histogram_by_definition(log2, F, mask, pts):
    """Objects per cell, written from the definitions: on a cyclic axis the
    coordinate is taken modulo the world width, a cell index is the
    coordinate shifted right by F (Section II.B), cells are packed z-major;
    an object with a clipped coordinate at or beyond the world width lives
    in the one outside cell (index = number of cells); an object with a
    clipped coordinate >= 2^30 is unusable and in no cell."""
    L = [1 << v for v in log2]
    ncells = L[0] * L[1] * L[2]
    hist = np.zeros(ncells + 1, dtype=np.int64)
    for j in range(len(pts[0])):
        c, out, bad = [], False, False
        for a in range(3):
            v = int(pts[a][j])
            W = L[a] << F
            if (mask >> a) & 1:
                v %= W
            elif v >= 1 << 30:
                bad = True
            elif v >= W:
                out = True
            c.append(v >> F)
        if bad:
            continue
        hist[ncells if out else (c[2] * L[1] + c[1]) * L[0] + c[0]] += 1
    return hist


@pytest.mark.parametrize("mask", range(8))
@pytest.mark.parametrize("shape", CASES)
def test_grid_counts_are_the_cell_histogram(orc, mask, shape):
    """The oracle grid's per-cell counts (the histogram the lattice rebuild is
    checked against) equal a histogram taken straight from the definitions,
    with objects outside the region and unusable ones included."""
    log2, F = shape
    rng = np.random.default_rng(5000 + mask * 10 + F)
    pts = _tiny(rng, log2, F, mask, 400, outside=True)
    g = orc.Grid(orc.Lattice(log2, F, mask), pts)
    got = g.counts()
    g.close()
    want = _histogram_by_definition(log2, F, mask, pts)
    np.testing.assert_array_equal(got.astype(np.int64), want)
    n_bad = sum(1 for j in range(len(pts[0]))
                if any(not (mask >> a) & 1 and int(pts[a][j]) >= 1 << 30 for a in range(3)))
    assert int(got.sum()) == len(pts[0]) - n_bad


@pytest.mark.parametrize("mask", range(8))
@pytest.mark.parametrize("shape", CASES)
def test_radius_counts_equal_brute_force_row_sizes(orc, mask, shape):
    """Row sizes without the rows (the neighbour-count checksum's input) equal
    the row lengths of the brute-force tier, all agents with and without the
    own object, and explicit centres (some outside the region)."""
    log2, F = shape
    rng = np.random.default_rng(6000 + mask * 10 + F)
    L = orc.Lattice(log2, F, mask)
    n = 300
    pts = _tiny(rng, log2, F, mask, n, outside=True)
    E = 1 << F
    g = orc.Grid(L, pts)
    for flags in (0, orc.EXCLUDE_SELF):
        r = rng.integers(0, 6 * E, n).astype(np.uint32)
        r[:5] = 0
        a = orc.radius_brute(L, pts, r, flags=flags)
        np.testing.assert_array_equal(g.radius_counts(r, flags=flags), np.diff(a.row_ptr))
    qs = _tiny(rng, log2, F, mask, 64, outside=True)
    r = rng.integers(0, 6 * E, 64).astype(np.uint32)
    a = orc.radius_brute(L, pts, r, queries=qs)
    np.testing.assert_array_equal(g.radius_counts(r, queries=qs), np.diff(a.row_ptr))
    g.close()


@pytest.mark.parametrize("mask", [0, 3, 7])
@pytest.mark.parametrize("shape", CASES)
def test_knn_tiers_agree(orc, mask, shape):
    log2, F = shape
    rng = np.random.default_rng(3000 + mask * 10 + F)
    L = orc.Lattice(log2, F, mask)
    n = 300
    pts = _tiny(rng, log2, F, mask, n, outside=True)
    E = 1 << F
    k = rng.integers(0, 40, n).astype(np.uint32)
    rmax = rng.integers(0, 8 * E, n).astype(np.uint32)
    a = orc.knn_brute(L, pts, k, rmax)
    g = orc.Grid(L, pts)
    b = g.knn(k, rmax)
    np.testing.assert_array_equal(a.row_ptr, b.row_ptr)
    np.testing.assert_array_equal(a.ids, b.ids)
    np.testing.assert_array_equal(a.dist2, b.dist2)
    # every K-NN row is the prefix of the radius row at the cap
    full = g.radius(rmax)
    for i in range(n):
        ids, d2 = b.row(i)
        fi, fd = full.row(i)
        m = min(int(k[i]), len(fi))
        assert len(ids) == m
        np.testing.assert_array_equal(ids, fi[:m])
    # a mixed batch equals its two halves
    kk = np.where(rng.random(n) < 0.5, k, 0).astype(np.uint32)
    mixed = g.mixed(kk, rmax)
    for i in range(0, n, 7):
        src = b if kk[i] > 0 else full
        np.testing.assert_array_equal(mixed.row(i)[0], src.row(i)[0])


def test_radius_rows_are_sorted_and_unique(orc):
    rng = np.random.default_rng(9)
    L = orc.Lattice((3, 3, 3), 3, 7)
    pts = _tiny(rng, (3, 3, 3), 3, 7, 500, outside=False)
    out = orc.Grid(L, pts).radius(np.full(500, 20, dtype=np.uint32))
    for i in range(500):
        ids, d2 = out.row(i)
        key = list(zip(d2.tolist(), ids.tolist()))
        assert key == sorted(key)
        assert len(set(ids.tolist())) == len(ids)


# ---------------------------------------------------------------------------
# Counter-based generator and the moving-agent step

def test_mix64_published_splitmix64_outputs(orc):
    # SplitMix64 seeded with 0 (state advanced by the golden gamma before
    # each output) yields e220a8397b1dcdaf, 6e789e6aa1b965f4, 06c45d188009454f.
    g = 0x9E3779B97F4A7C15
    exp = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    for k, e in enumerate(exp, start=1):
        assert orc.mix64((k * g) & (2 ** 64 - 1)) == e


def test_synth_generator_matches_oracle_hash(orc):
    from paper_cs_0608108_amd import synth
    i = np.arange(0, 1000, 37, dtype=np.uint64)
    got = synth.H(12345, 7, i)
    for a, b in zip(i.tolist(), got.tolist()):
        assert orc.hash64(12345, 7, a) == b


def test_move_displacement_bounded_uniform_and_wrapped(orc):
    L = orc.Lattice((4, 4, 4), 8, 7)
    W = 16 << 8
    n = 20000
    rng = np.random.default_rng(4)
    pts = tuple(rng.integers(0, W, n).astype(np.uint32) for _ in range(3))
    pts[0][:10] = 0
    pts[0][10:20] = W - 1
    nx = orc.move(L, 4, 0, pts)
    dmax = (1 << 8) // 4
    for a in range(3):
        d = (nx[a].astype(np.int64) - pts[a].astype(np.int64) + W // 2) % W - W // 2
        assert d.min() == -dmax and d.max() == dmax
        assert (nx[a] < W).all()
        hist = np.bincount(d + dmax, minlength=2 * dmax + 1)
        exp = n / (2 * dmax + 1)
        chi2 = float(((hist - exp) ** 2 / exp).sum())
        assert chi2 < 2 * (2 * dmax + 1)  # loose: ~ dof +- several sigma
    # different steps draw different displacements
    nx2 = orc.move(L, 4, 1, pts)
    assert not np.array_equal(nx[0], nx2[0])


def test_count_checksum_definition(orc):
    rp = np.array([0, 3, 3, 10], dtype=np.int64)
    s, h = orc.count_checksum(rp)
    assert s == 10
    exp = (orc.mix64((0 << 32) | 3) + orc.mix64((1 << 32) | 0) + orc.mix64((2 << 32) | 7)) % 2 ** 64
    assert h == exp


@pytest.mark.parametrize("log2,mask", [((2, 2, 2), 0), ((3, 3, 3), 7), ((3, 2, 3), 5)])
def test_cells_touched_equal_cells_of_brute_force_neighbours(orc, log2, mask):
    # Put an object at every integer position of the region: then a cell meets
    # the sphere iff it holds a neighbour, and lies wholly inside iff all of
    # its positions are neighbours.  Brute force gives both sets exactly.
    F = 2
    e = 1 << F
    L = orc.Lattice(log2, F, mask)
    W = [(1 << v) * e for v in log2]
    g = np.meshgrid(*[np.arange(w) for w in W], indexing="ij")
    pts = tuple(a.ravel().astype(np.uint32) for a in g)
    rng = np.random.default_rng(sum(log2) + mask)
    nq = 24
    q = [rng.integers(0, W[a], nq).astype(np.uint32) for a in range(3)]
    q[0][:4] = 0
    q[1][4:8] = W[1] - 1
    lim = min(((1 << v) // 2 - 1) * e for a, v in enumerate(log2) if (mask >> a) & 1) if mask else 3 * e
    r = rng.integers(0, lim + 1, nq).astype(np.uint32)
    kept, inter, cube = orc.cells_touched(L, q, r)
    res = orc.radius_brute(L, pts, r, queries=q)
    for i in range(nq):
        ids, _ = res.row(i)
        cells = np.stack([pts[a][ids] >> F for a in range(3)], axis=1)
        uniq, cnt = np.unique(cells, axis=0, return_counts=True)
        assert kept[i] == len(uniq)
        assert inter[i] == int((cnt == e ** 3).sum())
        assert cube[i] == orc.cube_cells(L, [q[0][i], q[1][i], q[2][i]], int(r[i]))


def test_cells_touched_undefined_beyond_the_cyclic_radius_limit(orc):
    # On a cyclic axis the cube must not wrap onto itself: ceil(r / 2^F) <= L/2 - 1.
    L = orc.Lattice((3, 3, 3), F16, 7)
    q = [np.array([5 * E16 + 7], dtype=np.uint32)] * 3
    ok = orc.cells_touched(L, q, np.array([3 * E16], dtype=np.uint32))
    bad = orc.cells_touched(L, q, np.array([3 * E16 + 1], dtype=np.uint32))
    assert ok[0][0] > 0 and bad[0][0] == -1
