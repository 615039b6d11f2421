"""Table designs compared on the host (Section II.A, III.A; more dimensions,
Sections I and V): the census of cells each design walks, pinned against the
paper's printed counts, the oracle's kept cells, cubes and table sets, the
paper's own claims (below one cell the specialised tables walk the
bin-lattice's cells; the ball/cube ratio falls with the dimension), and the
soundness of every rejection (no exact cell is ever left out)."""
import math

import numpy as np
import pytest

from goldens import read_matrix, read_pairs


@pytest.fixture(scope="module")
def sx():
    from paper_cs_0608108_amd import sphidx
    sphidx.load()
    return sphidx


def test_unshaved_counts_match_the_paper(sx):
    """Section II.A: 27, 54, 36, 8, 54 cells at b^2 = 0..4 in three dimensions,
    and the 2-D table of Fig. 2."""
    exp3 = read_pairs("shell_counts_3d.txt")
    _, _, h3 = sx.table_census_nd(3, 8, 0, 256, hist_len=5)
    assert {k: int(v) for k, v in enumerate(h3)} == exp3
    fig2 = read_matrix("fig2_min_bound_2d.txt")  # offsets -4..4: every entry b^2 <= 9 is in it
    _, _, h2 = sx.table_census_nd(2, 8, 0, 256, hist_len=10)
    want = np.bincount(fig2[fig2 < 10].ravel(), minlength=10)
    assert np.array_equal(h2, want)


def _queries(rng, F, n, rmax_cells):
    e = 1 << F
    f = [rng.integers(0, e, n).astype(np.uint32) for _ in range(3)]
    # some positions on the faces of the home cell, some radii on cell multiples
    f[0][:n // 10] = 0
    f[1][n // 10:n // 5] = e - 1
    r = rng.integers(0, rmax_cells * e, n).astype(np.uint32)
    r[:n // 8] = (r[:n // 8] // e) * e
    return f, r


def test_census_exact_and_cube_equal_the_oracle(sx, orc):
    """The exact and cube counts are the oracle's kept cells and bin-lattice
    cube for the same centres, placed inside a wrapping 32^3 world far from
    any wrap."""
    rng = np.random.default_rng(21)
    F = 10
    tab = sx.Tables(sx.desc_of((5, 5, 5), F, 7), 2, 8 << F)
    f, r = _queries(rng, F, 600, 8)
    c = sx.table_census(tab, f, r)
    cell = rng.integers(0, 32, (3, len(r)))
    q = tuple((cell[a].astype(np.uint64) << F | f[a]).astype(np.uint32) for a in range(3))
    kept, _, cube = orc.cells_touched(orc.Lattice((5, 5, 5), F, 7), q, r)
    assert np.array_equal(c["exact"], kept)
    assert np.array_equal(c["cube"], cube)


def test_census_subcell_prefix_is_the_oracle_table_set(sx, orc):
    rng = np.random.default_rng(22)
    F, s = 8, 2
    tab = sx.Tables(sx.desc_of((5, 5, 5), F, 7), s, 6 << F)
    f, r = _queries(rng, F, 120, 6)
    c = sx.table_census(tab, f, r)
    for i in range(len(r)):
        cls = [int(f[a][i]) >> (F - s) for a in range(3)]
        offs, _ = orc.table_set(F, s, cls, int(r[i]))
        assert c["subcell"][i] == len(offs), i


def test_census_orders_and_no_exact_cell_dropped(sx):
    rng = np.random.default_rng(23)
    F = 10
    tab = sx.Tables(sx.desc_of((5, 5, 5), F, 7), 2, 12 << F)
    f, r = _queries(rng, F, 3000, 12)
    c = sx.table_census(tab, f, r)
    assert (c["dropped"] == 0).all()
    assert (c["exact"] <= c["paper64_eq1"]).all()
    assert (c["paper64_eq1"] <= c["paper64"]).all()
    assert (c["paper64"] <= c["unshaved"]).all()
    assert (c["exact"] <= c["subcell"]).all() and (c["subcell"] <= c["unshaved"]).all()
    assert (c["exact"] <= c["cube"]).all()
    # the shaving does cut: on average fewer cells than the unshaved table
    assert c["paper64"].mean() < c["unshaved"].mean()
    assert c["paper64_eq1"].mean() < c["paper64"].mean()


def test_below_one_cell_the_specialised_tables_walk_the_cube(sx):
    """Section III.A: with the one-direction rule the sphere walk considers the
    same cells out of the 27 as the bin-lattice, for d < 1 (a radius equal to
    a lower-face distance is the one tie: the paper's real-valued face sits
    at f, the integer one at f + 1)."""
    rng = np.random.default_rng(24)
    F = 10
    e = 1 << F
    tab = sx.Tables(sx.desc_of((5, 5, 5), F, 7), 2, 2 * e)
    f = [rng.integers(0, e, 4000).astype(np.uint32) for _ in range(3)]
    r = rng.integers(0, e, 4000).astype(np.uint32)
    c = sx.table_census(tab, f, r)
    tie = (r[:, None] == np.stack(f, 1)).any(1)
    assert (c["paper64"][~tie] == c["cube"][~tie]).all()
    assert (c["unshaved"] == 27).all()


@pytest.mark.parametrize("dims,limit", [(2, math.pi / 4), (3, math.pi / 6), (4, math.pi ** 2 / 32)])
def test_ball_to_cube_ratio_falls_with_radius_towards_the_volume_ratio(sx, dims, limit):
    """Section I: the sphere/cube ratio tends to the volume ratio of the ball
    and its cube, about 52 % in three dimensions and 31 % in four."""
    ratios = []
    for rc in (4, 8, 16):
        s, cube, _ = sx.table_census_nd(dims, 8, 1, rc << 8)
        ratios.append(s / cube)
    assert ratios[0] > ratios[1] > ratios[2] > limit
    assert ratios[2] < limit * 1.25


def test_ratio_falls_with_the_dimension(sx):
    got = [sx.table_census_nd(d, 8, 1, 12 << 8)[0] / sx.table_census_nd(d, 8, 1, 12 << 8)[1] for d in (2, 3, 4)]
    assert got[0] > got[1] > got[2]


def test_census_argument_checks(sx):
    tab = sx.Tables(sx.desc_of((5, 5, 5), 8, 7), 1, 2 << 8)
    with pytest.raises(sx.SphidxError):
        sx.table_census(tab, ([256], [0], [0]), [10])  # position outside the home cell
    with pytest.raises(sx.SphidxError):
        sx.table_census(tab, ([0], [0], [0]), [3 << 8])  # above the tables' cap
    with pytest.raises(sx.SphidxError):
        sx.table_census_nd(5, 8, 1, 256)
    with pytest.raises(sx.SphidxError):
        sx.table_census_nd(4, 8, 3, 64 << 8)  # too many cell visits
