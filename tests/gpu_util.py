"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare it with the oracle, element by element."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lattice(sx, log2, F, mask, pts, cell_list=True):
    """A built lattice; with cell_list, its non-empty cell list is kept too
    (which only METHOD_AUTO and METHOD_LIST read)."""
    n = len(pts[0])
    lat = sx.Lattice(log2, F, mask, max(n, 1))
    if cell_list:
        lat.attach_cell_list()
    dev = tuple(sx.to_dev_u32(a) for a in pts)
    lat.build(*dev)
    lat._pts_dev = dev  # keep alive
    return lat


def per_query(sx, v):
    if v is None:
        return None
    if np.ndim(v) == 0:
        return int(v)
    return sx.to_dev_u32(np.asarray(v, dtype=np.uint32))


def run(sx, lat, tab, r, k=None, mode=0, queries=None, flags=0, launch=None, want_dist2=True, stash=False):
    Q = lat.n if queries is None else len(queries[0])
    cen = None if queries is None else tuple(sx.to_dev_u32(a) for a in queries)
    rad = per_query(sx, r)
    kk = per_query(sx, k)
    q = sx.make_queries(Q, cen, rad, kk, mode, flags)
    out = sx.run(lat, tab, q, launch, want_dist2=want_dist2, stash=stash)
    del cen, rad, kk
    return out


def assert_same(gpu, ref, what=""):
    rp, ids, d2 = gpu
    assert len(rp) == len(ref.row_ptr), what
    bad = np.nonzero(rp != ref.row_ptr)[0]
    if len(bad):
        i = bad[0]
        raise AssertionError(f"{what}: row_ptr differs first at {i}: {rp[i]} vs {ref.row_ptr[i]}")
    if not np.array_equal(ids, ref.ids):
        j = int(np.nonzero(ids != ref.ids)[0][0])
        row = int(np.searchsorted(ref.row_ptr, j, side="right") - 1)
        raise AssertionError(f"{what}: ids differ at {j} (row {row}): gpu {ids[j]} vs oracle {ref.ids[j]}; "
                             f"gpu row {ids[ref.row_ptr[row]:ref.row_ptr[row + 1]][:12]} "
                             f"oracle {ref.ids[ref.row_ptr[row]:ref.row_ptr[row + 1]][:12]}")
    if d2 is not None:
        assert np.array_equal(d2, ref.dist2), what


def tiny_points(rng, log2, F, mask, n, outside=False, invalid=False):
    pts = []
    for a in range(3):
        W = (1 << log2[a]) << F
        if (mask >> a) & 1:
            v = rng.integers(0, 1 << 32, n, dtype=np.uint64)
            v[: n // 3] = rng.integers(0, W, n // 3)
        else:
            v = rng.integers(0, W, n, dtype=np.uint64)
            if outside and n >= 16:
                k = n // 10
                v[:k] = rng.integers(W, 2 * W + 5, k)
            if invalid and n >= 16:
                v[n // 10:n // 10 + 2] = [1 << 30, (1 << 32) - 1]
        pts.append(v.astype(np.uint32))
    if n >= 8:
        for a in range(3):
            pts[a][-2] = pts[a][-3]                     # duplicate
            pts[a][-4] = (pts[a][-4] >> F) << F         # on a cell boundary
    return tuple(pts)
