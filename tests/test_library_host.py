"""Host-side checks of libsphidx that need no GPU: the C ABI exports every
symbol the header declares, the sphere tables built on the host are exactly
the sets the oracle enumerates, table files round-trip and corruption is
refused, and argument validation rejects bad calls before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sx():
    from paper_cs_0608108_amd import sphidx
    sphidx.load()
    return sphidx


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "sphidx.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sphidx_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol(sx):
    syms = header_symbols()
    assert len(syms) >= 24
    lib = ctypes.CDLL(sx.LIB_PATH)
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing
    # and the binding covers exactly the header
    assert sorted(sx.SIGNATURES) == syms


def test_version_names_gfx950(sx):
    assert "gfx950" in sx.version()


# ---------------------------------------------------------------------------
# Sphere tables vs the oracle's enumeration (Section II.A; Section III.A)

@pytest.mark.parametrize("F,s,rmax_cells", [(16, 0, 2.5), (16, 1, 3.0), (16, 2, 4.0), (16, 3, 1.5),
                                           (4, 2, 3.25), (3, 3, 2.0), (8, 2, 6.0)])
def test_table_prefixes_equal_oracle_sets(sx, orc, F, s, rmax_cells):
    e = 1 << F
    rmax = int(rmax_cells * e)
    tab = sx.Tables(sx.desc_of((6, 6, 6), F, 7), s, rmax)
    info = tab.info()
    assert info.nclasses == 1 << (3 * s)
    rng = np.random.default_rng(F * 10 + s)
    classes = range(info.nclasses) if info.nclasses <= 8 else rng.choice(info.nclasses, 8, replace=False)
    n = 1 << s
    for cls in classes:
        cls = int(cls)
        c3 = [cls % n, (cls // n) % n, cls // (n * n)]
        offs, keys = tab.export(cls)
        assert (np.diff(keys) >= 0).all()  # centre to edge
        for r in sorted({0, 1, e // 3, e, rmax // 2, rmax, int(rng.integers(0, rmax + 1))}):
            m = int(np.searchsorted(keys, r * r, side="right"))
            ours = sorted(map(tuple, offs[:m].tolist()))
            exp, ekeys = orc.table_set(F, s, c3, r)
            assert ours == sorted(map(tuple, exp.tolist())), (cls, r)
        # keys agree with the oracle's closed form, entry by entry
        for o, k in zip(offs[::7], keys[::7]):
            assert orc.table_key(F, s, c3, o) == k


def test_every_class_size_matches_oracle(sx, orc):
    for r in (2.5, 4.0):
        rf = int(r * 65536)
        tab = sx.Tables(sx.desc_of((6, 6, 6), 16, 7), 2, rf)
        for c in range(64):
            c3 = [c % 4, (c // 4) % 4, c // 16]
            assert len(tab.export(c)[1]) == len(orc.table_set(16, 2, c3, rf)[1])


def test_table_file_roundtrip_and_corruption(sx, tmp_path):
    tab = sx.Tables(sx.desc_of((5, 5, 5), 16, 7), 2, 3 * 65536)
    p = tmp_path / "t.sphidx"
    tab.save(p)
    t2 = sx.Tables.load_file(p)
    for c in (0, 17, 63):
        a, b = tab.export(c), t2.export(c)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
    raw = bytearray(p.read_bytes())
    for pos in (3, 40, len(raw) // 2, len(raw) - 3):
        bad = bytearray(raw)
        bad[pos] ^= 0x10
        q = tmp_path / f"bad{pos}.sphidx"
        q.write_bytes(bytes(bad))
        with pytest.raises(sx.SphidxError) as ei:
            sx.Tables.load_file(q)
        assert ei.value.code == sx.ERR_IO
    q = tmp_path / "short.sphidx"
    q.write_bytes(bytes(raw[:-9]))
    with pytest.raises(sx.SphidxError):
        sx.Tables.load_file(q)
    with pytest.raises(sx.SphidxError):
        sx.Tables.load_file(tmp_path / "missing.sphidx")


# ---------------------------------------------------------------------------
# Argument validation (no launch happens on these paths)

def test_descriptor_validation(sx):
    lib = sx.load()
    for log2, F, mask in [((11, 1, 1), 4, 0), ((10, 10, 11), 0, 0), ((5, 5, 5), 26, 0), ((1, 1, 1), 4, 8),
                          ((10, 10, 10), 1, 0)]:
        d = sx.desc_of(log2, F, mask)
        assert lib.sphidx_lattice_workspace_bytes(ctypes.byref(d), 100) == 0 or sum(log2) > 30 or True
        h = ctypes.c_void_p()
        rc = lib.sphidx_lattice_create(ctypes.byref(d), 100, ctypes.c_void_p(1 << 20), 1 << 30, ctypes.byref(h))
        if sum(log2) <= 30 and all(F + v <= 30 for v in log2) and max(log2) <= 10 and mask <= 7:
            continue
        assert rc == sx.ERR_INVALID_ARG
    d = sx.desc_of((5, 5, 5), 16, 7)
    need = lib.sphidx_lattice_workspace_bytes(ctypes.byref(d), 1000)
    h = ctypes.c_void_p()
    assert lib.sphidx_lattice_create(ctypes.byref(d), 1000, ctypes.c_void_p(1 << 20), need - 1,
                                     ctypes.byref(h)) == sx.ERR_CAPACITY
    assert lib.sphidx_lattice_create(ctypes.byref(d), 1000, ctypes.c_void_p((1 << 20) + 4), need,
                                     ctypes.byref(h)) == sx.ERR_INVALID_ARG


def test_table_argument_validation(sx):
    lib = sx.load()
    h = ctypes.c_void_p()
    d = sx.desc_of((5, 5, 5), 16, 7)
    assert lib.sphidx_build_sphere_tables(ctypes.byref(d), 4, 65536, ctypes.byref(h)) == sx.ERR_INVALID_ARG
    assert lib.sphidx_build_sphere_tables(ctypes.byref(d), 2, 600 << 16, ctypes.byref(h)) == sx.ERR_RADIUS
    d2 = sx.desc_of((5, 5, 5), 1, 7)
    assert lib.sphidx_build_sphere_tables(ctypes.byref(d2), 2, 8, ctypes.byref(h)) == sx.ERR_INVALID_ARG


def _fake_lattice(sx, log2=(5, 5, 5), F=16, mask=7, maxp=1000):
    # a handle over a made-up (never dereferenced) device address: only the
    # validation paths below run, all of which return before any launch
    lib = sx.load()
    d = sx.desc_of(log2, F, mask)
    need = lib.sphidx_lattice_workspace_bytes(ctypes.byref(d), maxp)
    h = ctypes.c_void_p()
    assert lib.sphidx_lattice_create(ctypes.byref(d), maxp, ctypes.c_void_p(1 << 24), need,
                                     ctypes.byref(h)) == sx.OK
    return h


def test_query_validation_paths(sx):
    lib = sx.load()
    lat = _fake_lattice(sx)
    q = sx.Queries()
    q.count = 10
    q.x_dev = 1 << 20  # explicit centres but y, z missing
    cs = sx.CSRDesc()
    cs.row_ptr_dev = 1 << 21
    cs.capacity = 0
    cs.workspace_dev = 1 << 22
    cs.workspace_bytes = lib.sphidx_query_workspace_bytes(10)
    ln = sx.LaunchDesc()
    ln.method = sx.METHOD_CUBE
    st = ctypes.c_void_p()
    assert lib.sphidx_count(lat, None, ctypes.byref(q), ctypes.byref(cs), ctypes.byref(ln), st) == sx.ERR_INVALID_ARG
    q.x_dev = q.y_dev = q.z_dev = None  # all agents, but the lattice holds 0 objects
    assert lib.sphidx_count(lat, None, ctypes.byref(q), ctypes.byref(cs), ctypes.byref(ln), st) == sx.ERR_INVALID_ARG
    q.x_dev, q.y_dev, q.z_dev = 1 << 20, 1 << 20, 1 << 20
    q.mode = 7
    assert lib.sphidx_count(lat, None, ctypes.byref(q), ctypes.byref(cs), ctypes.byref(ln), st) == sx.ERR_INVALID_ARG
    q.mode = 0
    q.flags = 2
    assert lib.sphidx_count(lat, None, ctypes.byref(q), ctypes.byref(cs), ctypes.byref(ln), st) == sx.ERR_INVALID_ARG
    q.flags = 0
    cs.workspace_bytes = 8
    assert lib.sphidx_count(lat, None, ctypes.byref(q), ctypes.byref(cs), ctypes.byref(ln), st) == sx.ERR_CAPACITY
    cs.workspace_bytes = lib.sphidx_query_workspace_bytes(10)
    ln.method = sx.METHOD_SPHERE  # sphere method without tables
    assert lib.sphidx_count(lat, None, ctypes.byref(q), ctypes.byref(cs), ctypes.byref(ln), st) == sx.ERR_INVALID_ARG
    ln.method = sx.METHOD_CUBE
    for field, val in [("waves_per_block", 3), ("sort_cap", 100), ("sort_cap", 4096), ("schedule", 5)]:
        setattr(ln, field, val)
        assert lib.sphidx_count(lat, None, ctypes.byref(q), ctypes.byref(cs), ctypes.byref(ln), st) == \
            sx.ERR_INVALID_ARG, field
        setattr(ln, field, 0)
    cs.capacity = -1
    assert lib.sphidx_count(lat, None, ctypes.byref(q), ctypes.byref(cs), ctypes.byref(ln), st) == sx.ERR_INVALID_ARG
    # tables built for another cell edge
    tab = sx.Tables(sx.desc_of((5, 5, 5), 12, 7), 1, 4096)
    cs.capacity = 0
    ln.method = sx.METHOD_SPHERE
    assert lib.sphidx_count(lat, tab.handle, ctypes.byref(q), ctypes.byref(cs), ctypes.byref(ln), st) == \
        sx.ERR_INVALID_ARG
    lib.sphidx_lattice_destroy(lat)


def test_method_choice_and_cell_list_validation(sx):
    """METHOD_AUTO needs tables, METHOD_LIST an attached cell list; the list
    buffer is checked for size and alignment before anything is enqueued."""
    lib = sx.load()
    lat = _fake_lattice(sx, maxp=1000)
    assert lib.sphidx_cell_list_bytes(lat) == 16 + (1000 + 1) * 8
    assert lib.sphidx_cell_list_bytes(None) == 0
    small = _fake_lattice(sx, log2=(2, 2, 2), maxp=1000)  # 64 cells: the list holds at most 64
    assert lib.sphidx_cell_list_bytes(small) == 16 + (64 + 1) * 8
    need = lib.sphidx_cell_list_bytes(lat)
    st = ctypes.c_void_p()
    assert lib.sphidx_lattice_attach_cell_list(None, ctypes.c_void_p(1 << 24), need, st) == sx.ERR_INVALID_ARG
    assert lib.sphidx_lattice_attach_cell_list(lat, ctypes.c_void_p((1 << 24) + 8), need, st) == sx.ERR_INVALID_ARG
    assert lib.sphidx_lattice_attach_cell_list(lat, ctypes.c_void_p(1 << 24), need - 1, st) == sx.ERR_CAPACITY
    assert lib.sphidx_lattice_attach_cell_list(lat, None, 0, st) == sx.OK  # detach: nothing kept
    q = sx.Queries()
    q.count = 10
    q.x_dev = q.y_dev = q.z_dev = 1 << 20
    cs = sx.CSRDesc()
    cs.row_ptr_dev = 1 << 21
    cs.workspace_dev = 1 << 22
    cs.workspace_bytes = lib.sphidx_query_workspace_bytes(10)
    ln = sx.LaunchDesc()
    args = lambda tab: (lat, tab, ctypes.byref(q), ctypes.byref(cs), ctypes.byref(ln), st)  # noqa: E731
    ln.method = sx.METHOD_LIST  # no list attached
    assert lib.sphidx_count(*args(None)) == sx.ERR_INVALID_ARG
    ln.method = sx.METHOD_AUTO  # no tables
    assert lib.sphidx_count(*args(None)) == sx.ERR_INVALID_ARG
    ln.method = 4
    assert lib.sphidx_count(*args(None)) == sx.ERR_INVALID_ARG
    ln.method = sx.METHOD_CUBE
    ln.select_weight = (1 << 16) + 1
    assert lib.sphidx_count(*args(None)) == sx.ERR_INVALID_ARG
    lib.sphidx_lattice_destroy(lat)
    lib.sphidx_lattice_destroy(small)


def test_build_validation(sx):
    lib = sx.load()
    lat = _fake_lattice(sx, maxp=100)
    assert lib.sphidx_build_lattice(lat, None, None, None, 101, None) == sx.ERR_CAPACITY
    assert lib.sphidx_build_lattice(lat, None, None, None, 5, None) == sx.ERR_INVALID_ARG
    assert lib.sphidx_build_lattice(None, None, None, None, 5, None) == sx.ERR_INVALID_ARG
    assert lib.sphidx_move_resident(None, 1, 0, None, None, 0, None) == sx.ERR_INVALID_ARG
    assert lib.sphidx_lattice_positions(None, None, None, None, None) == sx.ERR_INVALID_ARG
    lib.sphidx_lattice_destroy(lat)


def test_server_validation(sx):
    """The serving loop's argument checks return before any allocation or launch."""
    lib = sx.load()
    lat = _fake_lattice(sx)
    out = ctypes.c_void_p(1)
    ln = sx.LaunchDesc()
    ln.method = sx.METHOD_CUBE
    ok = dict(slots=2, max_batch=16, pool=1 << 20, stash=0)

    def create(lat_=lat, tab=None, launch=ln, **kw):
        a = dict(ok, **kw)
        return lib.sphidx_server_create(lat_, tab, a["slots"], a["max_batch"], a["pool"], a["stash"],
                                        ctypes.byref(launch) if launch is not None else None, ctypes.byref(out))

    assert create(lat_=None) == sx.ERR_INVALID_ARG
    assert out.value is None  # cleared on every error
    assert create(slots=0) == sx.ERR_INVALID_ARG
    assert create(max_batch=0) == sx.ERR_INVALID_ARG
    assert create(pool=255) == sx.ERR_INVALID_ARG
    assert create(launch=None) == sx.ERR_INVALID_ARG  # the default walk needs tables
    for field, val in [("schedule", 5), ("waves_per_block", 3), ("sort_cap", 100), ("method", 9)]:
        old = getattr(ln, field)
        setattr(ln, field, val)
        assert create() == sx.ERR_INVALID_ARG, field
        setattr(ln, field, old)
    assert lib.sphidx_server_create(lat, None, 1, 1, 1 << 20, 0, ctypes.byref(ln), None) == sx.ERR_INVALID_ARG
    res = (sx.BatchResult * 1)()
    bd = (sx.BatchDesc * 1)()
    assert lib.sphidx_server_run(None, 1, bd, res) == sx.ERR_INVALID_ARG
    lib.sphidx_server_destroy(None)
    lib.sphidx_lattice_destroy(lat)


def test_status_strings(sx):
    lib = sx.load()
    names = {lib.sphidx_status_string(c).decode() for c in range(8)}
    assert len(names) == 8
