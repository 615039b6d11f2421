"""CPU oracle for spherical-indexing neighbourhood queries (Brodu, arXiv cs/0608108).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library in ``paper_cs_0608108_amd``.
It shares no code with the HIP path.  The arithmetic lives in ``oracle.c``
(plain C99, exact integer math); this module only marshals numpy arrays.

Definitions followed (see the C file for the per-function citations):
  * radius query: objects at distance <= d from the centre (Section II.A),
    rows ordered by (squared distance, id);
  * K nearest: the first min(K, |R|) entries of the radius result at the
    search cap (Section II.A, last paragraph);
  * tier 0 = every query against every object (Section I, naive query);
    tier 1 = bin-lattice bounding-cube scan over a plain grid (Section I,
    Section III.C).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EXCLUDE_SELF = 1


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc + OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
             _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(ctypes.Structure):
    _fields_ = [("log2_cells", ctypes.c_uint32 * 3), ("frac_bits", ctypes.c_uint32),
                ("cyclic_mask", ctypes.c_uint32)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P, U32, I64, U64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int64, ctypes.c_uint64
    D = ctypes.POINTER(_Desc)
    sig = {
        "orc_radius_brute": (P, [D, U32, P, P, P, U32, P, P, P, P, U32]),
        "orc_radius_images": (P, [D, U32, P, P, P, U32, P, P, P, P, U32]),
        "orc_knn_brute": (P, [D, U32, P, P, P, U32, P, P, P, P, P, U32]),
        "orc_grid_build": (P, [D, U32, P, P, P]),
        "orc_grid_free": (None, [P]),
        "orc_grid_counts": (None, [P, P]),
        "orc_grid_radius": (P, [P, U32, P, P, P, P, U32]),
        "orc_grid_radius_counts": (None, [P, U32, P, P, P, P, U32, P]),
        "orc_grid_knn": (P, [P, U32, P, P, P, P, P, U32]),
        "orc_grid_mixed": (P, [P, U32, P, P, P, P, P, U32]),
        "orc_result_total": (I64, [P]),
        "orc_result_copy": (None, [P, P, P, P]),
        "orc_result_free": (None, [P]),
        "orc_cells_touched": (None, [D, U32, P, P, P, P, P, P, P]),
        "orc_base_minbound2": (I64, [ctypes.c_int, P]),
        "orc_table_key": (I64, [U32, U32, P, P]),
        "orc_table_key_brute": (I64, [U32, U32, P, P]),
        "orc_table_set": (I64, [U32, U32, P, U32, P, P]),
        "orc_mix64": (U64, [U64]),
        "orc_hash": (U64, [U64, U64, U64]),
        "orc_move": (None, [D, U64, U32, U32, P, P, P]),
        "orc_count_checksum": (None, [P, U32, P]),
        "orc_num_threads": (ctypes.c_int, []),
        "orc_set_num_threads": (None, [ctypes.c_int]),
        "orc_cube_cells": (I64, [D, P, U32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


@dataclass(frozen=True)
class Lattice:
    """Power-of-two cubic-cell lattice (Section II.B): cells per axis
    ``2**log2_cells[a]``, cell edge ``2**frac_bits`` fixed-point units, axis
    ``a`` cyclic when bit ``a`` of ``cyclic_mask`` is set."""
    log2_cells: tuple
    frac_bits: int
    cyclic_mask: int

    def c(self):
        d = _Desc()
        for a in range(3):
            d.log2_cells[a] = int(self.log2_cells[a])
        d.frac_bits = int(self.frac_bits)
        d.cyclic_mask = int(self.cyclic_mask)
        return d


@dataclass
class CSR:
    row_ptr: np.ndarray  # int64 [Q+1]
    ids: np.ndarray      # uint32 [P]
    dist2: np.ndarray    # int64 [P]

    def row(self, i):
        b, e = self.row_ptr[i], self.row_ptr[i + 1]
        return self.ids[b:e], self.dist2[b:e]


def _u32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint32)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _collect(res, nq) -> CSR:
    lib = _load()
    tot = int(lib.orc_result_total(res))
    rp = np.empty(nq + 1, dtype=np.int64)
    ids = np.empty(tot, dtype=np.uint32)
    d2 = np.empty(tot, dtype=np.int64)
    lib.orc_result_copy(res, _ptr(rp), _ptr(ids), _ptr(d2))
    lib.orc_result_free(res)
    return CSR(rp, ids, d2)


def _queries(q, n):
    if q is None:
        return None, None, None, n
    qx, qy, qz = (_u32(a) for a in q)
    return qx, qy, qz, len(qx)


def _per_query(v, nq):
    v = np.asarray(v)
    if v.ndim == 0:
        v = np.full(nq, int(v), dtype=np.uint32)
    return _u32(v)


def radius_brute(lat: Lattice, pts, r_fx, queries=None, flags=0) -> CSR:
    """Tier 0 radius query: every query against every point."""
    lib = _load()
    x, y, z = (_u32(a) for a in pts)
    qx, qy, qz, nq = _queries(queries, len(x))
    r = _per_query(r_fx, nq)
    d = lat.c()
    res = lib.orc_radius_brute(ctypes.byref(d), len(x), _ptr(x), _ptr(y), _ptr(z), nq,
                               _ptr(qx), _ptr(qy), _ptr(qz), _ptr(r), flags)
    return _collect(res, nq)


def radius_images(lat: Lattice, pts, r_fx, queries=None, flags=0) -> CSR:
    """Tier 0 with explicit periodic images instead of the minimum-image formula."""
    lib = _load()
    x, y, z = (_u32(a) for a in pts)
    qx, qy, qz, nq = _queries(queries, len(x))
    r = _per_query(r_fx, nq)
    d = lat.c()
    res = lib.orc_radius_images(ctypes.byref(d), len(x), _ptr(x), _ptr(y), _ptr(z), nq,
                                _ptr(qx), _ptr(qy), _ptr(qz), _ptr(r), flags)
    return _collect(res, nq)


def knn_brute(lat: Lattice, pts, k, rmax_fx, queries=None, flags=0) -> CSR:
    lib = _load()
    x, y, z = (_u32(a) for a in pts)
    qx, qy, qz, nq = _queries(queries, len(x))
    kk = _per_query(k, nq)
    r = _per_query(rmax_fx, nq)
    d = lat.c()
    res = lib.orc_knn_brute(ctypes.byref(d), len(x), _ptr(x), _ptr(y), _ptr(z), nq,
                            _ptr(qx), _ptr(qy), _ptr(qz), _ptr(kk), _ptr(r), flags)
    return _collect(res, nq)


class Grid:
    """Tier-1 oracle: a plain cell grid built by the oracle's own counting sort."""

    def __init__(self, lat: Lattice, pts):
        lib = _load()
        self.lat = lat
        self._keep = [_u32(a) for a in pts]
        x, y, z = self._keep
        self.n = len(x)
        d = lat.c()
        self._h = lib.orc_grid_build(ctypes.byref(d), len(x), _ptr(x), _ptr(y), _ptr(z))

    def close(self):
        if self._h:
            _load().orc_grid_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def counts(self) -> np.ndarray:
        L = [1 << int(v) for v in self.lat.log2_cells]
        out = np.empty(L[0] * L[1] * L[2] + 1, dtype=np.uint32)
        _load().orc_grid_counts(self._h, _ptr(out))
        return out

    def radius(self, r_fx, queries=None, flags=0) -> CSR:
        qx, qy, qz, nq = _queries(queries, self.n)
        r = _per_query(r_fx, nq)
        res = _load().orc_grid_radius(self._h, nq, _ptr(qx), _ptr(qy), _ptr(qz), _ptr(r), flags)
        return _collect(res, nq)

    def radius_counts(self, r_fx, queries=None, flags=0) -> np.ndarray:
        """Row sizes of the radius query (int64 [Q]), without the rows."""
        qx, qy, qz, nq = _queries(queries, self.n)
        r = _per_query(r_fx, nq)
        out = np.empty(nq, dtype=np.int64)
        _load().orc_grid_radius_counts(self._h, nq, _ptr(qx), _ptr(qy), _ptr(qz), _ptr(r), flags, _ptr(out))
        return out

    def knn(self, k, rmax_fx, queries=None, flags=0) -> CSR:
        qx, qy, qz, nq = _queries(queries, self.n)
        kk = _per_query(k, nq)
        r = _per_query(rmax_fx, nq)
        res = _load().orc_grid_knn(self._h, nq, _ptr(qx), _ptr(qy), _ptr(qz), _ptr(kk), _ptr(r), flags)
        return _collect(res, nq)

    def mixed(self, k, r_fx, queries=None, flags=0) -> CSR:
        """Query i is K-NN (cap r_fx[i]) when k[i] > 0, else radius r_fx[i]."""
        qx, qy, qz, nq = _queries(queries, self.n)
        kk = _per_query(k, nq)
        r = _per_query(r_fx, nq)
        res = _load().orc_grid_mixed(self._h, nq, _ptr(qx), _ptr(qy), _ptr(qz), _ptr(kk), _ptr(r), flags)
        return _collect(res, nq)


def cells_touched(lat: Lattice, queries, r_fx):
    """Per query: (kept, interior, cube) cell counts; -1 where undefined."""
    lib = _load()
    qx, qy, qz, nq = _queries(queries, 0)
    r = _per_query(r_fx, nq)
    kept = np.empty(nq, dtype=np.int64)
    inter = np.empty(nq, dtype=np.int64)
    cube = np.empty(nq, dtype=np.int64)
    d = lat.c()
    lib.orc_cells_touched(ctypes.byref(d), nq, _ptr(qx), _ptr(qy), _ptr(qz), _ptr(r),
                          _ptr(kept), _ptr(inter), _ptr(cube))
    return kept, inter, cube


def base_minbound2(offset) -> int:
    o = np.ascontiguousarray(offset, dtype=np.int32)
    return int(_load().orc_base_minbound2(len(o), _ptr(o)))


def table_key(F, s, cls, offset) -> int:
    c = np.ascontiguousarray(cls, dtype=np.uint32)
    o = np.ascontiguousarray(offset, dtype=np.int32)
    return int(_load().orc_table_key(F, s, _ptr(c), _ptr(o)))


def table_key_brute(F, s, cls, offset) -> int:
    c = np.ascontiguousarray(cls, dtype=np.uint32)
    o = np.ascontiguousarray(offset, dtype=np.int32)
    return int(_load().orc_table_key_brute(F, s, _ptr(c), _ptr(o)))


def table_set(F, s, cls, r_fx):
    """Offsets (int32 [m,3]) with key <= r^2 for class ``cls`` and their keys."""
    lib = _load()
    c = np.ascontiguousarray(cls, dtype=np.uint32)
    m = int(lib.orc_table_set(F, s, _ptr(c), int(r_fx), None, None))
    out = np.empty((m, 3), dtype=np.int32)
    keys = np.empty(m, dtype=np.int64)
    lib.orc_table_set(F, s, _ptr(c), int(r_fx), _ptr(out), _ptr(keys))
    return out, keys


def mix64(z: int) -> int:
    return int(_load().orc_mix64(z & 0xFFFFFFFFFFFFFFFF))


def hash64(seed: int, tag: int, i: int) -> int:
    return int(_load().orc_hash(seed, tag, i))


def move(lat: Lattice, seed, step, pts):
    """One movement step of the agents (returns new arrays)."""
    x, y, z = (np.array(a, dtype=np.uint32, copy=True) for a in pts)
    d = lat.c()
    _load().orc_move(ctypes.byref(d), seed, step, len(x), _ptr(x), _ptr(y), _ptr(z))
    return x, y, z


def count_checksum(row_ptr) -> tuple:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    out = np.zeros(2, dtype=np.uint64)
    _load().orc_count_checksum(_ptr(rp), len(rp) - 1, _ptr(out))
    return int(out[0]), int(out[1])


def cube_cells(lat: Lattice, q, r_fx) -> int:
    """Distinct cells of the bin-lattice bounding cube of sphere (q, r)."""
    qq = np.ascontiguousarray(q, dtype=np.uint32)
    d = lat.c()
    return int(_load().orc_cube_cells(ctypes.byref(d), _ptr(qq), int(r_fx)))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    _load().orc_set_num_threads(int(n))
