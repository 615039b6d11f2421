"""Thin ctypes binding of libsphidx (C ABI in include/sphidx.h).

Argument marshalling only: every step of the query path runs in the HIP
kernels of ``libsphidx.so``.  PyTorch provides device memory and streams.
The library must have been built (``python -m paper_cs_0608108_amd.build``);
importing this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsphidx.so")

OK, ERR_INVALID_ARG, ERR_RANGE, ERR_RADIUS, ERR_CAPACITY, ERR_OOM, ERR_DEVICE, ERR_IO = range(8)
FLAG_RANGE, FLAG_CAPACITY, FLAG_FALLBACK = 1, 2, 4
MODE_RADIUS, MODE_KNN, MODE_MIXED = 0, 1, 2
EXCLUDE_SELF = 1
METHOD_SPHERE, METHOD_CUBE, METHOD_AUTO, METHOD_LIST, METHOD_PAPER64 = 0, 1, 2, 3, 4
SCHED_PLAIN, SCHED_PERSISTENT = 0, 1
ORDER_ANY, ORDER_X = 0, 1

U32, I32, U64, I64, SZ, P = (ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                             ctypes.c_size_t, ctypes.c_void_p)


class LatticeDesc(ctypes.Structure):
    _fields_ = [("log2_cells", U32 * 3), ("frac_bits", U32), ("cyclic_mask", U32)]


class LatticeView(ctypes.Structure):
    _fields_ = [("cell_start", P), ("points", P), ("n", U32), ("ncells", U32)]


class TablesInfo(ctypes.Structure):
    _fields_ = [("subcell_bits", U32), ("frac_bits", U32), ("rmax_fx", U32), ("nclasses", U32),
                ("total_entries", U64), ("device_bytes", U64)]


class Queries(ctypes.Structure):
    _fields_ = [("count", U32), ("x_dev", P), ("y_dev", P), ("z_dev", P), ("radius_fx_dev", P),
                ("radius_fx", U32), ("k_dev", P), ("k", U32), ("mode", U32), ("flags", U32)]


class CSRDesc(ctypes.Structure):
    _fields_ = [("row_ptr_dev", P), ("ids_dev", P), ("dist2_dev", P), ("capacity", I64),
                ("workspace_dev", P), ("workspace_bytes", SZ)]


class LaunchDesc(ctypes.Structure):
    _fields_ = [("method", U32), ("schedule", U32), ("waves_per_block", U32), ("tile", U32),
                ("blocks_per_cu", U32), ("sort_cap", U32), ("table_in_lds", U32), ("interior", U32),
                ("stats_dev", P), ("event_begin", P), ("event_end", P), ("no_stash", U32),
                ("grouped", U32), ("select_weight", U32), ("reversal_fx", U32), ("knn_reversal_fx", U32),
                ("select_model", U32), ("method_dev", P), ("long_row_waves", U32)]



class BatchDesc(ctypes.Structure):
    _fields_ = [("count", U32), ("x", P), ("y", P), ("z", P), ("radius_fx", P), ("k", P),
                ("arrival_s", ctypes.c_double), ("row_ptr_out", P), ("ids_out", P), ("ids_capacity", U64)]


class BatchResult(ctypes.Structure):
    _fields_ = [("start_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("pairs", I64), ("pool_in_use", U64), ("rejected", U32), ("status", U32)]

# Every symbol include/sphidx.h declares, with its ctypes signature.
SIGNATURES = {
    "sphidx_lattice_workspace_bytes": (SZ, [ctypes.POINTER(LatticeDesc), U32]),
    "sphidx_lattice_create": (ctypes.c_int, [ctypes.POINTER(LatticeDesc), U32, P, SZ, ctypes.POINTER(P)]),
    "sphidx_lattice_destroy": (None, [P]),
    "sphidx_build_lattice": (ctypes.c_int, [P, P, P, P, U32, P]),
    "sphidx_lattice_get_view": (ctypes.c_int, [P, ctypes.POINTER(LatticeView)]),
    "sphidx_lattice_status": (ctypes.c_int, [P, P, ctypes.POINTER(U32)]),
    "sphidx_lattice_set_cell_order": (ctypes.c_int, [P, U32]),
    "sphidx_stream_status": (ctypes.c_int, [P, ctypes.POINTER(U32)]),
    "sphidx_cell_list_bytes": (SZ, [P]),
    "sphidx_lattice_attach_cell_list": (ctypes.c_int, [P, P, SZ, P]),
    "sphidx_build_sphere_tables": (ctypes.c_int, [ctypes.POINTER(LatticeDesc), U32, U32, ctypes.POINTER(P)]),
    "sphidx_tables_destroy": (None, [P]),
    "sphidx_tables_get_info": (ctypes.c_int, [P, ctypes.POINTER(TablesInfo)]),
    "sphidx_tables_export": (ctypes.c_int, [P, U32, P, P, ctypes.POINTER(U64)]),
    "sphidx_tables_save": (ctypes.c_int, [P, ctypes.c_char_p]),
    "sphidx_tables_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(P)]),
    "sphidx_table_census": (ctypes.c_int, [P, U32, P, P, P, P, P]),
    "sphidx_table_census_nd": (ctypes.c_int, [U32, U32, U32, U32, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double), P, U32]),
    "sphidx_query_workspace_bytes": (SZ, [U32]),
    "sphidx_query_stash_bytes": (SZ, [ctypes.c_uint64, ctypes.c_int]),
    "sphidx_count": (ctypes.c_int, [P, P, ctypes.POINTER(Queries), ctypes.POINTER(CSRDesc),
                                    ctypes.POINTER(LaunchDesc), P]),
    "sphidx_write": (ctypes.c_int, [P, P, ctypes.POINTER(Queries), ctypes.POINTER(CSRDesc),
                                    ctypes.POINTER(LaunchDesc), P]),
    "sphidx_query": (ctypes.c_int, [P, P, ctypes.POINTER(Queries), ctypes.POINTER(CSRDesc),
                                    ctypes.POINTER(LaunchDesc), P]),
    "sphidx_query_noalloc": (ctypes.c_int, [P, P, ctypes.POINTER(Queries), ctypes.POINTER(CSRDesc),
                                            ctypes.POINTER(LaunchDesc), P]),
    "sphidx_radius_count": (ctypes.c_int, [P, P, ctypes.POINTER(Queries), ctypes.POINTER(CSRDesc), P]),
    "sphidx_radius_query": (ctypes.c_int, [P, P, ctypes.POINTER(Queries), ctypes.POINTER(CSRDesc), P]),
    "sphidx_knn_query": (ctypes.c_int, [P, P, ctypes.POINTER(Queries), ctypes.POINTER(CSRDesc), P]),
    "sphidx_cube_scan_radius": (ctypes.c_int, [P, ctypes.POINTER(Queries), ctypes.POINTER(CSRDesc), P]),
    "sphidx_cube_scan_knn": (ctypes.c_int, [P, ctypes.POINTER(Queries), ctypes.POINTER(CSRDesc), P]),
    "sphidx_move_agents": (ctypes.c_int, [ctypes.POINTER(LatticeDesc), U64, U32, P, P, P, U32, P]),
    "sphidx_move_agents_counted": (ctypes.c_int, [ctypes.POINTER(LatticeDesc), U64, P, P, P, P, U32, P]),
    "sphidx_move_resident": (ctypes.c_int, [P, U64, U32, P, P, ctypes.c_size_t, P]),
    "sphidx_move_incremental_scratch_bytes": (SZ, [P]),
    "sphidx_move_incremental": (ctypes.c_int, [P, U64, U32, P, P, ctypes.c_size_t, P]),
    "sphidx_lattice_positions": (ctypes.c_int, [P, P, P, P, P]),
    "sphidx_count_checksum": (ctypes.c_int, [P, U32, P, P]),
    "sphidx_server_create": (ctypes.c_int, [P, P, U32, U32, SZ, U64, ctypes.POINTER(LaunchDesc),
                                             ctypes.POINTER(P)]),
    "sphidx_server_destroy": (None, [P]),
    "sphidx_server_run": (ctypes.c_int, [P, U32, ctypes.POINTER(BatchDesc), ctypes.POINTER(BatchResult)]),
    "sphidx_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sphidx_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libsphidx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_cs_0608108_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class SphidxError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = load().sphidx_status_string(code).decode()
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


def check(code, what=""):
    if code != OK:
        raise SphidxError(code, what)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def desc_of(log2_cells, frac_bits, cyclic_mask) -> LatticeDesc:
    d = LatticeDesc()
    for a in range(3):
        d.log2_cells[a] = int(log2_cells[a])
    d.frac_bits = int(frac_bits)
    d.cyclic_mask = int(cyclic_mask)
    return d


def to_dev_u32(a, device="cuda"):
    """Host uint32 array -> device tensor holding the same 32-bit patterns (int32 storage)."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).to(device)


def to_host_u32(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Lattice:
    """A lattice handle bound to a device workspace owned by this object."""

    def __init__(self, log2_cells, frac_bits, cyclic_mask, max_points, device="cuda"):
        lib = load()
        self.desc = desc_of(log2_cells, frac_bits, cyclic_mask)
        self.max_points = int(max_points)
        nbytes = lib.sphidx_lattice_workspace_bytes(ctypes.byref(self.desc), self.max_points)
        if nbytes == 0:
            raise SphidxError(ERR_INVALID_ARG, "lattice descriptor")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        h = P()
        check(lib.sphidx_lattice_create(ctypes.byref(self.desc), self.max_points, ctypes.c_void_p(self._ws_ptr),
                                        nbytes, ctypes.byref(h)), "lattice_create")
        self.handle = h
        self.n = 0
        self.log2_cells = tuple(int(v) for v in log2_cells)
        self.frac_bits = int(frac_bits)
        self.cyclic_mask = int(cyclic_mask)
        self.cell_list = None

    def __del__(self):
        try:
            if self.handle:
                load().sphidx_lattice_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    @property
    def ncells(self):
        return 1 << sum(self.log2_cells)

    def build(self, x, y, z, stream=None):
        n = int(x.numel())
        check(load().sphidx_build_lattice(self.handle, _ptr(x), _ptr(y), _ptr(z), n, _stream(stream)), "build")
        self.n = n

    def view(self):
        v = LatticeView()
        check(load().sphidx_lattice_get_view(self.handle, ctypes.byref(v)))
        return v

    def attach_cell_list(self, on=True, stream=None):
        """Keep the non-empty cell list (rebuilt with every build) in a buffer
        owned by this object, or detach it."""
        lib = load()
        if not on:
            check(lib.sphidx_lattice_attach_cell_list(self.handle, None, 0, _stream(stream)), "detach_cell_list")
            self.cell_list = None
            return
        nbytes = lib.sphidx_cell_list_bytes(self.handle)
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.workspace.device)
        off = (-buf.data_ptr()) % 256
        check(lib.sphidx_lattice_attach_cell_list(self.handle, ctypes.c_void_p(buf.data_ptr() + off), nbytes,
                                                  _stream(stream)), "attach_cell_list")
        self.cell_list = buf[off:off + nbytes]

    def cell_list_host(self):
        """(count, entries uint32[count + 1, 2]) of the attached list (synchronises)."""
        torch.cuda.synchronize()
        raw = self.cell_list.view(torch.int32).cpu().numpy().view(np.uint32)
        cnt = int(raw[0])
        return cnt, raw[4:4 + 2 * (cnt + 1)].reshape(cnt + 1, 2).copy()

    def set_cell_order(self, order):
        """ORDER_ANY or ORDER_X (objects inside each cell by x) for later builds."""
        check(load().sphidx_lattice_set_cell_order(self.handle, int(order)), "set_cell_order")

    def status(self, stream=None):
        """(status code, flags); synchronises the stream and clears the word."""
        f = U32(0)
        code = load().sphidx_lattice_status(self.handle, _stream(stream), ctypes.byref(f))
        return code, int(f.value)

    def host_arrays(self):
        """Copy cell_start and the sorted object records back to the host (for tests).
        The view's pointers lie inside this object's workspace tensor."""
        v = self.view()
        base = self.workspace.data_ptr()

        def grab(ptr, count):
            off = ptr - base
            t = self.workspace[off:off + 4 * count].view(torch.int32)
            return t.cpu().numpy().view(np.uint32)

        torch.cuda.synchronize()
        pts = grab(v.points, 4 * v.n).reshape(v.n, 4)
        return dict(cell_start=grab(v.cell_start, v.ncells + 3), xs=pts[:, 0].copy(), ys=pts[:, 1].copy(),
                    zs=pts[:, 2].copy(), ids=pts[:, 3].copy())


class Tables:
    def __init__(self, lattice_or_desc, subcell_bits=2, rmax_fx=None, handle=None):
        lib = load()
        if handle is not None:
            self.handle = handle
        else:
            desc = lattice_or_desc.desc if isinstance(lattice_or_desc, Lattice) else lattice_or_desc
            h = P()
            check(lib.sphidx_build_sphere_tables(ctypes.byref(desc), int(subcell_bits), int(rmax_fx),
                                                 ctypes.byref(h)), "build_sphere_tables")
            self.handle = h

    @classmethod
    def load_file(cls, path):
        h = P()
        check(load().sphidx_tables_load(str(path).encode(), ctypes.byref(h)), "tables_load")
        return cls(None, handle=h)

    def save(self, path):
        check(load().sphidx_tables_save(self.handle, str(path).encode()), "tables_save")

    def __del__(self):
        try:
            if self.handle:
                load().sphidx_tables_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def info(self) -> TablesInfo:
        i = TablesInfo()
        check(load().sphidx_tables_get_info(self.handle, ctypes.byref(i)))
        return i

    def export(self, cls):
        n = U64(0)
        check(load().sphidx_tables_export(self.handle, int(cls), None, None, ctypes.byref(n)))
        offs = np.empty((n.value, 3), dtype=np.int32)
        keys = np.empty(n.value, dtype=np.int64)
        check(load().sphidx_tables_export(self.handle, int(cls), ctypes.c_void_p(offs.ctypes.data),
                                          ctypes.c_void_p(keys.ctypes.data), ctypes.byref(n)))
        return offs, keys


CENSUS_FIELDS = ("cube", "unshaved", "paper64", "paper64_eq1", "subcell", "exact", "dropped")


def table_census(tab, f, r):
    """Cells walked per table design (host only): f = (fx, fy, fz) positions
    inside the home cell, r radii; returns {design: uint64[n]}."""
    f = [np.ascontiguousarray(a, dtype=np.uint32) for a in f]
    r = np.ascontiguousarray(r, dtype=np.uint32)
    out = np.zeros((len(r), 7), dtype=np.uint64)
    check(load().sphidx_table_census(tab.handle, len(r), *(ctypes.c_void_p(a.ctypes.data) for a in f),
                                     ctypes.c_void_p(r.ctypes.data), ctypes.c_void_p(out.ctypes.data)),
          "table_census")
    return {k: out[:, i] for i, k in enumerate(CENSUS_FIELDS)}


def table_census_nd(dims, frac_bits, subcell_bits, r_fx, hist_len=0):
    """(mean sphere cells, mean bounding-box cells, unshaved b^2 histogram)."""
    s, c = ctypes.c_double(), ctypes.c_double()
    hist = np.zeros(max(hist_len, 1), dtype=np.uint64)
    check(load().sphidx_table_census_nd(int(dims), int(frac_bits), int(subcell_bits), int(r_fx), ctypes.byref(s),
                                        ctypes.byref(c), ctypes.c_void_p(hist.ctypes.data), int(hist_len)),
          "table_census_nd")
    return s.value, c.value, hist[:hist_len]


@dataclass
class LaunchConfig:
    method: int = METHOD_SPHERE
    schedule: int = SCHED_PERSISTENT
    waves_per_block: int = 0
    tile: int = 0
    blocks_per_cu: int = 0
    sort_cap: int = 0
    table_in_lds: int = 0
    interior: int = 0
    stats: torch.Tensor | None = None
    events: tuple | None = None  # (begin, end) torch.cuda.Event around the pass's main kernel
    no_stash: int = 0
    grouped: int = 0
    select_weight: int = 0  # METHOD_AUTO: Q8 weight of the sphere's cell count (0 = 256)
    reversal_fx: int = 0
    knn_reversal_fx: int = 0
    select_model: int = 0  # 0: compare cells (the paper); 1: compare estimated lane work
    method_out: torch.Tensor | None = None  # int32[Q]: the walk each query used
    long_row_waves: int = 0  # waves per long radius row in the write pass (0 = 4, 1 = one wave, windowed)

    def c(self) -> LaunchDesc:
        d = LaunchDesc()
        d.method, d.schedule = self.method, self.schedule
        d.waves_per_block, d.tile, d.blocks_per_cu = self.waves_per_block, self.tile, self.blocks_per_cu
        d.sort_cap, d.table_in_lds = self.sort_cap, self.table_in_lds
        d.interior = self.interior
        d.no_stash = self.no_stash
        d.grouped = self.grouped
        d.select_weight, d.reversal_fx, d.knn_reversal_fx = self.select_weight, self.reversal_fx, self.knn_reversal_fx
        d.select_model = self.select_model
        d.long_row_waves = self.long_row_waves
        d.method_dev = None if self.method_out is None else self.method_out.data_ptr()
        d.stats_dev = None if self.stats is None else self.stats.data_ptr()
        if self.events is not None:
            for ev in self.events:
                if not ev.cuda_event:  # torch creates the HIP event at its first record
                    ev.record()
            d.event_begin, d.event_end = self.events[0].cuda_event, self.events[1].cuda_event
        return d


def make_queries(count, centres=None, radius=None, k=None, mode=MODE_RADIUS, flags=0) -> Queries:
    """centres: None (all agents) or (x, y, z) device tensors; radius / k:
    an int (uniform) or a device tensor (per query)."""
    q = Queries()
    q.count = int(count)
    if centres is not None:
        q.x_dev, q.y_dev, q.z_dev = (c.data_ptr() for c in centres)
    if isinstance(radius, torch.Tensor):
        q.radius_fx_dev = radius.data_ptr()
    else:
        q.radius_fx = int(radius or 0)
    if isinstance(k, torch.Tensor):
        q.k_dev = k.data_ptr()
    else:
        q.k = int(k or 0)
    q.mode, q.flags = int(mode), int(flags)
    return q


class QueryBuffers:
    """Device outputs and workspace of one query call.

    The workspace is zero-filled when (re)allocated.  `reserve_stash(pairs)`
    enlarges it so that a following count pass can keep up to that many
    sorted pairs for the write pass; it must be called before the count, as
    the write pass reads what the count pass left in the workspace."""

    def __init__(self, Q, capacity, want_dist2=True, device="cuda", stash_pairs=0):
        self.Q = int(Q)
        self.device = device
        self.row_ptr = torch.empty(self.Q + 1, dtype=torch.int64, device=device)
        self.capacity = int(capacity)
        self.ids = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.dist2 = torch.empty(max(self.capacity, 1), dtype=torch.int64, device=device) if want_dist2 else None
        self.stash_pairs = 0
        self._alloc_workspace(int(stash_pairs))

    def _alloc_workspace(self, stash_pairs):
        lib = load()
        wsb = lib.sphidx_query_workspace_bytes(self.Q)
        if stash_pairs > 0:
            wsb += lib.sphidx_query_stash_bytes(stash_pairs, int(self.dist2 is not None))
        self.workspace = None
        self.workspace = torch.zeros(wsb + 256, dtype=torch.uint8, device=self.device)
        self._ws = self.workspace.data_ptr() + ((-self.workspace.data_ptr()) % 256)
        self._wsb = wsb
        self.stash_pairs = stash_pairs

    def grow(self, capacity):
        """Larger outputs; the workspace (and what a count left there) is kept."""
        if capacity > self.capacity:
            dev = self.ids.device
            self.capacity = int(capacity)
            self.ids = torch.empty(self.capacity, dtype=torch.int32, device=dev)
            if self.dist2 is not None:
                self.dist2 = torch.empty(self.capacity, dtype=torch.int64, device=dev)

    def reserve_stash(self, pairs):
        if pairs > self.stash_pairs:
            self._alloc_workspace(int(pairs))

    def c(self) -> CSRDesc:
        d = CSRDesc()
        d.row_ptr_dev = self.row_ptr.data_ptr()
        d.ids_dev = self.ids.data_ptr()
        d.dist2_dev = None if self.dist2 is None else self.dist2.data_ptr()
        d.capacity = self.capacity
        d.workspace_dev = self._ws
        d.workspace_bytes = self._wsb
        return d

    def host(self):
        rp = self.row_ptr.cpu().numpy()
        tot = int(rp[-1])
        ids = self.ids[:tot].cpu().numpy().view(np.uint32)
        d2 = self.dist2[:tot].cpu().numpy() if self.dist2 is not None else None
        return rp, ids, d2


def count(lat, tab, q: Queries, buf: QueryBuffers, launch: LaunchConfig | None = None, stream=None):
    ln = (launch or LaunchConfig()).c()
    cs = buf.c()
    check(load().sphidx_count(lat.handle, tab.handle if tab else None, ctypes.byref(q), ctypes.byref(cs),
                              ctypes.byref(ln), _stream(stream)), "count")


def stream_status(stream=None):
    """(status code, flags) of every lattice the stream's calls touched since
    the last report; synchronises the stream and clears the words."""
    f = U32(0)
    code = load().sphidx_stream_status(_stream(stream), ctypes.byref(f))
    return code, int(f.value)


def write(lat, tab, q: Queries, buf: QueryBuffers, launch: LaunchConfig | None = None, stream=None):
    ln = (launch or LaunchConfig()).c()
    cs = buf.c()
    check(load().sphidx_write(lat.handle, tab.handle if tab else None, ctypes.byref(q), ctypes.byref(cs),
                              ctypes.byref(ln), _stream(stream)), "write")


def query(lat, tab, q: Queries, buf: QueryBuffers, launch: LaunchConfig | None = None, stream=None):
    ln = (launch or LaunchConfig()).c()
    cs = buf.c()
    check(load().sphidx_query(lat.handle, tab.handle if tab else None, ctypes.byref(q), ctypes.byref(cs),
                              ctypes.byref(ln), _stream(stream)), "query")


def run(lat, tab, q: Queries, launch: LaunchConfig | None = None, want_dist2=True, stream=None, stash=False):
    """Count, size the outputs exactly, write; returns host (row_ptr, ids, dist2).
    stash=True counts a second time with a workspace that keeps every row, so
    that the write pass copies rows instead of walking again."""
    buf = QueryBuffers(q.count, 0, want_dist2)
    count(lat, tab, q, buf, launch, stream)
    total = int(buf.row_ptr[-1].item())
    buf.grow(max(total, 1))
    if stash:
        buf.reserve_stash(max(total, 1))
        count(lat, tab, q, buf, launch, stream)
    write(lat, tab, q, buf, launch, stream)
    torch.cuda.synchronize()
    return buf.host()


def move_agents(desc: LatticeDesc, seed, step, x, y, z, stream=None):
    check(load().sphidx_move_agents(ctypes.byref(desc), int(seed), int(step), _ptr(x), _ptr(y), _ptr(z),
                                    int(x.numel()), _stream(stream)), "move_agents")


def move_agents_counted(desc: LatticeDesc, seed, step_dev, x, y, z, stream=None):
    check(load().sphidx_move_agents_counted(ctypes.byref(desc), int(seed), _ptr(step_dev), _ptr(x), _ptr(y),
                                            _ptr(z), int(x.numel()), _stream(stream)), "move_agents_counted")


def move_resident(lat, seed, scratch, step=0, step_dev=None, stream=None):
    """Move the lattice's own records (incremental maintenance) and rebuild
    from them; `scratch` is a device tensor of at least 16 * n bytes."""
    check(load().sphidx_move_resident(lat.handle, int(seed), int(step), None if step_dev is None else _ptr(step_dev),
                                      _ptr(scratch), int(scratch.numel() * scratch.element_size()), _stream(stream)),
          "move_resident")


def move_incremental_scratch_bytes(lat):
    return int(load().sphidx_move_incremental_scratch_bytes(lat.handle))


def move_incremental(lat, seed, scratch, step=0, step_dev=None, stream=None):
    """Move the lattice's records and update the lattice incrementally (only
    objects that change cell take an atomic); `scratch` is a device tensor of
    at least move_incremental_scratch_bytes(lat) bytes, 256-byte aligned."""
    check(load().sphidx_move_incremental(lat.handle, int(seed), int(step),
                                         None if step_dev is None else _ptr(step_dev), _ptr(scratch),
                                         int(scratch.numel() * scratch.element_size()), _stream(stream)),
          "move_incremental")


def lattice_positions(lat, x, y, z, stream=None):
    """By-id coordinates of the lattice's objects into device arrays x, y, z."""
    check(load().sphidx_lattice_positions(lat.handle, _ptr(x), _ptr(y), _ptr(z), _stream(stream)), "lattice_positions")


def count_checksum(row_ptr, Q, out, stream=None):
    check(load().sphidx_count_checksum(_ptr(row_ptr), int(Q), _ptr(out), _stream(stream)), "count_checksum")


def version() -> str:
    return load().sphidx_version().decode()


class Server:
    """A serving loop in the library (sphidx_server_*): `slots` batches in
    flight on their own streams, an output pool of `pool_bytes` admitted by
    memory in arrival order.  The lattice must be built and its stream
    synchronised before `run`."""

    def __init__(self, lat, tab, slots, max_batch, pool_bytes, stash_pairs=0, launch: LaunchConfig | None = None):
        self.lat, self.tab = lat, tab  # kept alive for the server's life
        self.max_batch = int(max_batch)
        self.handle = None
        h = P()
        ln = launch.c() if launch is not None else None
        check(load().sphidx_server_create(lat.handle, tab.handle if tab else None, int(slots), self.max_batch,
                                          int(pool_bytes), int(stash_pairs),
                                          ctypes.byref(ln) if ln is not None else None, ctypes.byref(h)),
              "server_create")
        self.handle = h.value

    def close(self):
        if self.handle:
            load().sphidx_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, arrivals, centres, radius, k, keep=False):
        """Replay batches: arrivals[i] (seconds, non-decreasing), centres[i]
        = (x, y, z) host uint32 arrays, radius[i], k[i] host uint32 arrays
        (k[i] None: radius queries only).  Returns the per-batch results
        (structured numpy array) and, with keep, each batch's (row_ptr, ids)
        on the host (None for a rejected batch)."""
        n = len(arrivals)
        descs = (BatchDesc * max(n, 1))()
        res = (BatchResult * max(n, 1))()
        hold, outs = [], []
        for i in range(n):
            x, y, z = (np.ascontiguousarray(a, dtype=np.uint32) for a in centres[i])
            r = np.ascontiguousarray(radius[i], dtype=np.uint32)
            kk = None if k[i] is None else np.ascontiguousarray(k[i], dtype=np.uint32)
            hold.append((x, y, z, r, kk))
            d = descs[i]
            d.count = len(r)
            d.x, d.y, d.z, d.radius_fx = x.ctypes.data, y.ctypes.data, z.ctypes.data, r.ctypes.data
            d.k = None if kk is None else kk.ctypes.data
            d.arrival_s = float(arrivals[i])
            if keep:
                rp = np.empty(len(r) + 1, dtype=np.int64)
                outs.append([rp, None])
                d.row_ptr_out = rp.ctypes.data
        if keep:
            # sizes first: the ids copies need each batch's total
            code = load().sphidx_server_run(self.handle, n, descs, res)
            check(code, "server_run")
            for i in range(n):
                tot = int(res[i].pairs)
                ids = np.empty(max(tot, 1), dtype=np.uint32)
                outs[i][1] = ids
                descs[i].ids_out = ids.ctypes.data
                descs[i].ids_capacity = tot
        code = load().sphidx_server_run(self.handle, n, descs, res)
        check(code, "server_run")
        out = np.ctypeslib.as_array(res)[:n].copy()
        if not keep:
            return out, None
        rows = [None if out["rejected"][i] else (outs[i][0], outs[i][1][: int(out["pairs"][i])]) for i in range(n)]
        return out, rows

