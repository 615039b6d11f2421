"""Readers for the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                yield ln


def read_matrix(name):
    return np.array([[int(v) for v in ln.split()] for ln in _lines(name)], dtype=np.int64)


def read_pairs(name):
    return {int(a): int(b) for a, b in (ln.split() for ln in _lines(name))}


def read_keyed(name):
    out = {}
    for ln in _lines(name):
        k, *v = ln.split()
        out[k] = v
    return out


def read_hand(name):
    """Hand fixture: lattice, points and expected rows."""
    lat = {}
    pts = []
    rows = []
    for ln in _lines(name):
        head, _, tail = ln.partition(":")
        f = head.split()
        if f[0] == "lattice_log2":
            lat["log2_cells"] = tuple(int(v) for v in f[1:4])
        elif f[0] in ("frac_bits", "cyclic_mask"):
            lat[f[0]] = int(f[1])
        elif f[0] == "point":
            pts.append([int(v) for v in f[1:5]])
        elif f[0] in ("radius", "knn"):
            exp = [tuple(int(t) for t in e.split(":")) for e in tail.split()]
            if f[0] == "radius":
                rows.append(dict(kind="radius", q=int(f[1]), r=int(f[2]), k=0, flags=int(f[3]), exp=exp))
            else:
                rows.append(dict(kind="knn", q=int(f[1]), k=int(f[2]), r=int(f[3]), flags=int(f[4]),
                                 exp=exp))
    pts.sort()
    ids = [p[0] for p in pts]
    assert ids == list(range(len(ids)))
    arr = np.array([p[1:] for p in pts], dtype=np.uint64)
    return lat, tuple(arr[:, a].astype(np.uint32) for a in range(3)), rows
