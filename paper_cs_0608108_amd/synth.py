"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers; it holds none of the query arithmetic.
Every draw is a counter-based hash, so any element can be regenerated alone:

    mix64(z)          the SplitMix64 output finaliser (Steele, Lea and Flood,
                      "Fast splittable pseudorandom number generators",
                      OOPSLA 2014)
    H(seed, tag, i) = mix64(seed XOR mix64((tag << 40) XOR i))

Tags: 1..3 point coordinates x, y, z; 4 per-query radius; 5 per-query K;
6 radius/K-NN choice; 7..9 query centres; 20..22 cluster centres;
23 cluster membership; 24..29 Gaussian uniforms; 40..43 serving arrivals.
(The moving-agent displacement uses tags 1000 + 3*step + axis and is drawn
on the device by the library itself, not here.)

The paper's experiments use randomly placed objects and random query centres
in 16^3 and 32^3 worlds (Section IV); the workloads below keep that recipe at
larger sizes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def mix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def H(seed: int, tag: int, i):
    i = np.asarray(i, dtype=np.uint64)
    inner = mix64((np.uint64(tag) << np.uint64(40)) ^ i)
    return mix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ inner)


def uniform_bits(seed, tag, i, bits):
    """Uniform integers in [0, 2^bits) (top bits of the hash)."""
    if bits == 0:
        return np.zeros(np.shape(i), dtype=np.uint64)
    return H(seed, tag, i) >> np.uint64(64 - bits)


def uniform_int(seed, tag, i, lo, hi):
    """Uniform integers in [lo, hi] by multiply-shift of the top 32 bits."""
    span = np.uint64(hi - lo + 1)
    h = H(seed, tag, i) >> np.uint64(32)
    with np.errstate(over="ignore"):
        return (np.uint64(lo) + ((h * span) >> np.uint64(32))).astype(np.int64)


def uniform01(seed, tag, i):
    """Uniform doubles in (0, 1] from 53 hash bits."""
    h = H(seed, tag, i) >> np.uint64(11)
    return (h.astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


@dataclass(frozen=True)
class LatticeSpec:
    log2_cells: tuple
    frac_bits: int
    cyclic_mask: int

    @property
    def cells(self):
        return tuple(1 << v for v in self.log2_cells)

    @property
    def ncells(self):
        c = self.cells
        return c[0] * c[1] * c[2]

    def width(self, a):
        return (1 << self.log2_cells[a]) << self.frac_bits

    @property
    def edge(self):
        return 1 << self.frac_bits


def uniform_points(lat: LatticeSpec, n: int, seed: int, tag0: int = 1):
    """n points uniform over the region: coordinate a = top (F + log2 L_a) bits."""
    i = np.arange(n, dtype=np.uint64)
    return tuple(uniform_bits(seed, tag0 + a, i, lat.frac_bits + lat.log2_cells[a]).astype(np.uint32)
                 for a in range(3))


def gaussian_cluster_points(lat: LatticeSpec, n: int, seed: int, nclusters: int, sigma_fx: float):
    """Mixture of isotropic Gaussian clusters with uniform centres, wrapped
    into the (cyclic) region.  Box-Muller on two 53-bit uniforms per axis,
    rounded to the nearest fixed-point unit.  Generated once on the host so
    every consumer sees the same arrays."""
    c = np.arange(nclusters, dtype=np.uint64)
    centres = [uniform_bits(seed, 20 + a, c, lat.frac_bits + lat.log2_cells[a]).astype(np.int64)
               for a in range(3)]
    i = np.arange(n, dtype=np.uint64)
    lg = int(nclusters).bit_length() - 1
    assert (1 << lg) == nclusters
    member = (H(seed, 23, i) >> np.uint64(64 - lg)).astype(np.int64) if lg > 0 else np.zeros(n, np.int64)
    out = []
    for a in range(3):
        u1 = uniform01(seed, 24 + 2 * a, i)
        u2 = uniform01(seed, 25 + 2 * a, i)
        g = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        v = centres[a][member] + np.rint(g * sigma_fx).astype(np.int64)
        out.append(np.mod(v, lat.width(a)).astype(np.uint32))
    return tuple(out)


def per_query_radius(seed, n, lo_k, hi_k, unit, tag=4, offset=0):
    """Radius r = k * unit with k uniform in [lo_k, hi_k]."""
    i = np.arange(offset, offset + n, dtype=np.uint64)
    return (uniform_int(seed, tag, i, lo_k, hi_k) * unit).astype(np.uint32)


def choice(seed, tag, n, values, offset=0):
    i = np.arange(offset, offset + n, dtype=np.uint64)
    idx = uniform_int(seed, tag, i, 0, len(values) - 1)
    return np.asarray(values, dtype=np.uint32)[idx]


# ---------------------------------------------------------------------------
# The five workloads.  Each returns a dict of host arrays and parameters.

@dataclass
class Workload:
    name: str
    lat: LatticeSpec
    pts: tuple
    r_fx: np.ndarray | None = None   # per query radius (or K-NN cap)
    k: np.ndarray | None = None      # per query K (0 = radius query)
    queries: tuple | None = None     # explicit centres; None = all agents
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return len(self.pts[0])


def radius_uniform_cyclic(n=4096, log2=5, r_cells_fx=163840, seed=1):
    """N uniform points, cyclic L^3, F = 16, every point queries radius r."""
    lat = LatticeSpec((log2,) * 3, 16, 7)
    pts = uniform_points(lat, n, seed)
    return Workload(f"radius_uniform_cyclic_{1 << log2}^3_n{n}", lat, pts,
                    r_fx=np.full(n, r_cells_fx, dtype=np.uint32))


def radius_uneven_clipped(n=1 << 20, log2=7, seed=2):
    """N uniform points in a clipped L^3; per-point radius uniform in
    [0.5, 4] cells quantised to 1/64 cell (k * 1024 units, k in [32, 256])."""
    lat = LatticeSpec((log2,) * 3, 16, 0)
    pts = uniform_points(lat, n, seed)
    r = per_query_radius(seed, n, 32, 256, 1024)
    return Workload(f"radius_uneven_clipped_{1 << log2}^3_n{n}", lat, pts, r_fx=r)


def knn_clustered(n=1 << 22, log2=8, nclusters=64, k=16, seed=3):
    """64 Gaussian clusters (sigma 3 cells) in a cyclic L^3; K-NN, cap 8 cells."""
    lat = LatticeSpec((log2,) * 3, 16, 7)
    pts = gaussian_cluster_points(lat, n, seed, nclusters, 3.0 * lat.edge)
    return Workload(f"knn_clustered_{1 << log2}^3_n{n}_k{k}", lat, pts,
                    r_fx=np.full(n, 8 * lat.edge, dtype=np.uint32),
                    k=np.full(n, k, dtype=np.uint32))


def agents_timestep(n=1 << 23, log2=8, seed=4):
    """Moving agents: uniform start in a cyclic L^3, radius 3 cells."""
    lat = LatticeSpec((log2,) * 3, 16, 7)
    pts = uniform_points(lat, n, seed)
    return Workload(f"agents_timestep_{1 << log2}^3_n{n}", lat, pts,
                    r_fx=np.full(n, 3 * lat.edge, dtype=np.uint32), extra={"seed": seed})


def sweep_world(log2, cyclic_mask, load, seed=6):
    """Section IV worlds: L^3 cells (L = 16 or 32), objects uniform at `load`
    objects per cell on average."""
    lat = LatticeSpec((log2,) * 3, 16, cyclic_mask)
    n = int(round(load * lat.ncells))
    pts = uniform_points(lat, n, seed)
    kind = "wrapping" if cyclic_mask == 7 else "clipped"
    return Workload(f"sweep_{1 << log2}^3_{kind}_load{load}", lat, pts, extra={"seed": seed})


def sweep_centres(lat: LatticeSpec, seed: int, count: int):
    """Random query centres uniform over the region (tags 7..9)."""
    i = np.arange(count, dtype=np.uint64)
    return tuple(uniform_bits(seed, 7 + a, i, lat.frac_bits + lat.log2_cells[a]).astype(np.uint32)
                 for a in range(3))


def serving_lattice(n=1 << 24, log2=9, seed=5):
    """Device-resident lattice for the serving loop: uniform, cyclic L^3."""
    lat = LatticeSpec((log2,) * 3, 16, 7)
    pts = uniform_points(lat, n, seed)
    return Workload(f"serving_{1 << log2}^3_n{n}", lat, pts, extra={"seed": seed})


def serving_batch(lat: LatticeSpec, seed: int, batch_index: int, size: int,
                  rmin_k=64, rmax_k=1024, ks=(1, 8, 32, 128), knn_cap_cells=16):
    """One serving batch: uniform centres; each query is a radius query
    (r = k * 1024, k in [64, 1024], i.e. 1..16 cells) or a K-NN query
    (K from `ks`, cap 16 cells) with probability 1/2 each."""
    off = (batch_index << 17)
    i = np.arange(off, off + size, dtype=np.uint64)
    q = tuple(uniform_bits(seed, 7 + a, i, lat.frac_bits + lat.log2_cells[a]).astype(np.uint32)
              for a in range(3))
    is_knn = (H(seed, 6, i) >> np.uint64(63)).astype(bool)
    r = per_query_radius(seed, size, rmin_k, rmax_k, 1024, offset=off)
    kk = choice(seed, 5, size, ks, offset=off)
    r = np.where(is_knn, np.uint32(knn_cap_cells * lat.edge), r).astype(np.uint32)
    kk = np.where(is_knn, kk, 0).astype(np.uint32)
    return q, r, kk


def serving_batch_sizes(seed: int, count: int, max_size=65536):
    """Log-uniform batch sizes floor(exp(u * ln(max+1))) clamped to [1, max]."""
    u = uniform01(seed, 40, np.arange(count, dtype=np.uint64))
    s = np.floor(np.exp(u * np.log(max_size + 1.0))).astype(np.int64)
    return np.clip(s, 1, max_size)


def serving_interarrivals(seed: int, count: int, rate_per_s: float):
    """Poisson arrivals: exponential gaps with the given mean rate."""
    u = uniform01(seed, 41, np.arange(count, dtype=np.uint64))
    return -np.log(u) / rate_per_s
