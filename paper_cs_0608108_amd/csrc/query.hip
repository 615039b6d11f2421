// Neighbourhood query kernels for gfx950 (wave64).
//
// Per query:
//   setup   (one thread per query, setup_kernel) home cell = q >> F, sub-cell
//           class = the top s bits of q's position inside its cell along y
//           and z (Section III.A: the position inside the cell selects a
//           specialised table), the method, and the class table's prefix end
//           from the radius index (Section II.A: one lookup tells where to
//           stop in the sorted table), stored as a 64-byte descriptor.
//   walk    the class table lists x-rows of cells (oy, oz) sorted by their
//           minimum distance, centre to edge; 64 rows per step, one per lane.
//           A lane solves the exact test of Eq. 1 for its row's contiguous
//           run of cells, wraps cyclic axes or clips to the region (Section
//           II.B), and turns the run into one range of objects (two when it
//           wraps), since objects are sorted by packed ZYX cell.
//   scan    the objects of the rows are spread over the lanes: a DPP prefix
//           sum of per-lane counts, an LDS map of where each lane's range
//           starts and a DPP max-scan give every slot its owner, so a wave
//           tests 64 candidates per step whatever the cell loads.  One
//           16-byte load fetches a candidate's coordinates and id.
//   output  count pass: hits per row (K-NN: min(K, hits within the cap),
//           stopping once K are found); with workspace to spare it also
//           sorts each radius row by (dist^2, id) and keeps it (the stash),
//           and the write pass only copies the kept rows into place.  Rows
//           not kept are walked again by the write pass.  K-NN rows and
//           long rows go to the top-M kernel, which keeps the M best (in
//           registers for M <= 64), shrinks the bound to the M-th distance
//           once M are held and stops at the first row whose key exceeds it
//           (Section II.A, K nearest).
// The count pass can also take radius queries in groups of several per
// wavefront, so that short rows and small radii fill whole steps.  Queries
// whose radius exceeds the tables' cap or the cyclic limit, or whose centre
// is outside the region, and every query of the cube method, scan the
// bin-lattice bounding cube instead (Section I; Section III.B).  With the
// per-query choice each query takes the sphere, the cube or the lattice's
// non-empty cell list, whichever the comparison of their cells (Section
// III.B, III.C) or of their estimated work finds smallest; a list entry is
// one more kind of row.
#include <algorithm>

#include "sphidx_internal.h"

namespace {

constexpr uint32_t kMaxId = 0xFFFFFFFFu;
constexpr uint64_t kMaxD2 = ~0ull;
// Walk kinds: sphere rows only, cube rows only, either (chosen per query),
// or the paper's cell tables (cube rows for the queries they do not serve).
constexpr int kSphere = 0, kCube = 1, kEither = 2, kPaper = 3;

// ---------------------------------------------------------------------------
// Wave primitives

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t bperm(uint32_t v, uint32_t lane) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(lane << 2), (int)v);
}
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
__device__ __forceinline__ uint32_t lane_val(uint32_t v, uint32_t l) { return __builtin_amdgcn_readlane(v, l); }
// LDS ordering point for one wavefront: its LDS operations execute in order;
// this keeps the compiler from moving them across the point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL, int ROWS, bool BOUND>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, BOUND);
}

// Inclusive prefix sum over the 64 lanes: shifts by 1, 2, 4, 8 inside each
// row of 16 lanes, then row 0's total into row 1 and row 2's into row 3
// (row_bcast:15), then rows 0-1's total into rows 2-3 (row_bcast:31).
__device__ __forceinline__ uint32_t scan_add(uint32_t v) {
    v += dpp<0x111, 0xF, true>(v);
    v += dpp<0x112, 0xF, true>(v);
    v += dpp<0x114, 0xF, true>(v);
    v += dpp<0x118, 0xF, true>(v);
    v += dpp<0x142, 0xA, false>(v);
    v += dpp<0x143, 0xC, false>(v);
    return v;
}

__device__ __forceinline__ uint32_t scan_max(uint32_t v) {
    v = max(v, dpp<0x111, 0xF, true>(v));
    v = max(v, dpp<0x112, 0xF, true>(v));
    v = max(v, dpp<0x114, 0xF, true>(v));
    v = max(v, dpp<0x118, 0xF, true>(v));
    v = max(v, dpp<0x142, 0xA, false>(v));
    v = max(v, dpp<0x143, 0xC, false>(v));
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return lane_val(scan_add(v), 63); }

__device__ __forceinline__ bool key_less(uint64_t da, uint32_t ia, uint64_t db, uint32_t ib) {
    return da < db || (da == db && ia < ib);
}

// Sort one (d2, id) key per lane ascending over the 64 lanes (bitonic).
__device__ __forceinline__ void wave_sort64(uint64_t& d, uint32_t& id) {
    const uint32_t l = lane_id();
#pragma unroll
    for (uint32_t k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            uint32_t plo = __shfl_xor((uint32_t)d, j);
            uint32_t phi = __shfl_xor((uint32_t)(d >> 32), j);
            uint32_t pid = __shfl_xor(id, j);
            uint64_t pd = ((uint64_t)phi << 32) | plo;
            bool want_min = ((l & j) == 0) == ((l & k) == 0);
            bool take = want_min ? key_less(pd, pid, d, id) : key_less(d, id, pd, pid);
            if (take) {
                d = pd;
                id = pid;
            }
        }
    }
}

// Sort a bitonic sequence of one (d2, id) key per lane ascending.
__device__ __forceinline__ void wave_bitonic_clean64(uint64_t& d, uint32_t& id) {
    const uint32_t l = lane_id();
#pragma unroll
    for (uint32_t j = 32; j > 0; j >>= 1) {
        uint32_t plo = __shfl_xor((uint32_t)d, j);
        uint32_t phi = __shfl_xor((uint32_t)(d >> 32), j);
        uint32_t pid = __shfl_xor(id, j);
        uint64_t pd = ((uint64_t)phi << 32) | plo;
        bool take = (l & j) == 0 ? key_less(pd, pid, d, id) : key_less(d, id, pd, pid);
        if (take) {
            d = pd;
            id = pid;
        }
    }
}

__device__ __forceinline__ uint64_t lane_val64(uint64_t v, uint32_t l) {
    return ((uint64_t)lane_val((uint32_t)(v >> 32), l) << 32) | lane_val((uint32_t)v, l);
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, uint32_t src) {
    return ((uint64_t)__shfl((uint32_t)(v >> 32), src) << 32) | (uint32_t)__shfl((uint32_t)v, src);
}

// Exact quotient (a < 2^31, 1 <= b < 2^31) from a double reciprocal and one
// correction step.
__device__ __forceinline__ uint32_t exact_div(uint32_t a, uint32_t b, double inv_b) {
    uint32_t q = (uint32_t)((double)a * inv_b);
    if ((uint64_t)q * b > a) --q;
    if ((uint64_t)(q + 1) * b <= a) ++q;
    return q;
}

__device__ __forceinline__ uint64_t sq(uint32_t g) { return (uint64_t)g * (uint64_t)g; }


// ---------------------------------------------------------------------------
// Query descriptors

// F_LIST: the query walks the non-empty cell list (neither F_SPHERE nor
// F_LIST: the bounding cube).
// F_KBOUND: a K-NN row whose count pass found K objects within the radius
// stored in descriptor word 12 (an upper bound of its K-th distance; sphere
// walks only, which leave that word unused).  F_LONG: a radius row expected
// to be longer than a wavefront's buffer, counted and kept one block per row.
enum : uint32_t {
    F_VALID = 1u, F_KNN = 2u, F_SPHERE = 4u, F_OUTSIDE = 8u, F_LIST = 16u, F_KBOUND = 32u, F_LONG = 64u
};

struct Query {
    uint32_t q[3];  // normalised centre
    uint32_t row;   // output row
    uint32_t r;     // radius, or the K-NN cap
    uint32_t k;
    uint32_t flags;
    uint32_t tb;    // sphere: first entry of the class table
    uint32_t tend;  // sphere: prefix length
    uint32_t ncube; // cube: cells of the bounding cube
    uint32_t nn[3]; // cube: cells per axis (cell list: 0, its length, 1)
    int32_t lo[3];  // cube: first cell per axis
    uint32_t self;  // sorted position excluded (EXCLUDE_SELF, all agents) or ~0
    uint32_t kbr;   // F_KBOUND: a radius holding K objects
    uint32_t c[3];  // home cell
    uint32_t f[3];  // position inside the home cell
    uint32_t up[3]; // e - f: distance to the next cell up
    uint32_t dn[3]; // f + 1: distance to the last position of the cell below
    uint64_t r2;
};

__device__ __forceinline__ uint32_t pack_cell(const LatArgs& L, uint32_t x, uint32_t y, uint32_t z) {
    return (z << (L.lg[0] + L.lg[1])) | (y << L.lg[0]) | x;
}

// One thread per query: centre, radius, K, method and walk extent.
// K-NN first search radius in the grouped count: the radius of the ball
// expected to hold knn_target(K) objects at the density around the home cell.
// For small K that is 1.2^3 K (about 1.7K): smaller leaves more rows short of
// K (searched again), larger overflows more hit buffers; on clustered K = 16
// the step took 5.93, 5.29, 5.23, 5.24, 5.34, 5.53, 6.50 and 8.45 ms at radius
// factors 1.1, 1.15, 1.18, 1.2, 1.22, 1.25, 1.35 and 1.5 (home cell density,
// cells in counting-sort order); with cells in x order and the three-cell
// density, 3.98, 3.82 and 4.30 ms at 1.15, 1.2 and 1.3.  For large K the count
// inside a ball varies relatively less (about sqrt(K)), so K + 3 sqrt(K) + 3
// is enough, and a row of K up to half the hit buffer fits it.
__host__ __device__ inline float knn_target(float k) {
    const float a = 1.728f * k, b = k + 3.0f * __builtin_sqrtf(k) + 3.0f;
    return a < b ? a : b;
}

template <int METHOD>
__global__ __launch_bounds__(256) void setup_kernel(LatArgs L, TabArgs T, QArgs A) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool range_bad = false, fallback = false, to_list = false, longrow = false;
    if (i < A.Q) {
        uint32_t q[3], row, r, k;
        bool valid = true;
        if (A.qx == nullptr) {
            const uint4 P = L.pts[i];
            q[0] = P.x;
            q[1] = P.y;
            q[2] = P.z;
            row = P.w;
            // objects left out by the build (clipped coordinate >= 2^30) sit
            // after the outside cell; their rows stay empty
            valid = i < L.cs[L.ncells + 1];
        } else {
            q[0] = A.qx[i];
            q[1] = A.qy[i];
            q[2] = A.qz[i];
            row = i;
            for (int a = 0; a < 3; ++a) {
                if ((L.cyc >> a) & 1u)
                    q[a] &= (1u << (L.lg[a] + L.F)) - 1u;
                else if (q[a] >= (1u << 30))
                    valid = false;
            }
            range_bad = !valid;
        }
        r = A.rad ? A.rad[row] : A.rad_u;
        k = A.kk ? A.kk[row] : A.k_u;
        const bool knn = A.mode == SPHIDX_MODE_KNN || (A.mode == SPHIDX_MODE_MIXED && k > 0);
        if (knn && k == 0) valid = false;
        const uint32_t e = 1u << L.F;
        bool inside = true, cyc_ok = true, outside = false;
        uint32_t ncube = 1, nn[3] = {0, 0, 0};
        uint64_t nfull = 1;  // the cube's cells before clipping to the region
        int32_t lo3[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {
            const uint32_t La = 1u << L.lg[a];
            int64_t lo = ((int64_t)q[a] - (int64_t)r) >> L.F;
            int64_t hi = ((int64_t)q[a] + (int64_t)r) >> L.F;
            nfull *= (uint64_t)min(hi - lo + 1, ((L.cyc >> a) & 1u) ? (int64_t)La : hi - lo + 1);
            if ((L.cyc >> a) & 1u) {
                // the sphere walk needs ceil(r/e) <= L/2 - 1 (no offset repeats a cell)
                if (La < 4 || (uint64_t)r > (uint64_t)(La / 2 - 1) * e) cyc_ok = false;
                if (hi - lo + 1 >= (int64_t)La) {
                    lo = 0;
                    hi = La - 1;
                }
            } else {
                if (q[a] >= (La << L.F)) inside = false;
                if (hi >= (int64_t)La) outside = true;
                if (lo < 0) lo = 0;
                if (hi > (int64_t)La - 1) hi = (int64_t)La - 1;
            }
            lo3[a] = (int32_t)lo;
            nn[a] = hi >= lo ? (uint32_t)(hi - lo + 1) : 0u;
            ncube *= nn[a];
        }
        // the tables serve centres inside the region, radii up to their cap
        // and, on cyclic axes, up to the limit where no offset repeats a cell
        const bool tables = METHOD == kSphere || METHOD == kPaper;
        const bool usable = tables && inside && cyc_ok && r <= T.rmax;
        bool sphere = usable, list = false;
        const uint32_t j = (uint32_t)(((uint64_t)r + (1u << T.rshift) - 1u) >> T.rshift);
        if (A.select == 2u) {
            sphere = false;
            list = true;
        } else if (A.select == 1u && valid) {
            // Section III.B/C: the walk with the fewest cells among the sphere
            // table's prefix, the bounding cube clipped to the region and the
            // non-empty cell list; the weight scales the sphere's count against
            // the cube's, and below the reversal distances the sphere is left
            // out (Appendix).  K-NN queries choose only between the sphere and
            // the cube (Section IV.B).
            // Model 1 (this design's reading of the weighting, for a row
            // walk): each walk's lane work, rows visited plus objects tested,
            // the latter as the mean objects per cell times the cells read.
            if (knn) {
                sphere = sphere && r >= A.knn_rev;
            } else {
                sphere = sphere && r >= A.rev;
                const uint64_t load = A.model ? min(((uint64_t)L.n << 8) / L.ncells, (uint64_t)1 << 24) : 0u;
                uint64_t ws = 0, tested = ncube;
                const uint64_t wc = A.model ? (uint64_t)nn[1] * nn[2] * 256u + load * ncube : ncube;
                uint64_t chosen = wc;
                if (sphere) {
                    const uint32_t cls3 = ((q[0] & (e - 1u)) >> (L.F - T.s)) |
                                          (((q[1] & (e - 1u)) >> (L.F - T.s)) << T.s) |
                                          (((q[2] & (e - 1u)) >> (L.F - T.s)) << (2u * T.s));
                    const uint64_t vs = T.vcount[(size_t)cls3 * T.nr + j];
                    if (A.model) {
                        // every table row takes a lane; objects are read only
                        // in the region: the sphere's cells scaled by the
                        // part of its bounding cube inside the region
                        const uint32_t rcls = cls3 >> T.s;
                        tested = vs * ncube / nfull;
                        ws = (uint64_t)T.rindex[(size_t)rcls * T.nr + j] * 256u + load * tested;
                    } else {
                        ws = vs;
                    }
                    sphere = (unsigned __int128)ws * A.weight <= (unsigned __int128)wc * 256u;
                    if (sphere) chosen = ws;
                }
                if (L.ncl) {
                    const uint64_t nl = *L.ncl;
                    // the list tests the objects of the cells the sphere meets
                    // (with the sphere left out: the cube's)
                    const uint64_t wl = A.model ? nl * 256u + load * tested : nl;
                    if (wl < chosen) {
                        sphere = false;
                        list = true;
                    }
                }
            }
        }
        fallback = valid && tables && !usable;
        // (chosen per query: the main kernels take every walk themselves)
        to_list = valid && tables && !sphere && A.select != 1u;
        // a radius row of the main kernels expected (at the lattice's mean
        // density) to pass 5/4 of a wavefront's row buffer: with the stash
        // and the block kernel, one block counts, orders and keeps it in a
        // single walk instead of a count walk and a write walk
        // (not with per-query statistics, which that kernel does not keep)
        if (valid && !knn && !to_list && A.stash && A.long_waves > 1 && !A.stats) {
            const float rc = (float)r / (float)e;
            const float expect = 4.18879f * rc * rc * rc * ((float)L.n / (float)L.ncells);
            longrow = expect > 1.25f * (float)A.sort_cap;
        }
        uint32_t tb = 0, tend = 0, kb = 0, kend = 0;
        if (METHOD == kPaper && sphere && valid) {
            // the paper's tables (Section III.A): with d = r / e, the unshaved
            // table below floor(d)^2, then, up to floor(d^2), the table chosen
            // by the six flags [frac(d) < zeta] (zeta: e - f up, f down);
            // tb = the specialised part's first entry, ncube = the unshaved
            // entries before it, tend = all entries
            const uint32_t D0 = r >> L.F, fu = r & (e - 1u);
            uint32_t tsel = 0;
            for (int a = 0; a < 3; ++a) {
                const uint32_t f = q[a] & (e - 1u);
                if (fu < e - f) tsel |= 1u << (2 * a);
                if (fu < f) tsel |= 1u << (2 * a + 1);
            }
            const uint32_t lo2 = D0 * D0;
            const uint32_t b2max = (uint32_t)(((uint64_t)r * r) >> (2 * L.F));
            const uint32_t* base_lo = T.p_lo + (size_t)64 * T.p_nb2;
            const uint32_t* spec_lo = T.p_lo + (size_t)tsel * T.p_nb2;
            const uint32_t nbase = base_lo[lo2] - base_lo[0];
            tb = spec_lo[lo2];
            tend = nbase + (spec_lo[b2max + 1] - tb);
            ncube = nbase;
        } else if (sphere && valid) {
            // row tables are specialised on the (y, z) sub-cell position
            const uint32_t cls = ((q[1] & (e - 1u)) >> (L.F - T.s)) | (((q[2] & (e - 1u)) >> (L.F - T.s)) << T.s);
            tb = T.cstart[cls];
            tend = T.rindex[(size_t)cls * T.nr + j];
            if (knn) {
                // K-NN: a first search radius expected to hold knn_target(K)
                // objects at the density of the home cell and its two
                // neighbours along x (one contiguous range of counts; the
                // lattice mean as a floor), and its table prefix; the grouped
                // count searches it as a radius row and keeps the first K
                // when it holds K.  (The home cell alone sent 3.4 % of the
                // clustered K = 16 rows to the one-query-per-wave kernel,
                // the three cells 2.0 %: 4.04 -> 3.82 ms per step.)
                const uint32_t home = pack_cell(L, q[0] >> L.F, q[1] >> L.F, q[2] >> L.F);
                const uint32_t hl = home > 0u ? home - 1u : 0u, hr = min(home + 2u, L.ncells);
                const float dens =
                    fmaxf((float)L.n / (float)L.ncells, (float)(L.cs[hr] - L.cs[hl]) / (float)(hr - hl));
                const float rho = (float)e * cbrtf(0.2387f * knn_target((float)k) / fmaxf(dens, 1e-6f));
                kb = rho >= (float)r ? r : max(1u, (uint32_t)rho);
                const uint32_t jb = (uint32_t)(((uint64_t)kb + (1u << T.rshift) - 1u) >> T.rshift);
                kend = T.rindex[(size_t)cls * T.nr + jb];
            }
        }
        if (list) {
            // the walk takes nn[1] * nn[2] entries: the whole list
            nn[0] = 0u;
            nn[1] = *L.ncl;
            nn[2] = 1u;
            lo3[0] = lo3[1] = lo3[2] = 0;
        }
        if (A.method_out)
            A.method_out[row] = !valid ? 0xFFFFFFFFu
                                       : sphere ? SPHIDX_METHOD_SPHERE : list ? SPHIDX_METHOD_LIST : SPHIDX_METHOD_CUBE;
        const uint32_t flags = (valid ? F_VALID : 0u) | (knn ? F_KNN : 0u) | (sphere ? F_SPHERE : 0u) |
                               (outside ? F_OUTSIDE : 0u) | (list ? F_LIST : 0u) | (longrow ? F_LONG : 0u);
        uint4* d = A.desc + 4 * (size_t)i;
        d[0] = make_uint4(q[0], q[1], q[2], row);
        d[1] = make_uint4(r, k, flags, tb);
        // (sphere K-NN queries walk no cube: its fields carry the first radius)
        const bool kfirst = METHOD != kPaper && sphere && valid && knn;
        d[2] = make_uint4(tend, kfirst ? kb : ncube, kfirst ? kend : nn[0], nn[1]);
        d[3] = make_uint4((uint32_t)lo3[0], (uint32_t)lo3[1], (uint32_t)lo3[2], nn[2]);
    }
    // queries for the fallback list's kernels (bounding cube or cell list):
    // one atomic per wavefront, the wavefront's queries in order
    const uint64_t lm = __ballot(to_list);
    if (lm) {
        uint32_t base = 0;
        if (lane_id() == 0) base = atomicAdd(A.fb_count, (uint32_t)__popcll(lm));
        base = uni(base);
        if (to_list) A.fbq[base + lanes_below(lm)] = i;
    }
    const uint64_t gm = __ballot(longrow);
    if (gm) {
        uint32_t base = 0;
        if (lane_id() == 0) base = atomicAdd(A.lq_count, (uint32_t)__popcll(gm));
        base = uni(base);
        if (longrow) A.lq[base + lanes_below(gm)] = i;
    }
    if (__ballot(range_bad) && lane_id() == 0) atomicOr(L.status, SPHIDX_FLAG_RANGE);
    if (__ballot(fallback) && lane_id() == 0) atomicOr(L.status, SPHIDX_FLAG_FALLBACK);
}

// Descriptors are read through the scalar cache (the address is uniform and
// the array was written by an earlier kernel).
typedef __attribute__((address_space(4))) const uint32_t const_u32;

__device__ __forceinline__ Query load_query(const LatArgs& L, const QArgs& A, uint32_t qi) {
    Query s;
    const const_u32* d = (const const_u32*)(A.desc + 4 * (size_t)uni(qi));
    s.q[0] = d[0];
    s.q[1] = d[1];
    s.q[2] = d[2];
    s.row = d[3];
    s.r = d[4];
    s.k = d[5];
    s.flags = d[6];
    s.tb = d[7];
    s.tend = d[8];
    s.ncube = d[9];
    if (!(s.flags & F_SPHERE)) {
        s.nn[0] = d[10];
        s.nn[1] = d[11];
        s.nn[2] = d[15];
        s.lo[0] = (int32_t)d[12];
        s.lo[1] = (int32_t)d[13];
        s.lo[2] = (int32_t)d[14];
    }
    s.kbr = (s.flags & F_KBOUND) ? d[12] : 0u;
    s.self = (A.qx == nullptr && (A.flags & SPHIDX_EXCLUDE_SELF)) ? qi : kMaxId;
    const uint32_t e = 1u << L.F;
    for (int a = 0; a < 3; ++a) {
        s.c[a] = s.q[a] >> L.F;
        s.f[a] = s.q[a] & (e - 1u);
        s.up[a] = e - s.f[a];
        s.dn[a] = s.f[a] + 1u;
    }
    s.r2 = (uint64_t)s.r * (uint64_t)s.r;
    return s;
}

// Cells of the bounding cube of query s (in-region cells only), for stats.
__device__ __forceinline__ uint32_t cube_cells(const LatArgs& L, const Query& s) {
    uint32_t n = 1;
    for (int a = 0; a < 3; ++a) {
        const int64_t La = (int64_t)1 << L.lg[a];
        int64_t lo = ((int64_t)s.q[a] - (int64_t)s.r) >> L.F;
        int64_t hi = ((int64_t)s.q[a] + (int64_t)s.r) >> L.F;
        if ((L.cyc >> a) & 1u) {
            if (hi - lo + 1 >= La) {
                lo = 0;
                hi = La - 1;
            }
        } else {
            if (lo < 0) lo = 0;
            if (hi > La - 1) hi = La - 1;
        }
        n *= hi >= lo ? (uint32_t)(hi - lo + 1) : 0u;
    }
    return n;
}

// Row j of the class table that starts at tb ((y, z) class cls): from the
// staged copy when it holds it, else from device memory.
template <bool TLDS>
__device__ __forceinline__ uint32_t row_word(const TabArgs& T, const uint32_t* tab_lds, uint32_t tb, uint32_t cls,
                                             uint32_t j) {
    if (TLDS) {
        if (T.lds_chunk == 0) return tab_lds[tb + j];
        if (j < T.lds_chunk) return tab_lds[cls * T.lds_chunk + j];
    }
    return T.rows[tb + j];
}

// (y, z) sub-cell class of a query (the row table it walks).
__device__ __forceinline__ uint32_t row_class(const LatArgs& L, const TabArgs& T, const uint32_t* f) {
    return (f[1] >> (L.F - T.s)) | ((f[2] >> (L.F - T.s)) << T.s);
}

// ---------------------------------------------------------------------------
// Rows of the walk

// Per lane, one x-row of cells: up to two object ranges to test (two when
// the run of cells wraps around a cyclic x axis), a range of objects in cells
// wholly inside the sphere (counted without reading them), and the number
// of cells of the row the sphere meets.
struct RowRef {
    uint32_t st0, cnt0, st1, cnt1;
    uint32_t ist, icnt;
    uint32_t kept;
    bool plain;  // one range (st1, cnt1): the run neither wraps nor has a wholly-inside part
};

// Per-axis distance from a position f inside the home cell to the farthest
// position of the cell at offset o along that axis.
__device__ __forceinline__ uint32_t axis_far(int o, uint32_t f, uint32_t F) {
    const uint32_t e = 1u << F;
    if (o > 0) return (((uint32_t)o + 1u) << F) - 1u - f;
    if (o < 0) return f + ((uint32_t)(-o) << F);
    return max(f, e - 1u - f);
}

// s^2 for s < 2^24: two 24-bit multiplies (low and high word) instead of a
// 64-bit multiply-add.
__device__ __forceinline__ uint64_t sq24(uint32_t s) {
    const uint32_t t = s & 0xFFFFFFu;
    return (uint64_t)t * t;
}

// floor(sqrt(v)) for v < 2^62.
// Below 2^41 (roots below 2^20.5): v in single precision (the high word is
// exact, the low word and the sum round once each: relative error at most
// 1.5 x 2^-24) and the hardware square root (within 1 ulp) give the root to
// within 0.25, so its truncation is the floor or one either side of it; two
// exact steps with 24-bit products settle it.
// Above: the hardware reciprocal square root in double precision (relative
// error about 2^-23) and one Newton step give the root to about 2^-45
// relative, well within one unit below 2^31; exact integer steps settle the
// floor.  (v = 0 takes the first branch.)
__device__ __forceinline__ uint32_t isqrt64(uint64_t v) {
    const uint32_t hi = (uint32_t)(v >> 32);
    uint32_t s;
    if (hi < (1u << 9)) {
        const float fv = __builtin_fmaf((float)hi, 4294967296.0f, (float)(uint32_t)v);
        s = (uint32_t)__builtin_amdgcn_sqrtf(fv);
        if (sq24(s) > v) --s;
        if (sq24(s + 1u) <= v) ++s;
    } else {
        const double d = (double)v;
        const double y = __builtin_amdgcn_rsq(d);
        double x = d * y;
        x = __builtin_fma(x, __builtin_fma(-x, 0.5 * y, 0.5), x);
        s = (uint32_t)x;
        if ((uint64_t)s * s > v) --s;
        if ((uint64_t)s * s > v) --s;
        if ((uint64_t)(s + 1u) * (s + 1u) <= v) ++s;
    }
    return s;
}

// Turn an unwrapped x-run [a, b] of the row starting at cell `base` (and its
// wholly-inside part [ia, ib], empty when ia > ib) into object ranges.  On a
// cyclic axis the run (shorter than the axis) may cross the world edge once:
// it is then two pieces and is tested whole; on a clipped axis it is clamped
// to the region.  Lanes with `live` false get empty ranges (their loads read
// the row start, always a valid index).
__device__ __forceinline__ RowRef row_ranges(const LatArgs& L, uint32_t base, int a, int b, int ia, int ib,
                                             bool live) {
    const int Lx = 1 << L.lg[0];
    int p0, p1, p2, p3;
    bool has_int = ia <= ib;
    bool wrap = false;
    if (L.cyc & 1u) {
        const bool lo_out = a < 0, hi_out = b >= Lx;
        wrap = lo_out || hi_out;
        // pieces in memory order when wrapped: [0, e0) then [s1, Lx)
        const int e0 = lo_out ? b + 1 : b - Lx + 1;
        const int s1 = lo_out ? a + Lx : a;
        ia = max(ia, a);
        ib = min(ib, b);
        has_int = has_int && !wrap && ia <= ib;
        p0 = wrap ? 0 : a;
        p1 = wrap ? e0 : (has_int ? ia : a);
        p2 = wrap ? s1 : (has_int ? ib + 1 : a);
        p3 = wrap ? Lx : b + 1;
    } else {
        a = max(a, 0);
        b = min(b, Lx - 1);
        live = live && a <= b;
        ia = max(ia, a);
        ib = min(ib, b);
        has_int = has_int && ia <= ib;
        p0 = a;
        p1 = has_int ? ia : a;
        p2 = has_int ? ib + 1 : a;
        p3 = b + 1;
    }
    if (!live) p0 = p1 = p2 = p3 = 0;
    const uint32_t* row = L.cs + base;
    // a plain run is one range [p0, p3): its middle bounds are needed only
    // when it wraps or has a wholly-inside part
    const uint32_t v0 = row[p0], v3 = row[p3];
    uint32_t v1 = v0, v2 = v0;
    if (wrap || has_int) {
        v1 = row[p1];
        v2 = row[p2];
    }
    RowRef r;
    r.st0 = v0;
    r.cnt0 = v1 - v0;
    r.st1 = v2;
    r.cnt1 = v3 - v2;
    r.ist = v1;
    r.icnt = has_int ? v2 - v1 : 0u;
    r.kept = (uint32_t)(wrap ? (p1 - p0) + (p3 - p2) : (p3 - p0));
    r.plain = !wrap && !has_int;
    return r;
}

// Cells in x order (objects inside each cell by x, cells of a row in x
// order): the objects of a plain run have increasing x, and those within the
// sphere's x-slab [qx - X, qx + X] on this row are one sub-range, found by
// two binary searches on x (interleaved, so that their loads overlap).  Only
// for rows with many objects, where the searches cost less than testing the
// objects outside the slab.
constexpr uint32_t kNarrowMin = 24;

__device__ __forceinline__ void narrow_x(const LatArgs& L, RowRef& r, uint32_t qx, uint32_t X) {
    const uint32_t* xs = (const uint32_t*)L.pts;  // x of sorted position p at xs[4 p]
    const uint32_t lo_t = qx > X ? qx - X : 0u, hi_t = qx + X;
    uint32_t a = r.st1, na = r.cnt1, b = r.st1, nb = r.cnt1;
    while (na | nb) {
        if (na) {
            const uint32_t h = na >> 1;
            if (xs[4 * (a + h)] < lo_t) {
                a += h + 1;
                na -= h + 1;
            } else {
                na = h;
            }
        }
        if (nb) {
            const uint32_t h = nb >> 1;
            if (xs[4 * (b + h)] <= hi_t) {
                b += h + 1;
                nb -= h + 1;
            } else {
                nb = h;
            }
        }
    }
    r.st1 = a;
    r.cnt1 = b - a;
}

// Squared distance along one axis from the query to the nearest position of
// the cell at offset o: 0 for o = 0, else (|o| - 1) cells plus the distance
// to the shared face (up = e - f above, dn = f + 1 below).  A lower bound
// only (the callers keep a cell or a row when it is within the bound, and
// test its objects exactly): a distance of 2^24 units or more is taken as
// 2^24 - 1, so that the square takes 24-bit products.
__device__ __forceinline__ uint64_t axis_gap2(int o, uint32_t up, uint32_t dn, uint32_t F) {
    const uint32_t ao = (uint32_t)(o < 0 ? -o : o);
    const uint32_t g = o == 0 ? 0u : ((ao - 1u) << F) + (o > 0 ? up : dn);
    return sq24(min(g, 0xFFFFFFu));
}

// Row (oy, oz) of the sphere table: the cells it meets are those whose
// x-gap satisfies gx^2 <= bound^2 - gy^2 - gz^2 -- the exact test of Eq. 1
// solved for x, one contiguous run; the wholly-inside cells solve the same
// with the far distances (Section III.A, last paragraph).
__device__ __forceinline__ RowRef sphere_row(const LatArgs& L, const Query& s, uint32_t w, bool has, uint64_t bound2,
                                             bool interior) {
    const int oy = ((int)(w << 16)) >> 16, oz = ((int)w) >> 16;
    const uint32_t Ly = 1u << L.lg[1], Lz = 1u << L.lg[2];
    uint32_t ty = (uint32_t)((int)s.c[1] + oy), tz = (uint32_t)((int)s.c[2] + oz);
    bool live = has;
    if (L.cyc & 2u)
        ty &= Ly - 1u;
    else
        live = live && ty < Ly;
    if (L.cyc & 4u)
        tz &= Lz - 1u;
    else
        live = live && tz < Lz;
    const uint64_t gyz = axis_gap2(oy, s.up[1], s.dn[1], L.F) + axis_gap2(oz, s.up[2], s.dn[2], L.F);
    live = live && gyz <= bound2;
    const uint32_t X = isqrt64(live ? bound2 - gyz : 0u);
    const uint32_t fx = s.f[0];
    const int npos = (int)((X + fx) >> L.F);
    const int nneg = X > fx ? (int)((X - fx - 1u) >> L.F) + 1 : 0;
    int ia = 1, ib = 0;
    if (interior) {
        const uint32_t hy = axis_far(oy, s.f[1], L.F), hz = axis_far(oz, s.f[2], L.F);
        const uint64_t hyz = sq(hy) + sq(hz);
        const uint32_t Xi = isqrt64(hyz <= s.r2 ? s.r2 - hyz : 0u);
        if (hyz <= s.r2 && Xi >= fx && Xi + fx + 1u >= (1u << L.F)) {
            ib = (int)s.c[0] + (int)((Xi + fx + 1u) >> L.F) - 1;
            ia = (int)s.c[0] - (int)((Xi - fx) >> L.F);
        }
    }
    if (!live) {
        ty = 0;
        tz = 0;
    }
    const uint32_t base = (tz << (L.lg[0] + L.lg[1])) | (ty << L.lg[0]);
    RowRef rr = row_ranges(L, base, (int)s.c[0] - nneg, (int)s.c[0] + npos, ia, ib, live);
    if (L.xsorted && rr.plain && rr.cnt1 >= kNarrowMin && *L.xsorted) narrow_x(L, rr, s.q[0], X);
    return rr;
}

// Row e of the bounding cube (no test: the bin-lattice scans every cell).
__device__ __forceinline__ RowRef cube_row(const LatArgs& L, const Query& s, uint32_t e, bool has, double inv_ny) {
    if (!has) e = 0;
    const uint32_t iz = exact_div(e, s.nn[1], inv_ny);
    const uint32_t iy = e - iz * s.nn[1];
    uint32_t ty = (uint32_t)(s.lo[1] + (int32_t)iy), tz = (uint32_t)(s.lo[2] + (int32_t)iz);
    if (L.cyc & 2u) ty &= (1u << L.lg[1]) - 1u;
    if (L.cyc & 4u) tz &= (1u << L.lg[2]) - 1u;
    if (!has) {
        // lanes without a row read the first row (always a valid index)
        ty = 0u;
        tz = 0u;
    }
    const uint32_t base = (tz << (L.lg[0] + L.lg[1])) | (ty << L.lg[0]);
    return row_ranges(L, base, s.lo[0], s.lo[0] + (int)s.nn[0] - 1, 1, 0, has);
}

// Entry `ent` of the non-empty cell list (Section III.B): the cell's objects
// are one range, kept when the cell's nearest position is within the radius
// -- the rejection of cells that are too far, instead of the sphere's
// rejection of empty cells.  On a cyclic axis the cell's offset is taken to
// the nearest image, o in [-L/2, L/2); at o = -L/2 the image at +L/2 is as
// many cells away, and the nearer face of the two counts.
__device__ __forceinline__ RowRef list_row(const LatArgs& L, const Query& s, uint32_t ent, bool has, uint64_t bound2) {
    // lanes without an entry read entry 0 (the closing entry of an empty
    // list), always present
    const uint2 c = L.cells[has ? ent : 0u];
    const uint32_t end = L.cells[has ? ent + 1u : 0u].y;
    const uint32_t cc[3] = {c.x & ((1u << L.lg[0]) - 1u), (c.x >> L.lg[0]) & ((1u << L.lg[1]) - 1u),
                            c.x >> (L.lg[0] + L.lg[1])};
    uint64_t g2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int o = (int)cc[a] - (int)s.c[a];
        uint32_t up = s.up[a], dn = s.dn[a];
        if ((L.cyc >> a) & 1u) {
            const int La = 1 << L.lg[a];
            o = ((o + La / 2) & (La - 1)) - La / 2;
            if (La >= 2 && o == -(La / 2)) dn = min(up, dn);
        }
        g2 += axis_gap2(o, up, dn, L.F);
    }
    const bool keep = has && g2 <= bound2;
    RowRef r;
    r.st0 = c.y;
    r.cnt0 = keep ? end - c.y : 0u;
    r.st1 = c.y;
    r.cnt1 = 0u;
    r.ist = c.y;
    r.icnt = 0u;
    r.kept = keep ? 1u : 0u;
    r.plain = false;
    return r;
}

// Entry `ent` of the paper's tables (Section III.A), one cell: the unshaved
// table's entries below floor(d)^2 come first (ent < s.ncube), then the
// query's specialised table from s.tb.  Cells with b e >= thr -- b at or
// above d - 1 when thr = (r - e)^2 -- take the run-time test of Eq. 1 with
// the paper's per-axis distances (b_o cells plus the distance to the face,
// e - f up and f down); objects of the kept cell are then tested one by one.
__device__ __forceinline__ RowRef paper_row(const LatArgs& L, const TabArgs& T, const Query& s, uint32_t ent,
                                            bool has, uint64_t bound2, uint64_t thr2) {
    const uint32_t idx = ent < s.ncube ? T.p_lo[(size_t)64 * T.p_nb2] + ent : s.tb + (ent - s.ncube);
    const uint32_t w = has ? T.p_off[idx] : 0u;
    const uint64_t b2e = has ? (uint64_t)T.p_b2[idx] << (2 * L.F) : 0ull;
    const int o[3] = {((int)(w << 22)) >> 22, ((int)(w << 12)) >> 22, ((int)(w << 2)) >> 22};
    const uint32_t e = 1u << L.F;
    bool live = has;
    uint32_t t[3];
    uint64_t g2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint32_t La = 1u << L.lg[a];
        uint32_t v = (uint32_t)((int)s.c[a] + o[a]);
        if ((L.cyc >> a) & 1u)
            v &= La - 1u;
        else
            live = live && v < La;
        t[a] = v;
        const uint32_t ao = (uint32_t)(o[a] < 0 ? -o[a] : o[a]);
        const uint64_t g = o[a] == 0 ? 0ull : ((uint64_t)(ao - 1u) << L.F) + (o[a] > 0 ? e - s.f[a] : s.f[a]);
        g2 += g * g;
    }
    if (b2e >= thr2 && g2 > bound2) live = false;
    if (!live) t[0] = t[1] = t[2] = 0u;
    const uint32_t cell = pack_cell(L, t[0], t[1], t[2]);
    const uint32_t st = L.cs[cell];
    RowRef r;
    r.st0 = st;
    r.cnt0 = live ? L.cs[cell + 1] - st : 0u;
    r.st1 = st;
    r.cnt1 = 0u;
    r.ist = st;
    r.icnt = 0u;
    r.kept = live ? 1u : 0u;
    r.plain = false;
    return r;
}

// Minimum-image squared distance of an object to the centre: on a cyclic
// axis ((p - q + W/2) mod W) - W/2; on a clipped axis plain p - q (both below
// 2^30, so the difference fits an int).
struct AxisWrap {
    uint32_t half[3];
    uint32_t mask[3];
};

__device__ __forceinline__ AxisWrap axis_wrap(const LatArgs& L) {
    AxisWrap w;
    for (int a = 0; a < 3; ++a) {
        if ((L.cyc >> a) & 1u) {
            const uint32_t W = 1u << (L.lg[a] + L.F);
            w.half[a] = W >> 1;
            w.mask[a] = W - 1u;
        } else {
            w.half[a] = 0u;
            w.mask[a] = 0xFFFFFFFFu;
        }
    }
    return w;
}

__device__ __forceinline__ uint64_t obj_dist2(const AxisWrap& w, const Query& s, const uint4& P) {
    const uint32_t pv[3] = {P.x, P.y, P.z};
    uint64_t d2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int32_t dd = (int32_t)(((pv[a] - s.q[a]) + w.half[a]) & w.mask[a]) - (int32_t)w.half[a];
        d2 += (uint64_t)((int64_t)dd * dd);
    }
    return d2;
}

// ---------------------------------------------------------------------------
// Candidate distribution: each lane holds two object ranges [st0, st0+cnt0)
// and [st1, st1+cnt1); every object becomes one slot, 64 slots per step.
// visit(active, position, record) returns true to stop (uniformly).

template <typename V>
__device__ __forceinline__ bool for_candidates(const LatArgs& L, uint32_t st0, uint32_t cnt0, uint32_t st1,
                                               uint32_t cnt1, uint32_t* own, uint32_t& total_out, V&& visit) {
    const uint32_t lane = lane_id();
    const uint32_t tl = cnt0 + cnt1;
    const uint32_t incl = scan_add(tl);
    const uint32_t total = lane_val(incl, 63);
    total_out += total;
    if (total == 0) return false;
    const uint32_t excl = incl - tl;
    const uint32_t smx0 = st0 - excl;
    const uint32_t bnd = excl + cnt0;
    const uint32_t smx1 = st1 - bnd;
    // slot cb + lane: mark where each lane's range starts inside the step's
    // 64 slots, then a max-scan hands every slot to the lane that owns it (a
    // step past the end marks nothing: lane 0 stands in)
    auto locate = [&](uint32_t cb, uint32_t& p) -> bool {
        wave_sync();
        own[lane] = 0;
        wave_sync();
        if (tl > 0 && excl < cb + 64 && incl > cb) own[excl > cb ? excl - cb : 0] = lane + 1;
        wave_sync();
        const uint32_t o = max(scan_max(own[lane]), 1u) - 1u;
        const uint32_t g = cb + lane;
        const uint32_t b = bperm(bnd, o);
        const uint32_t p0 = bperm(smx0, o) + g;
        const uint32_t p1 = bperm(smx1, o) + g;
        p = g < b ? p0 : p1;
        return g < total;
    };
    // two register sets taken in turn: the step after the one being visited
    // is already loading (lanes past the end load record 0, present whenever
    // a candidate is, and visit nothing)
    uint32_t pa = 0, pb = 0;
    bool aa = locate(0, pa), ab = false;
    uint4 PA = L.pts[aa ? pa : 0u], PB = PA;
    for (uint32_t cb = 0; cb < total; cb += 128) {
        ab = locate(cb + 64, pb);
        PB = L.pts[ab ? pb : 0u];
        if (visit(aa, pa, PA)) return true;
        if (cb + 64 >= total) break;
        aa = locate(cb + 128, pa);
        PA = L.pts[aa ? pa : 0u];
        if (visit(ab, pb, PB)) return true;
    }
    return false;
}

// Walk the query's rows: sphere-table rows or bounding-cube rows, 64 per
// step, one per lane.  When objects outside the region may be within r, the
// outside cell (Section II.B: every such object lives in one cell) is a
// leading pseudo-row of the first step.  on_step(row) returns true to stop.
// bound2_now() is re-read before every step (top-M shrinks it); KEY_STOP
// enables the cut-off on sorted row keys; `interior` marks the cells wholly
// inside the sphere (count pass).
// The steps of 64 entries a wavefront takes start at `first` and follow
// every `stride` entries (a block of W waves walks one row with first =
// 64 w, stride = 64 W; a lone wave takes them all).
template <int METHOD, bool TLDS, bool KEY_STOP, typename B, typename S>
__device__ __forceinline__ void walk(const LatArgs& L, const TabArgs& T, const uint32_t* tab_lds, const Query& s,
                                     bool interior, uint32_t& walked, B&& bound2_now, S&& on_step,
                                     uint32_t first = 0, uint32_t stride = 64) {
    const uint32_t lane = lane_id();
    const uint32_t pre = (s.flags & F_OUTSIDE) ? 1u : 0u;
    const bool sphere = METHOD == kSphere || ((METHOD == kEither || METHOD == kPaper) && (s.flags & F_SPHERE));
    const uint32_t nent = sphere ? s.tend : s.nn[1] * s.nn[2];
    const uint32_t total = nent + pre;
    const uint32_t rcls = TLDS ? row_class(L, T, s.f) : 0u;
    // entry index of this lane's row in the current step (pseudo-row: ~0)
    uint32_t ent = lane - pre + first;
    uint32_t nxt = 0;
    if (METHOD != kPaper && sphere && ent < nent) nxt = row_word<TLDS>(T, tab_lds, s.tb, rcls, ent);
    const double inv_ny = (!sphere && s.nn[1]) ? 1.0 / (double)s.nn[1] : 0.0;
    for (uint32_t base = first; base < total; base += stride, ent += stride) {
        const bool is_out = pre && base == 0 && lane == 0;
        RowRef r;
        if (METHOD == kPaper && sphere) {
            const uint64_t bound2 = bound2_now();
            // entries are sorted by b^2, and b e is below every cell's
            // distance: once b^2 e^2 exceeds the bound nothing further can
            // hold anything closer
            if (KEY_STOP && base > 0) {
                const uint32_t j = base - pre;
                const uint32_t idx = j < s.ncube ? T.p_lo[(size_t)64 * T.p_nb2] + j : s.tb + (j - s.ncube);
                if (((uint64_t)uni(T.p_b2[idx]) << (2 * L.F)) > bound2) break;
            }
            // the run-time test from b >= d - 1 on (every cell when d < 1)
            const uint32_t e = 1u << L.F;
            const uint32_t rt = uni(isqrt64(bound2));
            const uint64_t thr2 = rt > e ? sq(rt - e) : 0ull;
            r = paper_row(L, T, s, ent, ent < nent, bound2, thr2);
        } else if (METHOD == kSphere || (METHOD == kEither && sphere)) {
            const uint64_t bound2 = bound2_now();
            // rows are sorted by key: once the key exceeds the bound no
            // further row can hold anything closer (the first row's key is 0)
            if (KEY_STOP && base > 0 && uni64((uint64_t)T.rkey[s.tb + base - pre]) > bound2) break;
            const uint32_t w = nxt;
            if (ent + stride < nent) nxt = row_word<TLDS>(T, tab_lds, s.tb, rcls, ent + stride);
            r = sphere_row(L, s, w, ent < nent, bound2, interior);
        } else if (s.flags & F_LIST) {
            r = list_row(L, s, ent, ent < nent, bound2_now());
        } else {
            r = cube_row(L, s, ent, ent < nent, inv_ny);
        }
        if (is_out) {
            r.st0 = L.cs[L.ncells];
            r.cnt0 = L.cs[L.ncells + 1] - r.st0;
            r.cnt1 = 0u;
            r.icnt = 0u;
            r.kept = 0u;
        }
        walked += min(64u, total - base) - (base == 0 ? pre : 0u);
        if (on_step(r)) return;
    }
}

// ---------------------------------------------------------------------------
// Query scheduling: plain (each wave owns a fixed slice of `tile` queries,
// XCD-aware block order) or persistent (per-XCD work queues).

// Persistent grabs shrink with the work: about two per resident wave, at
// least `tmin` and at most A.tile (64 for the lists), so that a short batch
// or list of heavy queries is shared out instead of landing on a few waves,
// and a long one does not pay an atomic per query.
template <typename F>
__device__ __forceinline__ void for_each_range(uint32_t Q, const QArgs& A, uint32_t* queues, F&& f,
                                               uint32_t tmin = 1u) {
    if (Q == 0) return;
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t tmax = A.list ? 64u : A.tile;
    const uint32_t tile =
        A.persistent ? max(tmin, min(tmax, (uint32_t)((uint64_t)Q / ((uint64_t)gridDim.x * nw * 2u)))) : A.tile;
    // plain: consecutive block ids go round-robin over the 8 XCDs; give each
    // XCD a contiguous range of slices so neighbouring queries share its L2.
    // persistent: SPHIDX_NQUEUE queues, each over a contiguous range of
    // queries and served by blocks of one XCD (several queues per XCD, so
    // that fewer waves share each counter); a wave drains its own queue, then
    // looks at all the others at once and moves to the first with work left,
    // and stops when none has any.  Queues only drain, so every wave stops.
    uint32_t x = blockIdx.x % (A.persistent ? SPHIDX_NQUEUE : SPHIDX_NXCD);
    bool first = true;
    for (;;) {
        uint32_t b = 0, e = 0;
        if (!A.persistent) {
            if (!first) break;
            const uint32_t G = gridDim.x, bi = blockIdx.x;
            const uint32_t full = G / SPHIDX_NXCD, rem = G % SPHIDX_NXCD;
            const uint32_t lb = x * full + min(x, rem) + bi / SPHIDX_NXCD;
            const uint64_t q0 = ((uint64_t)lb * nw + wave) * tile;
            b = (uint32_t)min(q0, (uint64_t)Q);
            e = (uint32_t)min(q0 + tile, (uint64_t)Q);
        } else {
            const uint32_t qs = (uint32_t)(((uint64_t)x * Q) / SPHIDX_NQUEUE);
            const uint32_t qe = (uint32_t)(((uint64_t)(x + 1) * Q) / SPHIDX_NQUEUE);
            uint32_t* qc = queues + x * SPHIDX_QSTRIDE;
            uint32_t t = 0;
            if (lane == 0) {
                // an exhausted queue is skipped with a plain read, not an atomic
                t = __hip_atomic_load(qc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((uint64_t)qs + t < qe) t = atomicAdd(qc, tile);
            }
            t = uni(t);
            if ((uint64_t)qs + t >= qe) {
                // lane l reads queue x + 1 + l
                bool left = false;
                if (lane + 1u < SPHIDX_NQUEUE) {
                    const uint32_t y = (x + 1u + lane) % SPHIDX_NQUEUE;
                    const uint32_t ys = (uint32_t)(((uint64_t)y * Q) / SPHIDX_NQUEUE);
                    const uint32_t ye = (uint32_t)(((uint64_t)(y + 1) * Q) / SPHIDX_NQUEUE);
                    const uint32_t ty =
                        __hip_atomic_load(queues + y * SPHIDX_QSTRIDE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    left = (uint64_t)ys + ty < ye;
                }
                const uint64_t m = __ballot(left);
                if (m == 0) break;
                x = (x + 1u + (uint32_t)__builtin_ctzll(m)) % SPHIDX_NQUEUE;
                continue;
            }
            b = qs + t;
            e = (uint32_t)min((uint64_t)qe, (uint64_t)qs + t + tile);
        }
        first = false;
        if (b < e) f(b, e);
    }
}

template <typename F>
__device__ __forceinline__ void for_each_query(uint32_t Q, const QArgs& A, uint32_t* queues, F&& f) {
    for_each_range(Q, A, queues, [&](uint32_t b, uint32_t e) {
        for (uint32_t qi = b; qi < e; ++qi) f(qi);
    });
}

// Stage the row table in LDS (shared by the block's waves): the whole table,
// or, in chunks, the first lds_chunk rows of every (y, z) class -- the rows
// nearest the centre, which every query of the class walks first.
template <bool TLDS>
__device__ __forceinline__ const uint32_t* stage_table(const TabArgs& T, char* smem) {
    if (!TLDS) return nullptr;
    uint32_t* t = (uint32_t*)smem;
    if (T.lds_chunk == 0) {
        for (uint32_t i = threadIdx.x; i < T.total; i += blockDim.x) t[i] = T.rows[i];
    } else {
        const uint32_t n = T.nrcls * T.lds_chunk;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const uint32_t c = i / T.lds_chunk, j = i - c * T.lds_chunk;
            const uint32_t b = T.cstart[c];
            t[i] = b + j < T.cstart[c + 1] ? T.rows[b + j] : 0u;
        }
    }
    __syncthreads();
    return t;
}

template <bool TLDS>
__device__ __forceinline__ size_t table_lds_bytes(const TabArgs& T) {
    if (!TLDS) return 0;
    const size_t words = T.lds_chunk ? (size_t)T.nrcls * T.lds_chunk : (size_t)T.total;
    return (words * 4 + 15) & ~(size_t)15;
}



// ---------------------------------------------------------------------------
// Ordering a row by (dist^2, id) in LDS.

__device__ __forceinline__ void store_sorted(const QArgs& A, const uint64_t* td, const uint32_t* ti, uint32_t n,
                                             int64_t dst) {
    for (uint32_t t = lane_id(); t < n; t += 64) {
        A.out_ids[dst + t] = ti[t];
        if (A.out_d2) A.out_d2[dst + t] = (int64_t)td[t];
    }
}

// Sort the n <= cap pairs (td, ti) of one row by (dist^2, id) and store them
// at dst.  Every pair has dist^2 <= r2, so the bucket
// floor(n * dist^2 / r2) (float arithmetic: monotone in dist^2) never puts a
// larger distance in an earlier bucket; a histogram, its prefix sum and a
// scatter order the buckets, and each pair's place inside its bucket (about
// one pair per bucket) is the number of smaller pairs there.
__device__ __forceinline__ uint32_t sort_bucket(uint64_t d2, float scale, uint32_t n) {
    return min((uint32_t)((float)d2 * scale), n - 1u);
}

__device__ void bucket_sort_store(const uint64_t* td, const uint32_t* ti, uint64_t* sd, uint32_t* si, uint32_t* hist,
                                  uint32_t n, uint64_t r2, uint32_t* dst_ids, int64_t* dst_d2) {
    const uint32_t lane = lane_id();
    if (n == 0) return;
    const float scale = r2 > 0 ? (float)n / (float)r2 : 0.0f;
    for (uint32_t t = lane; t < n; t += 64) hist[t] = 0u;
    wave_sync();
    uint32_t slot[4];  // n <= 256 = 4 pairs per lane
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t t = lane + 64u * k;
        if (t < n) slot[k] = atomicAdd(&hist[sort_bucket(td[t], scale, n)], 1u);
    }
    wave_sync();
    // exclusive prefix over the buckets, each lane owning a run of them
    const uint32_t per = (n + 63u) >> 6;
    const uint32_t b0 = lane * per;
    uint32_t sum = 0;
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < n) sum += hist[b0 + k];
    uint32_t run = scan_add(sum) - sum;
    wave_sync();
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < n) {
            const uint32_t c = hist[b0 + k];
            hist[b0 + k] = run;
            run += c;
        }
    wave_sync();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t t = lane + 64u * k;
        if (t < n) {
            const uint32_t dst = hist[sort_bucket(td[t], scale, n)] + slot[k];
            sd[dst] = td[t];
            si[dst] = ti[t];
        }
    }
    wave_sync();
    for (uint32_t t = lane; t < n; t += 64) {
        const uint64_t d = sd[t];
        const uint32_t id = si[t];
        const uint32_t b = sort_bucket(d, scale, n);
        const uint32_t lo = hist[b], hi = b + 1 < n ? hist[b + 1] : n;
        uint32_t rank = lo;
        for (uint32_t j = lo; j < hi; ++j) rank += key_less(sd[j], si[j], d, id) ? 1u : 0u;
        dst_ids[rank] = id;
        if (dst_d2) dst_d2[rank] = (int64_t)d;
    }
}

// ---------------------------------------------------------------------------
// Top-M searches in registers

// First bound of a top-M search: the radius expected to hold `target`
// objects (K-NN rows: the density around the centre, the home cell's count
// with the lattice mean as a floor; radius rows of `rowlen`: the row's own
// mean density over its ball), never above the cap; the whole cap for the
// bounding cube and the cell list, which are scanned whole anyway.  A search
// grows it and starts again whenever fewer than M lie within it.
__device__ __forceinline__ uint64_t first_bound(const LatArgs& L, const Query& s, uint32_t target, uint32_t rowlen) {
    if (!(s.flags & F_SPHERE)) return s.r2;
    const float e = (float)(1u << L.F);
    float rho;
    if (s.flags & F_KBOUND) return min(s.r2, sq(s.kbr));
    if (s.flags & F_KNN) {
        const uint32_t home = pack_cell(L, s.c[0], s.c[1], s.c[2]);
        const float dens = fmaxf((float)L.n / (float)(L.ncells ? L.ncells : 1u), (float)(L.cs[home + 1] - L.cs[home]));
        rho = 1.25f * e * cbrtf(0.2387f * (float)target / fmaxf(dens, 1e-6f));
    } else {
        rho = 1.1f * (float)s.r * cbrtf((float)target / (float)rowlen);
    }
    return rho >= (float)s.r ? s.r2 : min(s.r2, (uint64_t)((double)rho * (double)rho));
}

// The M <= 64 nearest pairs (dist^2, id) of query s above the pair (ld, li)
// when has_lower, within the cap: lane i ends with the i-th in (rd, ri), and
// the count found, min(M, pairs within the cap), is returned.  The bound
// starts at B, shrinks to the M-th distance once M are held (Section II.A,
// K nearest) and, when fewer than M lie within it, grows by half and the
// walk starts again.  A few new pairs are inserted one by one (place = pairs
// ahead of it, the rest move up one lane); a large batch is sorted and
// merged (the 64 smallest of list and batch, as a bitonic sequence, then
// sorted).
template <int METHOD, bool TLDS>
__device__ __forceinline__ uint32_t topm_registers(const LatArgs& L, const TabArgs& T, const uint32_t* tab_lds,
                                                   const Query& s, const AxisWrap& aw, uint32_t* own, uint32_t M,
                                                   uint64_t B, bool has_lower, uint64_t ld, uint32_t li, uint64_t& rd,
                                                   uint32_t& ri, uint32_t* stat = nullptr) {
    const uint32_t lane = lane_id();
    rd = kMaxD2;
    ri = kMaxId;
    uint64_t kd = kMaxD2;
    uint32_t kid = kMaxId, held = 0, cand2 = 0, walked2 = 0, kept2 = 0;
    auto visit_r = [&](bool act, uint32_t p, const uint4& P) -> bool {
        const uint64_t d2 = obj_dist2(aw, s, P);
        const uint32_t id = P.w;
        bool cv = act && d2 <= B && p != s.self;
        if (cv && has_lower) cv = key_less(ld, li, d2, id);
        if (cv && held >= M) cv = key_less(d2, id, kd, kid);
        uint64_t qm = __ballot(cv);
        if (qm == 0) return false;
        const uint32_t nb = (uint32_t)__popcll(qm);
        if (nb > 6) {
            uint64_t cd = cv ? d2 : kMaxD2;
            uint32_t ci = cv ? id : kMaxId;
            wave_sort64(cd, ci);
            const uint64_t xd = shfl64(cd, 63u - lane);
            const uint32_t xi = __shfl(ci, 63u - lane);
            if (key_less(xd, xi, rd, ri)) {
                rd = xd;
                ri = xi;
            }
            wave_bitonic_clean64(rd, ri);
            held = min(held + nb, 64u);
        } else {
            while (qm) {
                const uint32_t j = (uint32_t)__builtin_ctzll(qm);
                qm &= qm - 1ull;
                const uint64_t nd = lane_val64(d2, j);
                const uint32_t ni = lane_val(id, j);
                if (held >= M && !key_less(nd, ni, kd, kid)) continue;
                const uint32_t pos = (uint32_t)__popcll(__ballot(key_less(rd, ri, nd, ni)));
                const uint32_t below = lane ? lane - 1u : 0u;
                const uint64_t sd = shfl64(rd, below);
                const uint32_t si = __shfl(ri, below);
                if (lane > pos) {
                    rd = sd;
                    ri = si;
                } else if (lane == pos) {
                    rd = nd;
                    ri = ni;
                }
                held = min(held + 1u, 64u);
                if (held >= M) {
                    kd = lane_val64(rd, M - 1u);
                    kid = lane_val(ri, M - 1u);
                }
            }
        }
        if (held >= M) {
            kd = lane_val64(rd, M - 1u);
            kid = lane_val(ri, M - 1u);
        }
        return false;
    };
    for (;;) {
        walk<METHOD, TLDS, true>(L, T, tab_lds, s, false, walked2, [&]() { return held >= M ? kd : B; },
                                 [&](const RowRef& r) -> bool {
            kept2 += r.kept;
            return for_candidates(L, r.st0, r.cnt0, r.st1, r.cnt1, own, cand2, visit_r);
        });
        if (held >= M || B >= s.r2) break;
        B = min(s.r2, B + B + (B >> 2) + 1u);  // radius x1.5
        held = 0;
        rd = kMaxD2;
        ri = kMaxId;
        kd = kMaxD2;
        kid = kMaxId;
    }
    if (stat) {
        // per-query statistics, every walk of the search included
        const uint32_t k2 = wave_sum(kept2);
        if (lane == 0) {
            stat[0] += walked2;
            stat[1] += k2;
            stat[2] += cand2;
        }
    }
    return min(held, M);
}

// ---------------------------------------------------------------------------
// Pass 0: row sizes

// Queue sets of the work counters.
constexpr int kQCount = 0, kQWrite = 1, kQTopm = 2, kQFbCount = 3, kQFbWrite = 4, kQWalk = 5, kQExtra = 6;
// the count pass's last list (rows the second grouped round left) takes the
// fallback write set, which only the write pass uses and clears
constexpr int kQExtra2 = kQFbWrite;
// Longest radius row the block-per-row kernel orders in LDS (28 bytes per pair).
constexpr uint32_t kLongCap = 3072;

__device__ __forceinline__ uint32_t* queue_set(const QArgs& A, int set) {
    return A.queues + (size_t)set * SPHIDX_NQUEUE * SPHIDX_QSTRIDE;
}

// Rows of at most 64 pairs whose key fits one 64-bit word: with id < 2^idbits
// and dist^2 < 2^(64 - idbits), (dist^2 << idbits) | id orders exactly as
// (dist^2, id) and is unique, so a pair's place is the number of smaller
// keys.  One pair per lane; the keys are read back as LDS broadcasts.
__device__ void sort_small_store(const uint64_t* td, const uint32_t* ti, uint64_t* ck, uint32_t n, uint32_t idbits,
                                 uint32_t* dst_ids, int64_t* dst_d2) {
    const uint32_t lane = lane_id();
    uint64_t d = 0, k = ~0ull;
    uint32_t id = 0;
    if (lane < n) {
        d = td[lane];
        id = ti[lane];
        k = (d << idbits) | id;
    }
    ck[lane] = k;  // lanes past n: the largest key, padding for the paired reads
    wave_sync();
    uint32_t rank = 0;
    for (uint32_t j = 0; j < n; j += 2) {
        const ulonglong2 p = *(const ulonglong2*)(ck + j);
        rank += (p.x < k ? 1u : 0u) + (p.y < k ? 1u : 0u);
    }
    if (lane < n) {
        dst_ids[rank] = id;
        if (dst_d2) dst_d2[rank] = (int64_t)d;
    }
    wave_sync();
}

// Order the n <= cap pairs of one row by (dist^2, id) and store them at dst.
__device__ __forceinline__ void sort_row_store(const uint64_t* td, const uint32_t* ti, uint64_t* sd, uint32_t* si,
                                               uint32_t* hist, uint32_t n, uint64_t r2, uint32_t idbits,
                                               uint32_t* dst_ids, int64_t* dst_d2) {
    const uint32_t r2bits = r2 ? 64u - (uint32_t)__builtin_clzll(r2) : 0u;
    if (n <= 64 && r2bits + idbits <= 64)
        sort_small_store(td, ti, sd, n, idbits, dst_ids, dst_d2);
    else
        bucket_sort_store(td, ti, sd, si, hist, n, r2, dst_ids, dst_d2);
}

// FROM_LIST: a query list (the sphere method's fallback queries, scanned with
// the bounding cube).  STASH: radius rows of at most sort_cap hits are also
// collected, sorted and kept in the workspace's stash, so that the write pass
// only copies them into place; other rows go to the walk list.  KSTASH (with
// STASH): K-NN rows of K <= 64 are searched here, top-K in registers, and
// kept the same way, so that no later pass walks them again.
template <int METHOD, bool TLDS, bool FROM_LIST, bool STASH, bool KSTASH>
__global__ __launch_bounds__(256) void count_kernel(LatArgs L, TabArgs T, QArgs A) {
    extern __shared__ __align__(16) char smem[];
    const uint32_t* tab_lds = stage_table<TLDS>(T, smem);
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t cap = A.sort_cap;
    char* wb = smem + table_lds_bytes<TLDS>(T) + (size_t)wave * (STASH ? (size_t)cap * 28 + 256 : 256);
    uint64_t* td = (uint64_t*)wb;
    uint64_t* sd = td + cap;
    uint32_t* ti = (uint32_t*)(sd + cap);
    uint32_t* si = ti + cap;
    uint32_t* hist = si + cap;
    uint32_t* own = STASH ? hist + cap : (uint32_t*)wb;
    const AxisWrap aw = axis_wrap(L);
    const uint32_t lane = lane_id();
    const uint32_t nq = FROM_LIST ? uni(*A.list_count) : A.Q;
    // this wave's stash chunk [cur, lim) in its region; `dry` once the
    // region is used up
    const uint32_t region = blockIdx.x % SPHIDX_NREGION;
    uint32_t cur = 0, lim = 0;
    bool dry = false;
    const uint32_t idbits = L.n > 1 ? 32u - (uint32_t)__builtin_clz(L.n - 1u) : 0u;  // ids are below n
    // room for n more stash elements in this wave's chunk, grabbing a new
    // chunk of the region when needed; false once the region is used up
    auto stash_room = [&](uint32_t n) -> bool {
        if (cur + n <= lim) return true;
        if (dry) return false;
        const uint32_t grab = max(A.stash_chunk, n);
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(A.stash_ctr + region * SPHIDX_QSTRIDE, grab);
        t = uni(t);
        if ((uint64_t)t + grab <= A.stash_region) {
            cur = region * A.stash_region + t;
            lim = cur + grab;
            return true;
        }
        dry = true;
        return false;
    };
    for_each_query(nq, A, queue_set(A, FROM_LIST ? (int)A.list_set : kQCount), [&](uint32_t ti_) {
        const uint32_t qi = FROM_LIST ? uni(A.list[ti_]) : ti_;
        const Query s = load_query(L, A, qi);
        if ((METHOD == kSphere || METHOD == kPaper) && (s.flags & F_VALID) && !(s.flags & F_SPHERE))
            return;  // fallback list
        if (!FROM_LIST && (s.flags & F_LONG)) return;  // counted one block per row
        const bool knn = s.flags & F_KNN;
        if (KSTASH && knn && (s.flags & F_VALID) && s.k <= 64u) {
            // the row itself: lane i ends with the i-th nearest
            uint64_t rd;
            uint32_t ri;
            uint32_t* stp = A.stats ? A.stats + 4 * (size_t)s.row : nullptr;
            const uint32_t got = topm_registers<METHOD, TLDS>(L, T, tab_lds, s, aw, own, s.k,
                                                               first_bound(L, s, s.k, 0u), false, 0ull, 0u, rd, ri,
                                                               stp);
            if (stp) {
                const uint32_t nc = cube_cells(L, s);
                if (lane == 0) stp[3] = nc;
            }
            if (lane == 0) A.row_ptr[s.row] = (int64_t)got;
            uint32_t off = 0u;  // empty rows: nothing to copy
            if (got > 0) {
                if (stash_room(got)) {
                    if (lane < got) {
                        A.stash_ids[cur + lane] = ri;
                        if (A.stash_d2) A.stash_d2[cur + lane] = (int64_t)rd;
                    }
                    off = cur;
                    cur += got;
                } else {
                    off = kMaxId;
                    if (lane == 0) A.walkq[atomicAdd(A.walk_count, 1u)] = qi;
                }
            }
            if (lane == 0) A.soff[s.row] = off;
            return;
        }
        uint32_t hits = 0, inner = 0, kept = 0, cand = 0, walked = 0;
        uint64_t dmax = 0;  // K-NN: the largest dist^2 among the hits so far
        bool self_inner = false;
        auto visit = [&](bool act, uint32_t p, const uint4& P) -> bool {
            const uint64_t d2 = obj_dist2(aw, s, P);
            const bool hit = act && d2 <= s.r2 && p != s.self;
            if (knn && hit) dmax = max(dmax, d2);
            const uint64_t hm = __ballot(hit);
            if (STASH && hit) {
                const uint32_t slot = hits + lanes_below(hm);
                if (slot < cap) {
                    td[slot] = d2;
                    ti[slot] = P.w;
                }
            }
            hits += (uint32_t)__popcll(hm);
            return knn && hits >= s.k;
        };
        auto on_row = [&](const RowRef& r) -> bool {
            kept += r.kept;
            // cells wholly inside: counted without reading objects; note when
            // the excluded own object was among them
            if (r.icnt && s.self - r.ist < r.icnt) self_inner = true;
            inner += r.icnt;
            return for_candidates(L, r.st0, r.cnt0, r.st1, r.cnt1, own, cand, visit);
        };
        if (s.flags & F_VALID) {
            walk<METHOD, TLDS, false>(L, T, tab_lds, s, !STASH && !knn && A.interior, walked,
                                      [&]() { return s.r2; }, on_row);
            uint32_t total = hits + wave_sum(inner);
            if (__ballot(self_inner) != 0) total -= 1;
            if (knn && (s.flags & F_SPHERE) && total >= s.k) {
                // the walk found K objects within the largest of their
                // distances: that radius (rounded up) bounds the K-th
                // distance, and the write pass's top-K starts from it
                const uint32_t rb = (uint32_t)min((double)s.r, ceil(sqrt((double)dmax)) + 1.0);
                const uint32_t rbm = lane_val(scan_max(rb), 63);
                if (lane == 0) {
                    uint32_t* dw = (uint32_t*)(A.desc + 4 * (size_t)qi);
                    dw[12] = rbm;
                    dw[6] = s.flags | F_KBOUND;
                }
            }
            if (knn && total > s.k) total = s.k;
            hits = total;
        }
        if (lane == 0) A.row_ptr[s.row] = (int64_t)hits;
        if (STASH) {
            uint32_t off = 0u;  // empty rows: nothing to copy
            if ((s.flags & F_VALID) && hits > 0) {
                const bool ok = !knn && hits <= cap && stash_room(hits);
                if (ok) {
                    wave_sync();
                    sort_row_store(td, ti, sd, si, hist, hits, s.r2, idbits, A.stash_ids + cur,
                                   A.stash_d2 ? A.stash_d2 + cur : nullptr);
                    wave_sync();
                    off = cur;
                    cur += hits;
                } else {
                    off = kMaxId;
                    if (lane == 0) A.walkq[atomicAdd(A.walk_count, 1u)] = qi;
                }
            }
            if (lane == 0) A.soff[s.row] = off;
        }
        if (A.stats) {
            const uint32_t kept_all = wave_sum(kept);
            const uint32_t ncube = (s.flags & F_VALID) ? cube_cells(L, s) : 0u;
            if (lane == 0) {
                // (added to: a grouped count may have walked the query first)
                uint32_t* stp = A.stats + 4 * (size_t)s.row;
                stp[0] += walked;
                stp[1] += kept_all;
                stp[2] += cand;
                stp[3] = ncube;
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Pass 0, radius queries in groups: a wavefront takes kGroup consecutive
// queries and spreads all their table rows over its lanes, 64 rows per
// step, and all their candidate objects, 64 per step, so that short rows
// and small radii fill whole steps.  Hits of the group are collected as
// one 64-bit key (query slot, dist^2, id) each, and one bucket sort orders
// the group's rows together; with the stash they are kept in one chunk.
// K-NN queries (the KNN variant) take part as radius rows at their first
// search radius and keep the first K.  Queries it does not take (K-NN of
// large K or off the sphere tables, keys that would not fit 64 bits, rows
// short of K inside the first radius) go to the extra list for the
// one-query-per-wave kernel.  The list-driven K-NN variant is the second
// round over that list: a K-NN row short of K inside its first radius is
// searched again in groups at the larger radius the first round wrote into
// its descriptor from the count it saw (the cap at most); what that round
// does not take goes on to the one-query-per-wave kernel.

constexpr uint32_t kGroup = 8, kGroupBits = 3;
// hit buffer keys and rows per group, in eighths of sort_cap
constexpr uint32_t kHitEighths = 8, kRowEighths = 6;
constexpr uint32_t kMaxHitCap = 256 * kHitEighths / 8;
// The group's hit buffer holds sort_cap keys, and a group ends before its
// rows would exceed 3/4 of sort_cap.  When the hits overflow the buffer the
// group keeps its leading queries whose hits fit (hits arrive query by
// query), and the next group starts at the first query left out and walks
// it again; the wave's row budget shrinks to what fitted and grows back by
// an eighth per group that fits, so that dense regions do not repeat the
// waste.  Only a query whose own hits exceed the buffer is left to the
// write pass.  A smaller buffer buys occupancy (LDS) at the price of more
// overflows.  On the uneven-radius workload (1 M queries, ms per step):
// 2 x sort_cap keys, an overflowing group left whole to the write pass,
// 1.154; 1.5 x 1.092, 1.25 x 1.062; keeping the leading queries, 1.25 x
// 1.028, 1 x 1.006 (0.988 within 80 VGPRs), 7/8 x 1.039; rows up to 7/8 of
// sort_cap at 1 x, 1.004.

// Per-wave LDS of the grouped kernel: slot data (kGroup x 80 B), 32 words of
// per-slot counters, the 64-word owner map, then (stash) the hit keys in
// arrival order, the same by bucket, and the bucket counts, or (no stash)
// sort_cap 16-byte row records.
__host__ __device__ constexpr uint32_t group_hitcap(uint32_t cap) { return cap * kHitEighths / 8; }
__host__ __device__ constexpr uint32_t group_rows(uint32_t cap) { return cap * kRowEighths / 8; }
// rows per chunk of the walk (at most 256): their 16-byte records
// fill the bucket buffer and the bucket counts, both free until the sort
__host__ __device__ constexpr uint32_t group_chunk(uint32_t cap) {
    return group_hitcap(cap) * 12 / 16 < 256u ? group_hitcap(cap) * 12 / 16 : 256u;
}
// 64-row layers of the largest chunk (sort_cap 256)
constexpr uint32_t kLayers = (group_chunk(256) + 63) / 64;
static_assert(kLayers * 64 + 1 <= 255, "candidate-step owner marks hold a chunk row + 1 in one byte");
__host__ __device__ constexpr size_t group_lds_per_wave(bool stash, uint32_t cap) {
    return 640 + 128 + 256 + (stash ? (size_t)group_hitcap(cap) * 20 : (size_t)group_chunk(cap) * 16);
}

// dist^2 field of a group hit key (slot | dist^2 | id)
__device__ __forceinline__ uint64_t key_d2(uint64_t k, uint32_t idbits, uint32_t d2bits) {
    return (k >> idbits) & ((1ull << d2bits) - 1ull);
}

// At most 80 VGPRs, so that six waves share each SIMD (the LDS of a
// sort_cap 256 hit buffer allows as many).
// KNN: K-NN queries of the batch are searched in the groups too (a radius
// batch takes the variant without that code).
template <int METHOD, bool TLDS, bool STASH, bool FROM_LIST, bool KNN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void group_count_kernel(LatArgs L,
                                                                                                 TabArgs T,
                                                                                                 QArgs A) {
    extern __shared__ __align__(16) char smem[];
    const uint32_t* tab_lds = stage_table<TLDS>(T, smem);
    const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
    const uint32_t hitcap = group_hitcap(A.sort_cap), grows = group_rows(A.sort_cap);  // hitcap <= kMaxHitCap
    uint32_t rlim = grows;  // rows per group (shrinks where hits overflow the buffer)
    char* wb = smem + table_lds_bytes<TLDS>(T) + (size_t)wave * group_lds_per_wave(STASH, A.sort_cap);
    uint4* qp = (uint4*)wb;                    // five records of kGroup slots each (slot s of record k
                                               // at qp[k * kGroup + s]): centre + table start, r^2 + self + rows,
                                               // cube extent, flags + row, W/2 - centre + self
    uint32_t* cnt = (uint32_t*)(wb + 640);     // [0, 8) hits, [8, 16) row start, [16, 24) hits,
    uint32_t* qst = cnt + 8;                   // [24, 32) bucket scale (float)
    uint32_t* qn = cnt + 16;
    float* qsc = (float*)(cnt + 24);
    uint32_t* own = cnt + 32;                  // 64: owner map
    uint64_t* hb = (uint64_t*)(own + 64);      // hitcap keys in arrival order
    uint64_t* hs = hb + hitcap;                // hitcap keys by bucket
    uint32_t* hh = (uint32_t*)(hs + hitcap);   // hitcap bucket counts, then starts
    // sort_cap row records of the chunk being walked (in the stash case the
    // bucket buffer, free until the sort)
    uint4* rinfo = STASH ? (uint4*)hs : (uint4*)(own + 64);
    const AxisWrap aw = axis_wrap(L);
    const uint32_t idbits = L.n > 1 ? 32u - (uint32_t)__builtin_clz(L.n - 1u) : 0u;
    const uint32_t d2bits = 64u - kGroupBits - idbits;
    const uint64_t idmask = idbits ? (~0ull >> (64u - idbits)) : 0ull;
    const uint32_t region = blockIdx.x % SPHIDX_NREGION;
    uint32_t cur = 0, lim = 0;
    bool dry = false;
    const uint32_t nq = FROM_LIST ? uni(*A.list_count) : A.Q;
    for_each_range(nq, A, queue_set(A, FROM_LIST ? (int)A.list_set : kQCount), [&](uint32_t b, uint32_t e) {
        for (uint32_t g0 = b, ng = 0; g0 < e; g0 += ng) {
            const uint32_t cand = min(kGroup, e - g0);
            // ---- slots: lane l < cand looks at query g0 + l (of the list);
            // the group keeps the leading slots whose rows fit rlim (at
            // least one)
            const uint32_t qi = FROM_LIST ? (lane < cand ? A.list[g0 + lane] : 0u) : g0 + lane;
            uint32_t rows = 0, row = 0;
            bool mine = false, extra = false, invalid = false, knn = false;
            uint4 d0 = make_uint4(0, 0, 0, 0), d1 = d0, d2 = d0, d3 = d0;
            if (lane < cand) {
                d0 = A.desc[4 * (size_t)qi];
                d1 = A.desc[4 * (size_t)qi + 1];
                d2 = A.desc[4 * (size_t)qi + 2];
                d3 = A.desc[4 * (size_t)qi + 3];
                row = d0.w;
                const uint32_t flags = d1.z;
                const uint64_t r2 = (uint64_t)d1.x * d1.x;
                const uint32_t r2bits = r2 ? 64u - (uint32_t)__builtin_clzll(r2) : 0u;
                const bool valid = flags & F_VALID, sph = flags & F_SPHERE;
                if (!valid) {
                    invalid = true;
                } else if (KNN && FROM_LIST && !((flags & F_KNN) && sph)) {
                    // the second round takes sphere-table K-NN rows only;
                    // everything else on its list goes on
                    extra = true;
                } else if (METHOD == kSphere && !sph) {
                    // counted by the fallback list's kernel
                } else if (KNN && (flags & F_KNN)) {
                    // K-NN (sphere tables, K up to half the buffer):
                    // a radius row at the first search radius d2.y, the
                    // table prefix d2.z; its first K are the K nearest when
                    // it holds K (Section II.A: beyond the radius every
                    // object is farther)
                    const uint64_t b2 = (uint64_t)d2.y * d2.y;
                    const uint32_t b2bits = b2 ? 64u - (uint32_t)__builtin_clzll(b2) : 0u;
                    if (!sph || (flags & F_LIST) || b2bits > d2bits || 2u * d1.y > hitcap) {
                        extra = true;
                    } else {
                        mine = true;
                        knn = true;
                        rows = d2.z + ((flags & F_OUTSIDE) ? 1u : 0u);
                    }
                } else if (flags & F_LONG) {
                    // counted one block per row
                } else if ((flags & (F_KNN | F_LIST)) || r2bits > d2bits) {
                    extra = true;
                } else {
                    mine = true;
                    rows = (sph ? d2.x : d2.w * d3.w) + ((flags & F_OUTSIDE) ? 1u : 0u);
                }
            }
            {
                const uint32_t pre_incl = scan_add(rows);
                const uint64_t fits = __ballot(lane < cand && pre_incl <= rlim);
                ng = max(1u, (uint32_t)__popcll(fits));
            }
            if (lane >= ng) {
                rows = 0;
                mine = extra = invalid = knn = false;
            }
            if (mine) {
                const uint64_t r2 = (KNN && knn) ? (uint64_t)d2.y * d2.y : (uint64_t)d1.x * d1.x;
                const uint32_t self = (A.qx == nullptr && (A.flags & SPHIDX_EXCLUDE_SELF)) ? qi : kMaxId;
                uint4* p = qp + lane;
                p[0] = make_uint4(d0.x, d0.y, d0.z, d1.w);
                p[kGroup] = make_uint4((uint32_t)r2, (uint32_t)(r2 >> 32), self, rows);
                // (a K-NN slot walks no cube: K and whether its search radius
                // covers the cap take the cube fields)
                p[2 * kGroup] = make_uint4(d3.x, d3.y, d3.z, (KNN && knn) ? d1.y : d2.z);
                p[3 * kGroup] = make_uint4(d2.w, (KNN && knn) ? (d2.y >= d1.x ? 1u : 0u) : d3.w, d1.z, row);
                // the candidate test's form of the centre: the minimum-image
                // offset is ((p + (W/2 - c)) mod W) - W/2
                p[4 * kGroup] = make_uint4(aw.half[0] - d0.x, aw.half[1] - d0.y, aw.half[2] - d0.z, self);
            }
            if (lane < kGroup) cnt[lane] = 0u;
            wave_sync();
            const uint32_t incl = scan_add(rows);
            const uint32_t R = lane_val(incl, 63);
            const uint32_t excl = incl - rows;
            uint32_t hcount = 0;
            // The group's rows go in chunks of sort_cap (at most kLayers x 64)
            // rows: first every row of the chunk, 64 per layer, one per lane,
            // gives its object ranges, numbered by a prefix over the chunk and
            // kept in LDS; then the chunk's candidates, 64 per step, in one
            // stream, with the next step's records loaded while this step's
            // are tested.
            const uint32_t CH = group_chunk(A.sort_cap);  // <= kLayers x 64
            for (uint32_t rb = 0; rb < R; rb += CH) {
                const uint32_t clen = min(CH, R - rb);
                uint32_t cex[kLayers], cin[kLayers];
#pragma unroll
                for (uint32_t k = 0; k < kLayers; ++k) cex[k] = cin[k] = 0u;
                uint32_t carry = 0;
                for (uint32_t k = 0; k * 64u < clen; ++k) {
                    // ---- this lane's row: owner slot and entry
                    const uint32_t base = rb + k * 64u;
                    own[lane] = 0;
                    wave_sync();
                    if (rows > 0 && excl < base + 64 && incl > base) own[excl > base ? excl - base : 0] = lane + 1;
                    wave_sync();
                    const bool act = k * 64u + lane < clen;
                    const uint32_t fr = base + lane;
                    const uint32_t gmax = scan_max(own[lane]);
                    const uint32_t gs = act ? gmax - 1u : 0u;
                    const uint32_t ent = fr - bperm(excl, gs);
                    const uint4* p = qp + gs;
                    const uint4 pa = p[0], pb = p[kGroup], pc = p[2 * kGroup], pd = p[3 * kGroup];
                    Query sq;
                    sq.q[0] = pa.x;
                    sq.q[1] = pa.y;
                    sq.q[2] = pa.z;
                    sq.tb = pa.w;
                    sq.r2 = (uint64_t)pb.x | ((uint64_t)pb.y << 32);
                    sq.self = pb.z;
                    sq.lo[0] = (int32_t)pc.x;
                    sq.lo[1] = (int32_t)pc.y;
                    sq.lo[2] = (int32_t)pc.z;
                    sq.nn[0] = pc.w;
                    sq.nn[1] = pd.x;
                    sq.nn[2] = pd.y;
                    sq.flags = pd.z;
                    const uint32_t e1 = 1u << L.F;
                    for (int a = 0; a < 3; ++a) {
                        sq.c[a] = sq.q[a] >> L.F;
                        sq.f[a] = sq.q[a] & (e1 - 1u);
                        sq.up[a] = e1 - sq.f[a];
                        sq.dn[a] = sq.f[a] + 1u;
                    }
                    const bool is_out = act && (sq.flags & F_OUTSIDE) && ent + 1u == pb.w;
                    const bool sph = METHOD == kSphere || (METHOD == kEither && (sq.flags & F_SPHERE));
                    const bool live = act && !is_out;
                    RowRef r;
                    if (sph) {
                        const uint32_t w =
                            live ? row_word<TLDS>(T, tab_lds, sq.tb, TLDS ? row_class(L, T, sq.f) : 0u, ent) : 0u;
                        r = sphere_row(L, sq, w, live, sq.r2, false);
                    } else {
                        const double inv_ny = sq.nn[1] ? 1.0 / (double)sq.nn[1] : 0.0;
                        r = cube_row(L, sq, live ? ent : 0u, live, inv_ny);
                    }
                    if (is_out) {
                        // every object outside the region lives in one cell (Section II.B)
                        r.st0 = L.cs[L.ncells];
                        r.cnt0 = L.cs[L.ncells + 1] - r.st0;
                        r.cnt1 = 0u;
                    }
                    if (A.stats && live) {
                        // per-query statistics, the outside cell's pseudo-row
                        // left out (rows walked again are counted again)
                        uint32_t* stp = A.stats + 4 * (size_t)pd.w;
                        atomicAdd(stp, 1u);
                        atomicAdd(stp + 1, r.kept);
                    }
                    const uint32_t tl = act ? r.cnt0 + r.cnt1 : 0u;
                    const uint32_t ci = scan_add(tl);
                    const uint32_t ce = carry + ci - tl;
                    // per row: position bases of its two ranges, the slot
                    // where the second starts, and the query slot
                    if (act) rinfo[k * 64u + lane] = make_uint4(r.st0 - ce, ce + r.cnt0, r.st1 - (ce + r.cnt0), gs);
#pragma unroll
                    for (uint32_t j = 0; j < kLayers; ++j) {
                        cex[j] = j == k ? ce : cex[j];
                        cin[j] = j == k ? ce + tl : cin[j];
                    }
                    carry += lane_val(ci, 63);
                }
                const uint32_t CT = carry;
                // ---- owner row of each of the 64 slots from cb: a row marks
                // where its range starts in the step (a row begun earlier
                // marks slot 0), and a max-scan hands every slot to its row
                // The marks cover a window of four steps (256 slots, one
                // byte each in the owner map's words): rows are marked once
                // per window, and each step max-scans its 64 bytes on top of
                // the owner the window's earlier steps ended with.  Steps are
                // located in order, each once.
                uint8_t* own8 = (uint8_t*)own;
                uint32_t wcarry = 0;
                auto locate = [&](uint32_t cb, uint32_t& pos, uint32_t& sl) -> bool {
                    const uint32_t wb = cb & ~255u, wo = cb - wb;
                    if (wo == 0) {
                        wave_sync();
                        own[lane] = 0;
                        wave_sync();
#pragma unroll
                        for (uint32_t k = 0; k < kLayers; ++k)
                            if (cin[k] > cex[k] && cex[k] < wb + 256u && cin[k] > wb)
                                own8[cex[k] > wb ? cex[k] - wb : 0] = (uint8_t)(k * 64u + lane + 1u);
                        wave_sync();
                        wcarry = 0;
                    }
                    const uint32_t m = max(scan_max((uint32_t)own8[wo + lane]), wcarry);
                    wcarry = lane_val(m, 63);
                    // (a step past the end marks nothing: row 0 stands in)
                    const uint32_t o = max(m, 1u) - 1u;
                    const uint4 ri = rinfo[o];
                    const uint32_t g = cb + lane;
                    pos = (g < ri.y ? ri.x : ri.z) + g;
                    sl = ri.w;
                    return g < CT;
                };
                auto test = [&](const uint4& P, uint32_t pos, uint32_t sl, bool cact, uint32_t cb) {
                    const uint4 ch = qp[4 * kGroup + sl];
                    const uint2 cr = *(const uint2*)(qp + kGroup + sl);
                    const uint32_t pv[3] = {P.x, P.y, P.z}, hv[3] = {ch.x, ch.y, ch.z};
                    uint64_t d2 = 0;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const int32_t dd = (int32_t)((pv[a] + hv[a]) & aw.mask[a]) - (int32_t)aw.half[a];
                        d2 += (uint64_t)((int64_t)dd * dd);
                    }
                    const uint64_t r2 = (uint64_t)cr.x | ((uint64_t)cr.y << 32);
                    const bool hit = cact && d2 <= r2 && pos != ch.w;
                    if (A.stats && cact) atomicAdd(A.stats + 4 * (size_t)qp[3 * kGroup + sl].w + 2, 1u);
                    const uint64_t H = __ballot(hit);
                    const uint32_t hp = hcount + lanes_below(H);
                    // hits per slot: a slot's candidates take contiguous lanes
                    // and its hits arrive in order, so the last lane of its
                    // run in a step records the group's hit count so far
                    const uint32_t nsl = bperm(sl, (lane + 1u) & 63u);
                    if (cact && (lane == 63u || cb + lane + 1u >= CT || nsl != sl)) cnt[sl] = hp + (hit ? 1u : 0u);
                    if (STASH && hit && hp < hitcap)
                        hb[hp] = ((uint64_t)sl << (64u - kGroupBits)) | (d2 << idbits) | (uint64_t)P.w;
                    hcount += (uint32_t)__popcll(H);
                };
                if (CT > 0) {
                    // two register sets taken in turn: the step after the one
                    // under test is already loading.  Lanes past the end load
                    // record 0 (present whenever a candidate is) and test
                    // nothing.
                    uint32_t pa = 0, sa = 0, pb = 0, sb = 0;
                    bool aa = locate(0, pa, sa), ab = false;
                    uint4 PA = L.pts[aa ? pa : 0u], PB = PA;
                    // (the step past the end, located once per chunk, has no
                    // active lane)
                    for (uint32_t cb = 0; cb < CT; cb += 128) {
                        ab = locate(cb + 64, pb, sb);
                        PB = L.pts[ab ? pb : 0u];
                        test(PA, pa, sa, aa, cb);
                        if (cb + 64 >= CT) break;
                        aa = locate(cb + 128, pa, sa);
                        PA = L.pts[aa ? pa : 0u];
                        test(PB, pb, sb, ab, cb + 64);
                    }
                }
                wave_sync();
            }
            // ---- row sizes: each slot's hits end where its last run left
            // the count (a slot without candidates left none: the max-scan
            // carries the previous slot's end)
            const uint32_t hend = scan_max(lane < kGroup ? cnt[lane] : 0u);
            const uint32_t hbeg = bperm(hend, (lane + 63u) & 63u);
            uint32_t nq = mine ? hend - (lane ? hbeg : 0u) : 0u;
            uint32_t total = hcount;
            if (STASH && hcount > hitcap && ng > 1) {
                // the hit buffer overflowed: keep the leading slots whose hits
                // fit (hits arrive slot by slot, so theirs are the buffer's
                // first keys); the next group starts at the first slot left
                // out and walks it again
                const uint32_t hi = scan_add(nq);
                ng = max(1u, (uint32_t)__popcll(__ballot(lane < ng && hi <= hitcap)));
                if (lane >= ng) {
                    mine = extra = invalid = knn = false;
                    nq = 0u;
                }
                total = lane_val(hi, ng - 1u);
                // later groups of this wave take no more rows than fitted
                // here, and grow back by an eighth per group that fits
                rlim = max(1u, lane_val(incl, ng - 1u));
            } else if (STASH) {
                rlim = min(grows, rlim + max(1u, grows / 8u));
            }
            // K-NN rows: the first K, or every object when the search radius
            // covers the cap; a row with fewer than K inside a smaller radius
            // is searched again by the one-query-per-wave kernel
            uint32_t nrow = nq;
            if (KNN && knn) {
                const uint32_t kk = qp[2 * kGroup + lane].w;
                if (nq >= kk) {
                    nrow = kk;
                } else if (qp[3 * kGroup + lane].y == 0u) {
                    mine = false;
                    extra = true;
                    if (!FROM_LIST) {
                        // for the second round: the radius expected to hold
                        // knn_target(K) at the density the first ball showed
                        // (grown by 1.15 to 2 times, the cap at most), and its
                        // table prefix from the radius index of the row class
                        const float sc =
                            fminf(2.0f, fmaxf(1.15f, cbrtf(knn_target((float)kk) / fmaxf((float)nq, 0.5f))));
                        const uint32_t kb = (uint32_t)min((uint64_t)d1.x, (uint64_t)((float)d2.y * sc) + 1u);
                        const uint32_t e1 = 1u << L.F, sh = L.F - T.s;
                        const uint32_t cls = ((d0.y & (e1 - 1u)) >> sh) | (((d0.z & (e1 - 1u)) >> sh) << T.s);
                        const uint32_t jb = (uint32_t)(((uint64_t)kb + (1u << T.rshift) - 1u) >> T.rshift);
                        A.desc[4 * (size_t)qi + 2] = make_uint4(d2.x, kb, T.rindex[(size_t)cls * T.nr + jb], d2.w);
                    }
                }
            }
            if (invalid) {
                A.row_ptr[row] = 0;
                if (STASH) A.soff[row] = 0u;
            }
            {
                // the queries left to the one-query-per-wave kernel
                const uint64_t xm = __ballot(extra);
                uint32_t xb = 0;
                if (xm != 0 && lane == 0) xb = atomicAdd(A.xq_count, (uint32_t)__popcll(xm));
                xb = uni(xb);
                if (extra) A.xq[xb + lanes_below(xm)] = qi;
            }
            if (mine) A.row_ptr[row] = (int64_t)nrow;
            if (STASH) {
                // pairs kept per slot: a K-NN row keeps its first K, so the
                // stash takes those only (K-NN variant); a radius row, all
                const uint32_t ko = KNN ? (mine ? nrow : 0u) : nq;
                const uint32_t kincl = scan_add(ko);
                const uint32_t qo0 = kincl - ko;
                const uint32_t tout = KNN ? lane_val(kincl, 63) : total;
                bool ok = total <= hitcap;
                if (ok && tout > 0 && cur + tout > lim) {
                    ok = false;
                    if (!dry) {
                        const uint32_t grab = max(A.stash_chunk, tout);
                        uint32_t t = 0;
                        if (lane == 0) t = atomicAdd(A.stash_ctr + region * SPHIDX_QSTRIDE, grab);
                        t = uni(t);
                        if ((uint64_t)t + grab <= A.stash_region) {
                            cur = region * A.stash_region + t;
                            lim = cur + grab;
                            ok = true;
                        } else {
                            dry = true;
                        }
                    }
                }
                const uint32_t qs0 = scan_add(nq) - nq;
                if (ok && tout > 0) {
                    // every hit's dist^2 is at most its slot's r^2: shifted
                    // right by gsh, the largest r^2 of the group fits 24 bits,
                    // so a bucket needs one 32-bit conversion
                    uint64_t r2 = 0;
                    if (lane < kGroup) {
                        const uint4 pb = qp[kGroup + lane];
                        r2 = nq > 0 ? (uint64_t)pb.x | ((uint64_t)pb.y << 32) : 0ull;
                    }
                    const uint32_t rbits = lane_val(scan_max(r2 ? 64u - (uint32_t)__builtin_clzll(r2) : 0u), 63);
                    const uint32_t gsh = rbits > 24u ? rbits - 24u : 0u;
                    const uint32_t dsh = idbits + gsh, dmask = (1u << (rbits - gsh)) - 1u;
                    if (lane < kGroup) {
                        qst[lane] = qs0;
                        qn[lane] = nq;
                        qsc[lane] = r2 > 0 ? (float)nq / (float)((uint32_t)(r2 >> gsh) + 1u) : 0.0f;
                        // (the owner map is free until the next group)
                        own[lane] = qo0;
                        own[kGroup + lane] = ko;
                    }
                    for (uint32_t t = lane; t < total; t += 64) hh[t] = 0u;
                    wave_sync();
                    // bucket of a key: its slot's rows start + about
                    // n * d^2 / r^2, below n, never smaller for a larger d^2
                    auto bucket = [&](uint64_t k) -> uint32_t {
                        const uint32_t sl = (uint32_t)(k >> (64u - kGroupBits));
                        const uint32_t d = (uint32_t)(k >> dsh) & dmask;
                        const uint32_t bi = min((uint32_t)((float)d * qsc[sl]), qn[sl] - 1u);
                        return qst[sl] + bi;
                    };
                    uint32_t slot[(kMaxHitCap + 63) / 64], bk[(kMaxHitCap + 63) / 64];
#pragma unroll
                    for (uint32_t k = 0; k < (kMaxHitCap + 63) / 64; ++k) {
                        const uint32_t t = lane + 64u * k;
                        bk[k] = 0u;
                        if (t < total) {
                            bk[k] = bucket(hb[t]);
                            slot[k] = atomicAdd(&hh[bk[k]], 1u);
                        }
                    }
                    wave_sync();
                    const uint32_t per = (total + 63u) >> 6;
                    const uint32_t bb = lane * per;
                    uint32_t sum = 0;
                    for (uint32_t k = 0; k < per; ++k)
                        if (bb + k < total) sum += hh[bb + k];
                    uint32_t run = scan_add(sum) - sum;
                    wave_sync();
                    for (uint32_t k = 0; k < per; ++k)
                        if (bb + k < total) {
                            const uint32_t c = hh[bb + k];
                            hh[bb + k] = run;
                            run += c;
                        }
                    wave_sync();
#pragma unroll
                    for (uint32_t k = 0; k < (kMaxHitCap + 63) / 64; ++k) {
                        const uint32_t t = lane + 64u * k;
                        if (t < total) hs[hh[bk[k]] + slot[k]] = hb[t];
                    }
                    wave_sync();
                    for (uint32_t t = lane; t < total; t += 64) {
                        const uint64_t key = hs[t];
                        const uint32_t bi = bucket(key);
                        const uint32_t lo = hh[bi], hi = bi + 1 < total ? hh[bi + 1] : total;
                        uint32_t rank = lo;
                        for (uint32_t j = lo; j < hi; ++j) rank += hs[j] < key ? 1u : 0u;
                        uint32_t o = cur + rank;
                        bool keep = true;
                        if (KNN) {
                            // its rank inside its slot's row, kept when below K
                            const uint32_t sl = (uint32_t)(key >> (64u - kGroupBits));
                            const uint32_t wr = rank - qst[sl];
                            keep = wr < own[kGroup + sl];
                            o = cur + own[sl] + wr;
                        }
                        if (keep) {
                            A.stash_ids[o] = (uint32_t)(key & idmask);
                            if (A.stash_d2) A.stash_d2[o] = (int64_t)key_d2(key, idbits, d2bits);
                        }
                    }
                    wave_sync();
                    if (mine) A.soff[row] = cur + (KNN ? qo0 : qs0);
                    cur += tout;
                } else {
                    // not kept: the write pass walks these rows again
                    const bool walk_again = mine && nq > 0;
                    if (mine) A.soff[row] = walk_again ? kMaxId : 0u;
                    const uint64_t wm = __ballot(walk_again);
                    uint32_t wb0 = 0;
                    if (wm != 0 && lane == 0) wb0 = atomicAdd(A.walk_count, (uint32_t)__popcll(wm));
                    wb0 = uni(wb0);
                    if (walk_again) A.walkq[wb0 + lanes_below(wm)] = qi;
                }
            }
            wave_sync();
        }
    }, kGroup);
}

// ---------------------------------------------------------------------------
// Pass 1, radius rows that fit the LDS buffer: collect, sort, store.

template <int METHOD, bool TLDS, bool FROM_LIST>
__global__ __launch_bounds__(256) void write_kernel(LatArgs L, TabArgs T, QArgs A) {
    extern __shared__ __align__(16) char smem[];
    const uint32_t* tab_lds = stage_table<TLDS>(T, smem);
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t cap = A.sort_cap;
    char* wb = smem + table_lds_bytes<TLDS>(T) + (size_t)wave * ((size_t)cap * 28 + 256);
    uint64_t* td = (uint64_t*)wb;
    uint64_t* sd = td + cap;
    uint32_t* ti = (uint32_t*)(sd + cap);
    uint32_t* si = ti + cap;
    uint32_t* hist = si + cap;
    uint32_t* own = hist + cap;
    if (A.row_ptr[A.Q] > A.capacity) {
        if (threadIdx.x == 0) atomicOr(L.status, SPHIDX_FLAG_CAPACITY);
        return;
    }
    const AxisWrap aw = axis_wrap(L);
    const uint32_t lane = lane_id();
    // after a stashing count pass only the rows it did not keep are walked:
    // the main launch takes the walk list, the list launch skips kept rows
    const bool stashed = A.stash_hdr[kHdrMode] != 0u;
    const bool from_walk = !FROM_LIST && stashed;
    const uint32_t idbits = L.n > 1 ? 32u - (uint32_t)__builtin_clz(L.n - 1u) : 0u;  // ids are below n
    const uint32_t nq = FROM_LIST ? uni(*A.list_count) : (from_walk ? uni(*A.walk_count) : A.Q);
    for_each_query(nq, A, queue_set(A, FROM_LIST ? (int)A.list_set : (from_walk ? kQWalk : kQWrite)),
                   [&](uint32_t ti_) {
        const uint32_t qi = FROM_LIST ? uni(A.list[ti_]) : (from_walk ? uni(A.walkq[ti_]) : ti_);
        const Query s = load_query(L, A, qi);
        if (FROM_LIST && stashed && uni(A.soff[s.row]) != kMaxId) return;  // copied by the gather kernel
        if ((METHOD == kSphere || METHOD == kPaper) && (s.flags & F_VALID) && !(s.flags & F_SPHERE))
            return;  // fallback list
        const int64_t rb = A.row_ptr[s.row];
        const uint32_t rowlen = (uint32_t)(A.row_ptr[s.row + 1] - rb);
        if (rowlen == 0 || !(s.flags & F_VALID)) return;
        if ((s.flags & F_KNN) || rowlen > cap) {
            // handled by the top-M kernel
            if (lane == 0) A.longq[atomicAdd(A.long_count, 1u)] = qi;
            return;
        }
        uint32_t n = 0, cand = 0, walked = 0;
        auto visit = [&](bool act, uint32_t p, const uint4& P) -> bool {
            const uint64_t d2 = obj_dist2(aw, s, P);
            const bool hit = act && d2 <= s.r2 && p != s.self;
            const uint64_t hm = __ballot(hit);
            if (hit) {
                const uint32_t slot = n + lanes_below(hm);
                if (slot < cap) {
                    td[slot] = d2;
                    ti[slot] = P.w;
                }
            }
            n += (uint32_t)__popcll(hm);
            return false;
        };
        walk<METHOD, TLDS, false>(L, T, tab_lds, s, false, walked, [&]() { return s.r2; },
                                         [&](const RowRef& r) -> bool {
            return for_candidates(L, r.st0, r.cnt0, r.st1, r.cnt1, own, cand, visit);
        });
        wave_sync();
        sort_row_store(td, ti, sd, si, hist, min(n, rowlen), s.r2, idbits, A.out_ids + rb,
                       A.out_d2 ? A.out_d2 + rb : nullptr);
        wave_sync();
    });
}

// ---------------------------------------------------------------------------
// Pass 1, K-NN rows and long radius rows: sorted top-M in LDS with the
// shrinking bound, in windows of at most `cap` entries (each window takes
// the M smallest pairs above the previous window's last one).

template <int METHOD, bool TLDS, bool FROM_LIST>
__global__ __launch_bounds__(256) void topm_kernel(LatArgs L, TabArgs T, QArgs A) {
    extern __shared__ __align__(16) char smem[];
    const uint32_t* tab_lds = stage_table<TLDS>(T, smem);
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t cap = A.sort_cap;
    char* wb = smem + table_lds_bytes<TLDS>(T) + (size_t)wave * ((size_t)cap * 24 + 64 * 12 + 256);
    uint64_t* tdA = (uint64_t*)wb;
    uint64_t* tdB = tdA + cap;
    uint64_t* bd = tdB + cap;
    uint32_t* tiA = (uint32_t*)(bd + 64);
    uint32_t* tiB = tiA + cap;
    uint32_t* bi = tiB + cap;
    uint32_t* own = bi + 64;
    if (A.row_ptr[A.Q] > A.capacity) {
        if (threadIdx.x == 0) atomicOr(L.status, SPHIDX_FLAG_CAPACITY);
        return;
    }
    const AxisWrap aw = axis_wrap(L);
    const uint32_t lane = lane_id();
    // every query, unless a stashing count pass kept rows and the copy placed
    // them: then only the rows it could not keep, which it listed on the walk
    // list (when this call asks for dist^2 and the stash holds none, the copy
    // placed nothing and every row is searched)
    const bool from_walk = !FROM_LIST && A.stash_hdr[kHdrMode] != 0u && !(A.out_d2 && A.stash_hdr[kHdrHasD2] == 0u);
    const uint32_t nq = FROM_LIST ? uni(*A.list_count) : from_walk ? uni(*A.walk_count) : A.Q;
    for_each_query(nq, A, queue_set(A, kQTopm), [&](uint32_t ti_) {
        const uint32_t qi = FROM_LIST ? uni(A.list[ti_]) : from_walk ? uni(A.walkq[ti_]) : ti_;
        const Query s = load_query(L, A, qi);
        if (!FROM_LIST && !(s.flags & F_KNN)) return;
        const int64_t rb = A.row_ptr[s.row];
        const uint32_t rowlen = (uint32_t)(A.row_ptr[s.row + 1] - rb);
        if (rowlen == 0 || !(s.flags & F_VALID)) return;
        // long radius rows the block-per-row kernel takes
        if (FROM_LIST && A.long_waves > 1 && !(s.flags & F_KNN) && rowlen <= kLongCap) return;
        uint64_t* td = tdA;
        uint64_t* ud = tdB;
        uint32_t* tix = tiA;
        uint32_t* uix = tiB;
        bool has_lower = false;
        uint64_t ld = 0;
        uint32_t li = 0;
        uint32_t written = 0;
        while (written < rowlen) {
            const uint32_t M = min(cap, rowlen - written);
            const uint32_t target = written + M;
            uint64_t B = first_bound(L, s, target, rowlen);
            if (M <= 64) {
                // ---- a window of at most 64 in registers
                uint64_t rd;
                uint32_t ri;
                const uint32_t got = topm_registers<METHOD, TLDS>(L, T, tab_lds, s, aw, own, M, B, has_lower, ld, li,
                                                                   rd, ri);
                if (lane < got) {
                    A.out_ids[rb + written + lane] = ri;
                    if (A.out_d2) A.out_d2[rb + written + lane] = (int64_t)rd;
                }
                if (got == 0) break;
                has_lower = true;
                ld = lane_val64(rd, got - 1u);
                li = lane_val(ri, got - 1u);
                written += got;
                continue;
            }
            uint32_t m = 0;
            uint64_t bdd = kMaxD2;
            uint32_t bii = kMaxId;
            uint32_t cand = 0, walked = 0;
            auto visit = [&](bool act, uint32_t p, const uint4& P) -> bool {
                const uint64_t d2 = obj_dist2(aw, s, P);
                const uint32_t id = P.w;
                bool cv = act && d2 <= B && p != s.self;
                if (cv && has_lower) cv = key_less(ld, li, d2, id);
                if (cv && m == M) cv = key_less(d2, id, bdd, bii);
                const uint64_t bm = __ballot(cv);
                if (bm == 0) return false;
                const uint32_t nb = (uint32_t)__popcll(bm);
                uint64_t cd = cv ? d2 : kMaxD2;
                uint32_t ci = cv ? id : kMaxId;
                wave_sort64(cd, ci);
                bd[lane] = cd;
                bi[lane] = ci;
                wave_sync();
                const uint32_t nm = min(M, m + nb);
                // merge: an element's place = own index + elements of the
                // other sorted list that are smaller (ids are unique)
                for (uint32_t t = lane; t < m; t += 64) {
                    const uint64_t xd = td[t];
                    const uint32_t xi = tix[t];
                    uint32_t lo = 0, hi = nb;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (key_less(bd[mid], bi[mid], xd, xi))
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    if (t + lo < nm) {
                        ud[t + lo] = xd;
                        uix[t + lo] = xi;
                    }
                }
                if (lane < nb) {
                    uint32_t lo = 0, hi = m;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (key_less(td[mid], tix[mid], cd, ci))
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    if (lane + lo < nm) {
                        ud[lane + lo] = cd;
                        uix[lane + lo] = ci;
                    }
                }
                wave_sync();
                uint64_t* sd = td;
                td = ud;
                ud = sd;
                uint32_t* si = tix;
                tix = uix;
                uix = si;
                m = nm;
                if (m == M) {
                    bdd = uni64(td[M - 1]);
                    bii = uni(tix[M - 1]);
                }
                return false;
            };
            // every object within B is visited and nothing beyond B is kept,
            // so M kept means they are the M nearest above the lower bound
            for (;;) {
                walk<METHOD, TLDS, true>(L, T, tab_lds, s, false, walked, [&]() { return m == M ? bdd : B; },
                                                [&](const RowRef& r) -> bool {
                    return for_candidates(L, r.st0, r.cnt0, r.st1, r.cnt1, own, cand, visit);
                });
                if (m == M || B >= s.r2) break;
                B = min(s.r2, B + B + (B >> 2) + 1u);  // radius x1.5
                m = 0;
                bdd = kMaxD2;
                bii = kMaxId;
            }
            wave_sync();
            const uint32_t got = min(m, M);
            store_sorted(A, td, tix, got, rb + written);
            if (got == 0) break;
            has_lower = true;
            ld = uni64(td[got - 1]);
            li = uni(tix[got - 1]);
            written += got;
            wave_sync();
        }
    });
}

// ---------------------------------------------------------------------------
// Pass 1, radius rows longer than a wavefront's LDS row buffer and at most
// kLongCap pairs: one block of W waves per row.  Wave w walks the row's
// table entries in 64-entry steps w, w + W, ..., tests their candidates and
// appends its hits to a block-wide LDS buffer (one LDS atomic per wave
// step).  The block then orders the row by (dist^2, id) with one bucket
// sort -- bucket floor(n d^2 / r^2), capped at n - 1, is monotone in d^2 --
// and an exact rank inside each bucket, and stores it.  Rows come from the
// long-row list one per block; the top-M kernel leaves them alone.

// Exclusive scan over the block of one value per thread; `wsum` holds one
// word per wavefront.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* wsum) {
    const uint32_t wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t incl = scan_add(v);
    if (lane_id() == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (uint32_t w = 0; w < nw; ++w) off += w < wave ? wsum[w] : 0u;
    __syncthreads();
    return off + incl - v;
}

// Sort the block's n <= kLongCap pairs (td, ti) by (dist^2, id) and store
// them at dst; every pair has dist^2 <= r2.  The pairs stay where they are:
// the bucket pass orders their indices (sx), which the rank pass follows.
__device__ void block_sort_store(const uint64_t* td, const uint32_t* ti, uint32_t* sx, uint32_t* hist,
                                 uint32_t* wsum, uint32_t n, uint64_t r2, uint32_t* dst_ids, int64_t* dst_d2) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const float scale = r2 > 0 ? (float)n / (float)r2 : 0.0f;
    for (uint32_t t = tid; t < n; t += nt) hist[t] = 0u;
    __syncthreads();
    for (uint32_t t = tid; t < n; t += nt) atomicAdd(&hist[sort_bucket(td[t], scale, n)], 1u);
    __syncthreads();
    // bucket starts: each thread owns a run of buckets
    const uint32_t per = (n + nt - 1) / nt, b0 = tid * per;
    uint32_t sum = 0;
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < n) sum += hist[b0 + k];
    uint32_t run = block_scan_excl(sum, wsum);
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < n) {
            const uint32_t c = hist[b0 + k];
            hist[b0 + k] = run;
            run += c;
        }
    __syncthreads();
    // scatter the indices by bucket: each bucket's cursor ends at the next
    // one's start
    for (uint32_t t = tid; t < n; t += nt) sx[atomicAdd(&hist[sort_bucket(td[t], scale, n)], 1u)] = t;
    __syncthreads();
    for (uint32_t t = tid; t < n; t += nt) {
        const uint32_t i = sx[t];
        const uint64_t d = td[i];
        const uint32_t id = ti[i];
        const uint32_t b = sort_bucket(d, scale, n);
        const uint32_t lo = b ? hist[b - 1] : 0u, hi = hist[b];
        uint32_t rank = lo;
        for (uint32_t j = lo; j < hi; ++j) {
            const uint32_t o = sx[j];
            rank += key_less(td[o], ti[o], d, id) ? 1u : 0u;
        }
        dst_ids[rank] = id;
        if (dst_d2) dst_d2[rank] = (int64_t)d;
    }
}

// COUNT: the count pass's form.  The rows come from the list of rows the
// setup expected to be long; the block counts the row, writes its size and,
// when it holds at most kLongCap pairs and the stash has room, orders it into
// the stash (one allocation per row) for the write pass to copy; otherwise
// the row goes on the walk list like any row the count pass did not keep.
template <int METHOD, bool COUNT>
__global__ __launch_bounds__(512) void long_kernel(LatArgs L, TabArgs T, QArgs A) {
    extern __shared__ __align__(16) char smem[];
    uint64_t* td = (uint64_t*)smem;  // hits in arrival order
    uint32_t* ti = (uint32_t*)(td + kLongCap);
    uint32_t* sx = ti + kLongCap;    // their indices by bucket
    uint32_t* hist = sx + kLongCap;
    uint32_t* ctl = hist + kLongCap;  // [0] hits so far, [1] list entry taken, [2] stash offset, [4, 12) wave sums
    const uint32_t wave = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = lane_id();
    uint32_t* own = ctl + 16 + wave * 64;
    if (!COUNT && A.row_ptr[A.Q] > A.capacity) return;  // (the write kernel sets the flag)
    const AxisWrap aw = axis_wrap(L);
    const uint32_t nq = uni(*A.list_count);
    uint32_t* qc = queue_set(A, (int)A.list_set);
    const uint32_t region = blockIdx.x % SPHIDX_NREGION;
    for (;;) {
        if (threadIdx.x == 0) {
            ctl[1] = atomicAdd(qc, 1u);
            ctl[0] = 0u;
        }
        __syncthreads();
        const uint32_t t = uni(ctl[1]);
        if (t >= nq) break;
        const uint32_t qi = uni(A.list[t]);
        const Query s = load_query(L, A, qi);
        int64_t rb = 0;
        uint32_t rowlen = kLongCap;
        if (!COUNT) {
            rb = A.row_ptr[s.row];
            rowlen = (uint32_t)(A.row_ptr[s.row + 1] - rb);
        }
        // the same for every wave of the block
        const bool mine = (s.flags & F_VALID) && !(s.flags & F_KNN) && rowlen > 0 && rowlen <= kLongCap;
        if (mine) {
            uint32_t cand = 0, walked = 0;
            auto visit = [&](bool act, uint32_t p, const uint4& P) -> bool {
                const uint64_t d2 = obj_dist2(aw, s, P);
                const bool hit = act && d2 <= s.r2 && p != s.self;
                const uint64_t hm = __ballot(hit);
                if (hm) {
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(&ctl[0], (uint32_t)__popcll(hm));
                    base = uni(base);
                    const uint32_t slot = base + lanes_below(hm);
                    if (hit && slot < kLongCap) {
                        td[slot] = d2;
                        ti[slot] = P.w;
                    }
                }
                return false;
            };
            walk<METHOD, false, false>(L, T, nullptr, s, false, walked, [&]() { return s.r2; },
                                       [&](const RowRef& r) -> bool {
                return for_candidates(L, r.st0, r.cnt0, r.st1, r.cnt1, own, cand, visit);
            }, 64u * wave, 64u * nw);
        }
        __syncthreads();
        if (COUNT) {
            const uint32_t n = (s.flags & F_VALID) ? ctl[0] : 0u;
            if (threadIdx.x == 0) {
                A.row_ptr[s.row] = (int64_t)n;
                uint32_t off = 0u;  // empty rows: nothing to copy
                if (n > 0) {
                    off = kMaxId;
                    if (n <= kLongCap && A.stash) {
                        const uint32_t c = atomicAdd(A.stash_ctr + region * SPHIDX_QSTRIDE, n);
                        if ((uint64_t)c + n <= A.stash_region) off = region * A.stash_region + c;
                    }
                    if (off == kMaxId) A.walkq[atomicAdd(A.walk_count, 1u)] = qi;
                }
                A.soff[s.row] = off;
                ctl[2] = off;
            }
            __syncthreads();
            const uint32_t off = ctl[2];
            if (n > 0 && off != kMaxId)
                block_sort_store(td, ti, sx, hist, ctl + 4, n, s.r2, A.stash_ids + off,
                                 A.stash_d2 ? A.stash_d2 + off : nullptr);
        } else if (mine) {
            block_sort_store(td, ti, sx, hist, ctl + 4, min(ctl[0], rowlen), s.r2, A.out_ids + rb,
                             A.out_d2 ? A.out_d2 + rb : nullptr);
        }
        __syncthreads();
    }
}

// Zero counter words [begin, end); the count pass also writes the stash
// header (hdr != NULL: four words) after clearing.
// Counters sit SPHIDX_QSTRIDE words apart and only those words are read:
// the others are left as they are.  One block; the stash header, inside the
// cleared range, is written after every clear.
__global__ void clear_counters_kernel(uint32_t* c, uint32_t begin, uint32_t end, uint32_t* hdr, uint4 hv) {
    for (uint32_t i = begin + threadIdx.x * SPHIDX_QSTRIDE; i < end; i += blockDim.x * SPHIDX_QSTRIDE) c[i] = 0u;
    __syncthreads();
    if (hdr && threadIdx.x == 0) {
        hdr[kHdrMode] = hv.x;
        hdr[kHdrElems] = hv.y;
        hdr[kHdrHasD2] = hv.z;
        hdr[kHdrD2Off] = hv.w;
    }
}

// Pass 1 with the stash: copy each kept row into place.  A wavefront takes 64
// consecutive output rows and reads each one's stash offset (kept per output
// row) and its place from row_ptr.  Their objects are numbered in row order (a
// prefix sum), and each lane copies every 64th of them: its row is the last
// whose first number is at most the object's, found by a binary search over
// the starts kept in LDS (read-only, so steps need no barrier and four are in
// flight).  The writes are then one sequential stream per wavefront and each
// stash row is one contiguous read; rows come out of the count pass in lattice
// order, which is not the output's order for all-agents queries, and writing
// rows scattered over the output costs more than reading them scattered.
// Rows the count pass could not keep are left to the write kernel (offset ~0).
// When the write wants dist^2 and the stash lacks it, every kept row is walked
// again instead, and the walk list takes query slots: then the wavefront takes
// 64 consecutive query slots and finds each one's output row.
__global__ __launch_bounds__(256) void gather_kernel(QArgs A, const uint4* pts, uint32_t* status) {
    __shared__ uint32_t starts_all[4 * 64];
    const uint32_t* hdr = A.stash_hdr;
    if (hdr[kHdrMode] == 0u) return;
    if (A.row_ptr[A.Q] > A.capacity) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(status, SPHIDX_FLAG_CAPACITY);
        return;
    }
    const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
    uint32_t* starts = starts_all + wave * 64;
    const uint64_t q0 = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + wave) * 64u;
    if (q0 >= A.Q) return;
    const uint32_t* s_ids = (const uint32_t*)A.stash_base;
    const bool has_d2 = hdr[kHdrHasD2] != 0u;
    const int64_t* s_d2 = (const int64_t*)(A.stash_base + hdr[kHdrD2Off] * (size_t)256);
    // walk again (dist^2 wanted, not stashed): by query slot; else by output row
    const bool again = A.out_d2 && !has_d2;
    const uint64_t qi = q0 + lane;
    uint32_t len = 0, src = 0;
    int64_t dst = 0;
    if (qi < A.Q) {
        // the output row: the object's id for all-agents queries (their
        // processing order is the sorted order), else the query index
        const uint32_t row = (again && A.qx == nullptr) ? pts[qi].w : (uint32_t)qi;
        src = A.soff[row];
        if (src != kMaxId) {
            dst = A.row_ptr[row];
            len = (uint32_t)(A.row_ptr[row + 1] - dst);
            if (len > 0 && again) {
                // the stash holds no dist^2 for this row: it is walked again,
                // by the main write kernel (from the walk list) or, for a row
                // off the sphere tables, by the list kernels, which walk rows
                // whose offset says "not kept"; marked so once, a later write
                // does not list it again
                A.soff[row] = kMaxId;
                A.walkq[atomicAdd(A.walk_count, 1u)] = (uint32_t)qi;
                len = 0;
            }
        }
    }
    const uint32_t incl = scan_add(len);
    const uint32_t total = lane_val(incl, 63);
    const uint32_t excl = incl - len;
    starts[lane] = excl;
    wave_sync();
    // object g of query o is at stash sbase[o] + g and output dbase[o] + g
    const uint32_t sbase = src - excl;
    const uint64_t dbase = (uint64_t)(dst - (int64_t)excl);
    const bool want_d2 = A.out_d2 != nullptr;
    constexpr uint32_t kSteps = 4;
    for (uint32_t cb = 0; cb < total; cb += 64u * kSteps) {
        uint32_t v[kSteps];
        int64_t w[kSteps], dp[kSteps];
#pragma unroll
        for (uint32_t k = 0; k < kSteps; ++k) {
            const uint32_t g = cb + 64u * k + lane;
            // the last query whose first object number is <= g (a query with
            // an empty row shares its start with the next, which wins)
            uint32_t o = 0;
#pragma unroll
            for (uint32_t step = 32; step; step >>= 1)
                if (starts[o + step] <= g) o += step;
            const uint32_t sp = bperm(sbase, o) + g;
            dp[k] = (int64_t)(((uint64_t)bperm((uint32_t)(dbase >> 32), o) << 32) | bperm((uint32_t)dbase, o)) + g;
            v[k] = 0u;
            w[k] = 0;
            if (g < total) {
                v[k] = s_ids[sp];
                if (want_d2) w[k] = s_d2[sp];
            }
        }
#pragma unroll
        for (uint32_t k = 0; k < kSteps; ++k) {
            if (cb + 64u * k + lane < total) {
                A.out_ids[dp[k]] = v[k];
                if (want_d2) A.out_d2[dp[k]] = w[k];
            }
        }
    }
}

// Kernel choice by variant: cube, sphere, sphere with the row table in LDS;
// SPHIDX_PICKP adds variant 3, the paper's cell tables.
#define SPHIDX_PICK(KERNEL, variant, SPH, ...)                                     \
    ((variant) == 0 ? (const void*)KERNEL<kCube, false __VA_ARGS__>                \
     : (variant) == 1 ? (const void*)KERNEL<SPH, false __VA_ARGS__>                \
                      : (const void*)KERNEL<SPH, true __VA_ARGS__>)
#define SPHIDX_PICKP(KERNEL, variant, SPH, ...) \
    ((variant) == 3 ? (const void*)KERNEL<kPaper, false __VA_ARGS__> : SPHIDX_PICK(KERNEL, variant, SPH, __VA_ARGS__))

hipError_t launch_ptr(const void* fn, uint32_t nq, const QArgs& q, uint32_t waves, uint32_t bpc, size_t shmem,
                      hipStream_t st, const LatArgs& L, const TabArgs& T) {
    uint32_t blocks;
    if (q.persistent) {
        blocks = (uint32_t)device_cu_count() * bpc;
    } else {
        const uint64_t per = (uint64_t)waves * q.tile;
        blocks = (uint32_t)((nq + per - 1) / per);
        if (blocks == 0) blocks = 1;
    }
    LatArgs l = L;
    TabArgs t = T;
    QArgs a = q;
    void* args[] = {&l, &t, &a};
    return hipLaunchKernel(fn, dim3(blocks), dim3(waves * 64), args, shmem, st);
}

}  // namespace

int device_cu_count() {
    static int cached = 0;
    if (cached) return cached;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    cached = cus;
    return cus;
}

size_t long_lds_bytes(uint32_t waves) { return (size_t)kLongCap * 20 + 64 + (size_t)waves * 256; }

// LDS bytes per block: pass 0 count (3 with the stash), 1 write, 2 top-M,
// 4 grouped count (5 with the stash).
size_t query_lds_bytes(int pass, uint32_t cap, uint32_t waves, size_t table_bytes) {
    size_t per = 256;
    if (pass == 1 || pass == 3) per = (size_t)cap * 28 + 256;
    if (pass == 2) per = (size_t)cap * 24 + 64 * 12 + 256;
    if (pass == 4 || pass == 5) per = group_lds_per_wave(pass == 5, cap);
    return table_bytes + per * waves;
}

hipError_t launch_query_pass(int pass, const LatArgs& L, const TabArgs& T, const QArgs& q,
                             uint32_t waves_per_block, uint32_t blocks_per_cu, hipStream_t st,
                             hipEvent_t ev_begin, hipEvent_t ev_end) {
    // optional timing events around the pass's main kernel(s)
    auto mark = [st](hipEvent_t ev) { return ev ? hipEventRecord(ev, st) : hipSuccess; };
    const size_t tb = tab_lds_bytes(T);
    const int variant = !T.has ? 0 : T.paper ? 3 : (T.lds ? 2 : 1);
    const uint32_t lists = SPHIDX_NQSETS * SPHIDX_NQUEUE * SPHIDX_QSTRIDE;
    const uint32_t set_words = SPHIDX_NQUEUE * SPHIDX_QSTRIDE;
    hipError_t e;
    // one block per long radius row (count pass: the rows the setup listed;
    // write pass: rows longer than a wavefront's buffer)
    auto launch_long = [&](bool count, const QArgs& qa) -> hipError_t {
        const void* lf =
            count ? (variant == 0   ? (const void*)long_kernel<kCube, true>
                     : variant == 3 ? (const void*)long_kernel<kPaper, true>
                                    : (const void*)long_kernel<kEither, true>)
                  : (variant == 0   ? (const void*)long_kernel<kCube, false>
                     : variant == 3 ? (const void*)long_kernel<kPaper, false>
                                    : (const void*)long_kernel<kEither, false>);
        const size_t lds = long_lds_bytes(qa.long_waves);
        const uint32_t per_cu = (uint32_t)std::max<size_t>(1, (160u * 1024u) / lds);
        LatArgs l = L;
        TabArgs t = T;
        QArgs a = qa;
        void* args[] = {&l, &t, &a};
        return hipLaunchKernel(lf, dim3((uint32_t)device_cu_count() * per_cu), dim3(64u * qa.long_waves), args, lds,
                               st);
    };
    // whether the setup can have listed rows for it: a radius at the tables'
    // cap (per-query radii) or the batch's radius, at the lattice's mean
    // density, expected above 5/4 of the row buffer (the setup's test, with a
    // margin for its single precision)
    auto long_rows_possible = [&]() -> bool {
        if (!q.stash || q.long_waves <= 1 || q.mode == SPHIDX_MODE_KNN || q.stats || L.ncells == 0) return false;
        if (q.rad && (!T.has || q.select == 1u)) return true;
        const double rc = (double)(q.rad ? T.rmax : q.rad_u) / (double)(1u << L.F);
        return 4.18879 * rc * rc * rc * ((double)L.n / (double)L.ncells) > 0.98 * 1.25 * (double)q.sort_cap;
    };
    if (pass == 0) {
        // everything, then the stash header for the write pass
        const uint4 hv = make_uint4(q.stash, q.stash ? q.stash_region * SPHIDX_NREGION : 0u, q.stash_d2 ? 1u : 0u,
                                    q.stash_d2 ? (uint32_t)(((char*)q.stash_d2 - q.stash_base) / 256) : 0u);
        clear_counters_kernel<<<1, 256, 0, st>>>(q.queues, 0u, SPHIDX_COUNTER_WORDS, q.stash_hdr, hv);
    } else {
        // the write-side queue sets and the long-row list; the descriptors,
        // the fallback and walk lists, the stash header and the stash
        // counters stay as the count pass left them
        clear_counters_kernel<<<1, 256, 0, st>>>(q.queues, set_words, lists + SPHIDX_QSTRIDE, nullptr,
                                                 make_uint4(0, 0, 0, 0));
    }
    e = hipGetLastError();
    if (e != hipSuccess || q.Q == 0) return e;
    if (pass == 0) {
        // per-query descriptors (and, for the sphere method, the fallback list)
        if (variant == 0)
            setup_kernel<kCube><<<(q.Q + 255) / 256, 256, 0, st>>>(L, T, q);
        else if (variant == 3)
            setup_kernel<kPaper><<<(q.Q + 255) / 256, 256, 0, st>>>(L, T, q);
        else
            setup_kernel<kSphere><<<(q.Q + 255) / 256, 256, 0, st>>>(L, T, q);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const uint32_t w = waves_per_block, b = blocks_per_cu;
    // per-query choice: the main kernels walk the sphere, the cube or the
    // cell list per query (grouping them apart would split the groups)
    const bool either = variant != 0 && q.select == 1u;
    QArgs ql = q;  // list-driven launches: persistent, grabs sized from the list
    ql.persistent = 1;
    // the count pass's long rows: the setup's list, with the walk-list queue
    // set (the write pass's, cleared when it starts)
    auto long_list = [&]() {
        QArgs a = ql;
        a.list = q.lq;
        a.list_count = q.lq_count;
        a.list_set = kQWalk;
        return a;
    };
    if (pass == 0) {
        const int lp = q.stash ? 3 : 0;
        // K-NN rows searched and kept by the count pass
        const bool ks = q.stash && q.mode != SPHIDX_MODE_RADIUS;
        if ((e = mark(ev_begin)) != hipSuccess) return e;
        if (q.group) {
            // radius queries in groups: all queries (those of the tables),
            // then the fallback list's (bounding cube); the rest through the
            // extra list, one query per wavefront
            const size_t gl = query_lds_bytes(q.stash ? 5 : 4, q.sort_cap, w, tb);
            const bool gk = q.mode != SPHIDX_MODE_RADIUS;  // K-NN queries in the batch
            if (q.stash)
                e = launch_ptr(gk ? (either ? SPHIDX_PICK(group_count_kernel, variant, kEither, , true, false, true)
                                            : SPHIDX_PICK(group_count_kernel, variant, kSphere, , true, false, true))
                                  : (either ? SPHIDX_PICK(group_count_kernel, variant, kEither, , true, false, false)
                                            : SPHIDX_PICK(group_count_kernel, variant, kSphere, , true, false, false)),
                               q.Q, q, w, b, gl, st, L, T);
            else
                e = launch_ptr(gk ? (either ? SPHIDX_PICK(group_count_kernel, variant, kEither, , false, false, true)
                                            : SPHIDX_PICK(group_count_kernel, variant, kSphere, , false, false, true))
                                  : (either ? SPHIDX_PICK(group_count_kernel, variant, kEither, , false, false, false)
                                            : SPHIDX_PICK(group_count_kernel, variant, kSphere, , false, false, false)),
                               q.Q, q, w, b, gl, st, L, T);
            if (e == hipSuccess) e = mark(ev_end);
            if (e != hipSuccess) return e;
            if (long_rows_possible() && (e = launch_long(true, long_list())) != hipSuccess) return e;
            if (variant != 0 && !either) {
                QArgs qg = ql;
                qg.list = q.fbq;
                qg.list_count = q.fb_count;
                qg.list_set = kQFbCount;
                const size_t gl0 = query_lds_bytes(q.stash ? 5 : 4, q.sort_cap, w, 0);
                e = launch_ptr(q.stash ? (const void*)group_count_kernel<kCube, false, true, true, false>
                                       : (const void*)group_count_kernel<kCube, false, false, true, false>,
                               0, qg, w, b, gl0, st, L, T);
                if (e != hipSuccess) return e;
            }
            ql.list = q.xq;
            ql.list_count = q.xq_count;
            ql.list_set = kQExtra;
            if (gk && variant != 0) {
                // K-NN rows short of K inside their first radius: a second
                // grouped round at a larger radius; what it leaves goes on
                // the long-row list (free until the write pass) to the
                // one-query-per-wave kernel
                QArgs qr = ql;
                qr.xq = q.longq;
                qr.xq_count = q.long_count;
                e = launch_ptr(q.stash ? (either ? SPHIDX_PICK(group_count_kernel, variant, kEither, , true, true, true)
                                                 : SPHIDX_PICK(group_count_kernel, variant, kSphere, , true, true, true))
                                       : (either ? SPHIDX_PICK(group_count_kernel, variant, kEither, , false, true, true)
                                                 : SPHIDX_PICK(group_count_kernel, variant, kSphere, , false, true, true)),
                               0, qr, w, b, gl, st, L, T);
                if (e != hipSuccess) return e;
                ql.list = q.longq;
                ql.list_count = q.long_count;
                ql.list_set = kQExtra2;
            }
            if (ks)
                return launch_ptr(SPHIDX_PICK(count_kernel, variant, kEither, , true, true, true), 0, ql, w, b,
                                  query_lds_bytes(lp, q.sort_cap, w, tb), st, L, T);
            if (q.stash)
                return launch_ptr(SPHIDX_PICK(count_kernel, variant, kEither, , true, true, false), 0, ql, w, b,
                                  query_lds_bytes(lp, q.sort_cap, w, tb), st, L, T);
            return launch_ptr(SPHIDX_PICK(count_kernel, variant, kEither, , true, false, false), 0, ql, w, b,
                              query_lds_bytes(lp, q.sort_cap, w, tb), st, L, T);
        }
        const void* fn;
        if (ks)
            fn = either ? SPHIDX_PICK(count_kernel, variant, kEither, , false, true, true)
                        : SPHIDX_PICKP(count_kernel, variant, kSphere, , false, true, true);
        else if (q.stash)
            fn = either ? SPHIDX_PICK(count_kernel, variant, kEither, , false, true, false)
                        : SPHIDX_PICKP(count_kernel, variant, kSphere, , false, true, false);
        else
            fn = either ? SPHIDX_PICK(count_kernel, variant, kEither, , false, false, false)
                        : SPHIDX_PICKP(count_kernel, variant, kSphere, , false, false, false);
        e = launch_ptr(fn, q.Q, q, w, b, query_lds_bytes(lp, q.sort_cap, w, tb), st, L, T);
        if (e == hipSuccess) e = mark(ev_end);
        if (e != hipSuccess) return e;
        if (long_rows_possible() && (e = launch_long(true, long_list())) != hipSuccess) return e;
        if (variant == 0 || either) return hipSuccess;
        ql.list = q.fbq;
        ql.list_count = q.fb_count;
        ql.list_set = kQFbCount;
        return launch_ptr(ks        ? (const void*)count_kernel<kCube, false, true, true, true>
                          : q.stash ? (const void*)count_kernel<kCube, false, true, true, false>
                                    : (const void*)count_kernel<kCube, false, true, false, false>,
                          0, ql, w, b, query_lds_bytes(lp, q.sort_cap, w, 0), st, L, T);
    }
    const size_t sh1 = query_lds_bytes(1, q.sort_cap, w, tb);
    const size_t sh2 = query_lds_bytes(2, q.sort_cap, w, tb);
    if (q.mode != SPHIDX_MODE_KNN) {
        if ((e = mark(ev_begin)) != hipSuccess) return e;
        // rows kept by a stashing count pass (does nothing otherwise)
        gather_kernel<<<(q.Q + 255) / 256, 256, 0, st>>>(q, L.pts, L.status);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        e = launch_ptr(either ? SPHIDX_PICK(write_kernel, variant, kEither, , false)
                              : SPHIDX_PICKP(write_kernel, variant, kSphere, , false),
                       q.Q, q, w, b, sh1, st, L, T);
        if (e == hipSuccess) e = mark(ev_end);
        if (e != hipSuccess) return e;
        if (variant != 0 && !either) {
            ql.list = q.fbq;
            ql.list_count = q.fb_count;
            ql.list_set = kQFbWrite;
            e = launch_ptr((const void*)write_kernel<kCube, false, true>, 0, ql, w, b,
                           query_lds_bytes(1, q.sort_cap, w, 0), st, L, T);
            if (e != hipSuccess) return e;
        }
        // K-NN rows of a mixed batch and long radius rows, from the list:
        // radius rows up to kLongCap pairs one block per row, the others
        // one wavefront per row (windowed top-M)
        ql.list = q.longq;
        ql.list_count = q.long_count;
        if (q.long_waves > 1) {
            ql.list_set = kQExtra;
            if ((e = launch_long(false, ql)) != hipSuccess) return e;
        }
        ql.list_set = kQTopm;
        return launch_ptr(SPHIDX_PICKP(topm_kernel, variant, kEither, , true), 0, ql, w, b, sh2, st, L, T);
    }
    if ((e = mark(ev_begin)) != hipSuccess) return e;
    // rows kept by the count pass (does nothing otherwise), then the rest
    gather_kernel<<<(q.Q + 255) / 256, 256, 0, st>>>(q, L.pts, L.status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = launch_ptr(SPHIDX_PICKP(topm_kernel, variant, kEither, , false), q.Q, q, w, b, sh2, st, L, T);
    return e == hipSuccess ? mark(ev_end) : e;
}
