// Neighbourhood query kernels for gfx950 (wave64), one wavefront per query.
//
// Per query (all values wave-uniform):
//   setup   cell = q >> F, sub-cell class = top s bits of q's position inside
//           its cell, r^2; the class table's prefix end from the radius index
//           (Section II.A: a single lookup gives where to stop; Section III.A:
//           the sub-cell position selects a specialised table).
//   walk    the 64 lanes take 64 consecutive table entries (cells sorted by
//           increasing key, centre to edge).  Each lane translates its offset
//           to an absolute cell (wrap on cyclic axes, region test on clipped
//           ones, Section II.B), applies the exact run-time test min-dist^2 <=
//           r^2 (Eq. 1, applied to every entry) and, in the count pass, the
//           unconditional inclusion of cells wholly inside the sphere
//           (Section III.A, last paragraph).
//   scan    the kept cells' objects are flattened over the lanes (inclusive
//           scan of per-lane counts + a 6-step search for the owning lane),
//           so a wave tests 64 candidates per step whatever the cell loads.
//   output  pass 0 counts hits per row (K-NN: min(K, hits within the cap),
//           stopping as soon as K are found).  Pass 1 collects the row in LDS
//           (ballot + mbcnt compaction), sorts it by (dist^2, id) and writes
//           it; K-NN rows (and radius rows longer than the LDS buffer) keep a
//           sorted top-M in LDS, shrink the bound to the M-th distance once M
//           are held and stop at the first table entry whose key exceeds it
//           (Section II.A, K nearest).
// Queries whose radius exceeds the tables' cap or the cyclic limit, or whose
// centre is outside the region, and every query of the cube method, scan the
// bin-lattice bounding cube instead (Section I; Section III.C).
#include "sphidx_internal.h"

namespace {

constexpr uint32_t kMaxId = 0xFFFFFFFFu;
constexpr uint64_t kMaxD2 = ~0ull;

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
// LDS ordering point for one wavefront (its LDS operations execute in order;
// this keeps the compiler from moving them across the point).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const uint32_t l = lane_id();
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d);
        if (l >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (uint32_t d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
    return uni(v);
}

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

// Exact u32 quotient (a < 2^31, 1 <= b < 2^31) from a double reciprocal and
// one correction step.
__device__ __forceinline__ uint32_t small_div(uint32_t a, uint32_t b, double inv_b) {
    uint32_t q = (uint32_t)((double)a * inv_b);
    if ((uint64_t)q * b > a) --q;
    if ((uint64_t)(q + 1) * b <= a) ++q;
    return q;
}

struct QState {
    uint32_t row;    // output row
    uint32_t self;   // sorted position excluded (EXCLUDE_SELF, all agents) or ~0
    uint32_t q[3];   // normalised centre
    uint32_t r;      // radius or K-NN cap
    uint64_t r2;
    uint32_t k;      // K for K-NN rows
    bool knn;
    bool valid;
    bool sphere;
    bool outside;    // objects of the outside cell may be within r
    // sphere walk
    uint32_t c[3];   // home cell
    uint32_t f[3];   // position inside the home cell
    uint32_t tb;     // first entry of the class table
    uint32_t tend;   // prefix length
    // bounding cube
    int32_t lo[3];
    uint32_t nn[3];
    uint32_t ncube;
    double inv_nx, inv_nxy;
};

__device__ __forceinline__ uint32_t pack_cell(const LatArgs& L, uint32_t x, uint32_t y, uint32_t z) {
    return (z << (L.lg[0] + L.lg[1])) | (y << L.lg[0]) | x;
}

__device__ void setup_query(const LatArgs& L, const TabArgs& T, const QArgs& A, uint32_t qi, QState& s) {
    uint32_t v[3];
    s.valid = true;
    if (A.qx == nullptr) {
        s.row = uni(L.ids[qi]);
        s.self = (A.flags & SPHIDX_EXCLUDE_SELF) ? qi : kMaxId;
        v[0] = uni(L.xs[qi]);
        v[1] = uni(L.ys[qi]);
        v[2] = uni(L.zs[qi]);
        // objects left out by the build (clipped coordinate >= 2^30) sit
        // after the outside cell; their rows stay empty
        s.valid = qi < uni(L.cs[L.ncells + 1]);
    } else {
        s.row = qi;
        s.self = kMaxId;
        v[0] = uni(A.qx[qi]);
        v[1] = uni(A.qy[qi]);
        v[2] = uni(A.qz[qi]);
        for (int a = 0; a < 3; ++a) {
            if ((L.cyc >> a) & 1u)
                v[a] &= (1u << (L.lg[a] + L.F)) - 1u;
            else if (v[a] >= (1u << 30))
                s.valid = false;
        }
        if (!s.valid) atomicOr(L.status, SPHIDX_FLAG_RANGE);
    }
    s.r = A.rad ? uni(A.rad[s.row]) : A.rad_u;
    s.r2 = (uint64_t)s.r * (uint64_t)s.r;
    uint32_t kk = A.kk ? uni(A.kk[s.row]) : A.k_u;
    s.knn = (A.mode == SPHIDX_MODE_KNN) || (A.mode == SPHIDX_MODE_MIXED && kk > 0);
    s.k = kk;
    if (s.knn && kk == 0) s.valid = false;
    const uint32_t e = 1u << L.F;
    bool inside = true, cyc_ok = true;
    s.outside = false;
    s.ncube = 1;
    for (int a = 0; a < 3; ++a) {
        s.q[a] = v[a];
        const uint32_t La = 1u << L.lg[a];
        const bool cyc = (L.cyc >> a) & 1u;
        // bounding cube along a: cells floor((q-r)/e) .. floor((q+r)/e)
        int64_t lo = ((int64_t)v[a] - (int64_t)s.r) >> L.F;
        int64_t hi = ((int64_t)v[a] + (int64_t)s.r) >> L.F;
        if (cyc) {
            if (hi - lo + 1 >= (int64_t)La) {
                lo = 0;
                hi = La - 1;
            }
            // limit of the sphere walk: ceil(r/e) <= L/2 - 1 (no offset repeats a cell)
            uint64_t lim = La >= 2 ? (uint64_t)(La / 2 - 1) * e : 0;
            if (La < 4 || (uint64_t)s.r > lim) cyc_ok = false;
        } else {
            if (hi >= (int64_t)La) s.outside = true;
            if (lo < 0) lo = 0;
            if (hi > (int64_t)La - 1) hi = (int64_t)La - 1;
            if (v[a] >= (La << L.F)) inside = false;
        }
        s.lo[a] = (int32_t)lo;
        s.nn[a] = hi >= lo ? (uint32_t)(hi - lo + 1) : 0u;
        s.ncube *= s.nn[a];
        s.c[a] = v[a] >> L.F;
        s.f[a] = v[a] & (e - 1u);
    }
    s.inv_nx = s.nn[0] ? 1.0 / (double)s.nn[0] : 0.0;
    s.inv_nxy = (s.nn[0] * s.nn[1]) ? 1.0 / (double)(s.nn[0] * s.nn[1]) : 0.0;
    s.sphere = (A.method == SPHIDX_METHOD_SPHERE) && T.has && inside && cyc_ok && s.r <= T.rmax;
    if (A.method == SPHIDX_METHOD_SPHERE && !s.sphere && s.valid) atomicOr(L.status, SPHIDX_FLAG_FALLBACK);
    s.tb = 0;
    s.tend = 0;
    if (s.sphere) {
        uint32_t cls = 0;
        for (int a = 0; a < 3; ++a) cls |= (s.f[a] >> (L.F - T.s)) << (a * T.s);
        s.tb = uni(T.cstart[cls]);
        uint32_t j = (uint32_t)(((uint64_t)s.r + (1u << T.rshift) - 1u) >> T.rshift);
        s.tend = uni(T.rindex[(size_t)cls * T.nr + j]);
    }
}

// Per-axis distances from the query (position f inside its cell) to the
// nearest and farthest positions of the cell at offset o along that axis.
__device__ __forceinline__ void axis_gap(int o, uint32_t f, uint32_t F, uint32_t& gmin, uint32_t& gmax) {
    const uint32_t e = 1u << F;
    if (o > 0) {
        gmin = ((uint32_t)o << F) - f;
        gmax = gmin + e - 1u;
    } else if (o < 0) {
        uint32_t a = (uint32_t)(-o);
        gmin = f + ((a - 1u) << F) + 1u;
        gmax = f + (a << F);
    } else {
        gmin = 0u;
        gmax = max(f, e - 1u - f);
    }
}

__device__ __forceinline__ uint64_t sq(uint32_t g) { return (uint64_t)g * (uint64_t)g; }

// One cell of the query's list.  `kept`: the cell is in the region and must
// be scanned; `interior`: every position of the cell is within r.
struct CellRef {
    uint32_t cell;
    bool kept;
    bool interior;
};

__device__ __forceinline__ CellRef sphere_entry(const LatArgs& L, const TabArgs& T, const uint32_t* tab_lds,
                                                const QState& s, uint32_t e, uint64_t bound2) {
    CellRef c;
    uint32_t w = tab_lds ? tab_lds[s.tb + e] : T.off[s.tb + e];
    int o[3];
    o[0] = ((int)(w << 22)) >> 22;
    o[1] = ((int)(w << 12)) >> 22;
    o[2] = ((int)(w << 2)) >> 22;
    uint64_t mind2 = 0, maxd2 = 0;
    bool in = true;
    uint32_t t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        uint32_t gmin, gmax;
        axis_gap(o[a], s.f[a], L.F, gmin, gmax);
        mind2 += sq(gmin);
        maxd2 += sq(gmax);
        int ta = (int)s.c[a] + o[a];
        const uint32_t La = 1u << L.lg[a];
        if ((L.cyc >> a) & 1u)
            t[a] = (uint32_t)ta & (La - 1u);
        else {
            in = in && (uint32_t)ta < La;
            t[a] = (uint32_t)ta;
        }
    }
    c.kept = in && mind2 <= bound2;
    c.interior = maxd2 <= s.r2;
    c.cell = c.kept ? pack_cell(L, t[0], t[1], t[2]) : 0u;
    return c;
}

__device__ __forceinline__ CellRef cube_entry(const LatArgs& L, const QState& s, uint32_t e) {
    CellRef c;
    uint32_t iz = small_div(e, s.nn[0] * s.nn[1], s.inv_nxy);
    uint32_t rem = e - iz * s.nn[0] * s.nn[1];
    uint32_t iy = small_div(rem, s.nn[0], s.inv_nx);
    uint32_t ix = rem - iy * s.nn[0];
    uint32_t i3[3] = {ix, iy, iz};
    uint32_t t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        uint32_t ta = (uint32_t)(s.lo[a] + (int32_t)i3[a]);
        if ((L.cyc >> a) & 1u) ta &= (1u << L.lg[a]) - 1u;
        t[a] = ta;
    }
    c.kept = true;
    c.interior = false;
    c.cell = pack_cell(L, t[0], t[1], t[2]);
    return c;
}

// Minimum-image squared distance between a stored object and the centre.
struct AxisWrap {
    uint32_t half[3];
    uint32_t mask[3];
};

__device__ __forceinline__ uint64_t obj_dist2(const LatArgs& L, const AxisWrap& w, const QState& s, uint32_t p) {
    uint32_t pv[3] = {L.xs[p], L.ys[p], L.zs[p]};
    uint64_t d2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int32_t dd = (int32_t)(((pv[a] - s.q[a]) + w.half[a]) & w.mask[a]) - (int32_t)w.half[a];
        uint32_t ad = (uint32_t)(dd < 0 ? -dd : dd);
        d2 += sq(ad);
    }
    return d2;
}

// Per-wave LDS layout of the write pass.
struct WaveLds {
    uint64_t* td;
    uint64_t* ud;
    uint64_t* bd;
    uint32_t* ti;
    uint32_t* ui;
    uint32_t* bi;
};

__host__ __device__ constexpr size_t wave_lds_bytes(uint32_t cap) { return (size_t)cap * 24 + 64 * 12; }

__device__ __forceinline__ WaveLds wave_lds(char* base, uint32_t cap) {
    WaveLds w;
    w.td = (uint64_t*)base;
    w.ud = w.td + cap;
    w.bd = w.ud + cap;
    w.ti = (uint32_t*)(w.bd + 64);
    w.ui = w.ti + cap;
    w.bi = w.ui + cap;
    return w;
}

// Candidate visitor modes.
enum { V_COUNT = 0, V_APPEND = 1, V_TOPM = 2 };

struct Walk {
    // pass-0 accumulators
    uint32_t hits;        // uniform
    uint32_t interior;    // per lane
    uint32_t kept;        // per lane (stats)
    uint32_t cand;        // uniform (stats)
    uint32_t walked;      // uniform (stats)
    bool stop;            // uniform: K-NN count reached K
    // append mode
    uint32_t n;           // uniform: collected so far
    // top-M mode
    uint32_t m, M;        // uniform
    uint64_t bd;          // uniform bound (d2, id) once m == M
    uint32_t bi;
    bool has_lower;
    uint64_t ld;
    uint32_t li;
};

// Visit the objects of the cells held by the lanes (one cell range per lane).
template <int MODE>
__device__ __forceinline__ void visit_candidates(const LatArgs& L, const AxisWrap& aw, const QState& s,
                                                 uint32_t start, uint32_t cnt, Walk& wk, WaveLds& lds,
                                                 uint32_t cap) {
    const uint32_t lane = lane_id();
    uint32_t incl = wave_incl_scan(cnt);
    uint32_t total = lane_val(incl, 63);
    wk.cand += total;
    uint32_t smx = start - (incl - cnt);
    for (uint32_t cb = 0; cb < total; cb += 64) {
        uint32_t g = cb + lane;
        // owner lane: number of lanes whose inclusive count is <= g
        uint32_t pos = 0;
#pragma unroll
        for (uint32_t st = 32; st >= 1; st >>= 1) {
            uint32_t v = bperm(incl, pos + st - 1);
            if (v <= g) pos += st;
        }
        uint32_t p = bperm(smx, pos) + g;
        bool act = g < total;
        uint64_t d2 = kMaxD2;
        if (act) d2 = obj_dist2(L, aw, s, p);
        if (MODE == V_COUNT) {
            bool hit = act && d2 <= s.r2 && p != s.self;
            uint64_t hm = __ballot(hit);
            wk.hits += (uint32_t)__popcll(hm);
            if (s.knn && wk.hits >= s.k) {
                wk.stop = true;
                return;
            }
        } else if (MODE == V_APPEND) {
            bool hit = act && d2 <= s.r2 && p != s.self;
            uint64_t hm = __ballot(hit);
            if (hit) {
                uint32_t slot = wk.n + lanes_below(hm);
                if (slot < cap) {
                    lds.td[slot] = d2;
                    lds.ti[slot] = L.ids[p];
                }
            }
            wk.n += (uint32_t)__popcll(hm);
        } else {
            bool c = act && d2 <= s.r2 && p != s.self;
            uint32_t id = kMaxId;
            if (c) {
                id = L.ids[p];
                if (wk.has_lower) c = key_less(wk.ld, wk.li, d2, id);
                if (c && wk.m == wk.M) c = key_less(d2, id, wk.bd, wk.bi);
            }
            uint64_t bm = __ballot(c);
            if (bm == 0) continue;
            uint32_t nb = (uint32_t)__popcll(bm);
            uint64_t cd = c ? d2 : kMaxD2;
            uint32_t ci = c ? id : kMaxId;
            wave_sort64(cd, ci);
            lds.bd[lane] = cd;
            lds.bi[lane] = ci;
            wave_sync();
            const uint32_t m = wk.m;
            const uint32_t nm = min(wk.M, m + nb);
            for (uint32_t t = lane; t < m; t += 64) {
                uint64_t xd = lds.td[t];
                uint32_t xi = lds.ti[t];
                uint32_t lo = 0, hi = nb;
                while (lo < hi) {
                    uint32_t mid = (lo + hi) >> 1;
                    if (key_less(lds.bd[mid], lds.bi[mid], xd, xi))
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                uint32_t dst = t + lo;
                if (dst < nm) {
                    lds.ud[dst] = xd;
                    lds.ui[dst] = xi;
                }
            }
            if (lane < nb) {
                uint32_t lo = 0, hi = m;
                while (lo < hi) {
                    uint32_t mid = (lo + hi) >> 1;
                    if (key_less(lds.td[mid], lds.ti[mid], cd, ci))
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                uint32_t dst = lane + lo;
                if (dst < nm) {
                    lds.ud[dst] = cd;
                    lds.ui[dst] = ci;
                }
            }
            wave_sync();
            uint64_t* sd = lds.td;
            lds.td = lds.ud;
            lds.ud = sd;
            uint32_t* si = lds.ti;
            lds.ti = lds.ui;
            lds.ui = si;
            wk.m = nm;
            if (nm == wk.M) {
                wk.bd = uni64(lds.td[nm - 1]);
                wk.bi = uni(lds.ti[nm - 1]);
            }
        }
    }
}

// Walk the query's cell list (outside cell first, then table entries or cube
// cells) and feed the candidates to the visitor.
template <int MODE>
__device__ void walk(const LatArgs& L, const TabArgs& T, const uint32_t* tab_lds, const AxisWrap& aw,
                     const QState& s, Walk& wk, WaveLds& lds, uint32_t cap, bool use_interior) {
    const uint32_t lane = lane_id();
    if (s.outside) {
        uint32_t st = 0, cnt = 0;
        if (lane == 0) {
            st = L.cs[L.ncells];
            cnt = L.cs[L.ncells + 1] - st;
        }
        visit_candidates<MODE>(L, aw, s, st, cnt, wk, lds, cap);
        if (wk.stop) return;
    }
    const uint32_t nent = s.sphere ? s.tend : s.ncube;
    for (uint32_t base = 0; base < nent; base += 64) {
        uint64_t bound2 = s.r2;
        if (MODE == V_TOPM && wk.m == wk.M) {
            bound2 = wk.bd;
            // entries are sorted by key: none further can hold a closer object
            if (s.sphere && uni64((uint64_t)T.key[s.tb + base]) > bound2) break;
        }
        uint32_t e = base + lane;
        CellRef c;
        c.kept = false;
        c.interior = false;
        c.cell = 0;
        if (e < nent) c = s.sphere ? sphere_entry(L, T, tab_lds, s, e, bound2) : cube_entry(L, s, e);
        wk.walked += min(64u, nent - base);
        uint32_t st = 0, cnt = 0;
        if (c.kept) {
            st = L.cs[c.cell];
            cnt = L.cs[c.cell + 1] - st;
            wk.kept += 1;
        }
        if (use_interior && c.kept && c.interior && s.sphere) {
            wk.interior += cnt;
            // the query's own object is inside its own (interior) cell only
            // when that cell is the home cell; exclusion handled by caller
            cnt = 0;
        }
        visit_candidates<MODE>(L, aw, s, st, cnt, wk, lds, cap);
        if (wk.stop) return;
    }
}

__device__ __forceinline__ AxisWrap axis_wrap(const LatArgs& L) {
    AxisWrap w;
    for (int a = 0; a < 3; ++a) {
        if ((L.cyc >> a) & 1u) {
            uint32_t W = 1u << (L.lg[a] + L.F);
            w.half[a] = W >> 1;
            w.mask[a] = W - 1u;
        } else {
            w.half[a] = 0u;
            w.mask[a] = 0xFFFFFFFFu;
        }
    }
    return w;
}

// Pass 0: row sizes.
__device__ void count_query(const LatArgs& L, const TabArgs& T, const uint32_t* tab_lds, const QArgs& A,
                            uint32_t qi) {
    QState s;
    setup_query(L, T, A, qi, s);
    const AxisWrap aw = axis_wrap(L);
    Walk wk = {};
    WaveLds lds = {};
    uint32_t total = 0;
    if (s.valid) {
        walk<V_COUNT>(L, T, tab_lds, aw, s, wk, lds, 0, !s.knn);
        total = wk.hits + wave_sum(wk.interior);
        // interior cells were counted whole, including the query's own object
        if (!s.knn && s.self != kMaxId) {
            // the self object is in the home cell; if that cell was counted as
            // interior it was not excluded by the candidate test
            bool home_interior = false;
            if (s.sphere) {
                uint32_t e = L.F;
                uint64_t mx = 0;
                for (int a = 0; a < 3; ++a) {
                    uint32_t f = s.f[a];
                    uint32_t g = max(f, (1u << e) - 1u - f);
                    mx += sq(g);
                }
                home_interior = mx <= s.r2;
            }
            if (home_interior) total -= 1;
        }
        if (s.knn && total > s.k) total = s.k;
    }
    if (lane_id() == 0) {
        A.row_ptr[s.row] = (int64_t)total;
        if (A.stats) {
            uint32_t* st = A.stats + 4 * (size_t)s.row;
            st[0] = wk.walked;
            st[3] = s.ncube;
        }
    }
    if (A.stats) {
        uint32_t kept = wave_sum(wk.kept);
        if (lane_id() == 0) {
            uint32_t* st = A.stats + 4 * (size_t)s.row;
            st[1] = kept;
            st[2] = wk.cand;
        }
    }
}

// Write `n` sorted (d2, id) pairs from LDS td/ti to the row at `dst`.
__device__ __forceinline__ void emit(const QArgs& A, const WaveLds& lds, uint32_t n, int64_t dst) {
    for (uint32_t t = lane_id(); t < n; t += 64) {
        A.out_ids[dst + t] = lds.ti[t];
        if (A.out_d2) A.out_d2[dst + t] = (int64_t)lds.td[t];
    }
}

// Pass 1: row contents.
__device__ void write_query(const LatArgs& L, const TabArgs& T, const uint32_t* tab_lds, const QArgs& A,
                            uint32_t qi, char* lds_base) {
    QState s;
    setup_query(L, T, A, qi, s);
    const int64_t rb = A.row_ptr[s.row];
    const uint32_t rowlen = (uint32_t)(A.row_ptr[s.row + 1] - rb);
    if (!s.valid || rowlen == 0) return;
    const AxisWrap aw = axis_wrap(L);
    const uint32_t cap = A.sort_cap;
    WaveLds lds = wave_lds(lds_base, cap);
    const uint32_t lane = lane_id();
    if (!s.knn && rowlen <= cap) {
        Walk wk = {};
        walk<V_APPEND>(L, T, tab_lds, aw, s, wk, lds, cap, false);
        wave_sync();
        const uint32_t n = min(wk.n, rowlen);
        if (n <= 64) {
            // rank sort: lane i holds pair i, its rank is the number of smaller pairs
            uint64_t d = kMaxD2;
            uint32_t id = kMaxId;
            if (lane < n) {
                d = lds.td[lane];
                id = lds.ti[lane];
            }
            uint32_t rank = 0;
            for (uint32_t j = 0; j < n; ++j) {
                uint64_t dj = ((uint64_t)lane_val((uint32_t)(d >> 32), j) << 32) | lane_val((uint32_t)d, j);
                uint32_t ij = lane_val(id, j);
                rank += key_less(dj, ij, d, id) ? 1u : 0u;
            }
            if (lane < n) {
                A.out_ids[rb + rank] = id;
                if (A.out_d2) A.out_d2[rb + rank] = (int64_t)d;
            }
        } else {
            uint32_t np = 64;
            while (np < n) np <<= 1;
            for (uint32_t t = n + lane; t < np; t += 64) {
                lds.td[t] = kMaxD2;
                lds.ti[t] = kMaxId;
            }
            wave_sync();
            for (uint32_t k = 2; k <= np; k <<= 1) {
                for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                    for (uint32_t t = lane; t < (np >> 1); t += 64) {
                        uint32_t i = ((t & ~(j - 1u)) << 1) | (t & (j - 1u));
                        uint32_t pj = i + j;
                        uint64_t di = lds.td[i], dp = lds.td[pj];
                        uint32_t ii = lds.ti[i], ip = lds.ti[pj];
                        bool up = (i & k) == 0;
                        bool sw = up ? key_less(dp, ip, di, ii) : key_less(di, ii, dp, ip);
                        if (sw) {
                            lds.td[i] = dp;
                            lds.td[pj] = di;
                            lds.ti[i] = ip;
                            lds.ti[pj] = ii;
                        }
                    }
                    wave_sync();
                }
            }
            emit(A, lds, n, rb);
        }
        return;
    }
    // top-M windows: K-NN rows, and radius rows longer than the LDS buffer
    Walk wk = {};
    uint32_t written = 0;
    while (written < rowlen) {
        wk.M = min(cap, rowlen - written);
        wk.m = 0;
        wk.bd = kMaxD2;
        wk.bi = kMaxId;
        walk<V_TOPM>(L, T, tab_lds, aw, s, wk, lds, cap, false);
        wave_sync();
        const uint32_t got = min(wk.m, wk.M);
        emit(A, lds, got, rb + written);
        if (got == 0) break;
        wk.has_lower = true;
        wk.ld = uni64(lds.td[got - 1]);
        wk.li = uni(lds.ti[got - 1]);
        written += got;
        wave_sync();
    }
}

template <int PASS>
__global__ __launch_bounds__(256) void query_kernel(LatArgs L, TabArgs T, QArgs A) {
    extern __shared__ __align__(16) char smem[];
    const uint32_t wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t* tab_lds = nullptr;
    size_t tab_bytes = 0;
    if (T.lds) {
        // the whole offset table, shared by the block's waves
        uint32_t* t = (uint32_t*)smem;
        for (uint32_t i = threadIdx.x; i < T.total; i += blockDim.x) t[i] = T.off[i];
        __syncthreads();
        tab_lds = t;
        tab_bytes = ((size_t)T.total * 4 + 15) & ~(size_t)15;
    }
    char* lds_base = smem + tab_bytes + (PASS == 1 ? (size_t)wave * wave_lds_bytes(A.sort_cap) : 0);
    if (PASS == 1) {
        int64_t tot = A.row_ptr[A.Q];
        if (tot > A.capacity) {
            if (threadIdx.x == 0) atomicOr(L.status, SPHIDX_FLAG_CAPACITY);
            return;
        }
    }
    const uint32_t lane = lane_id();
    if (!A.persistent) {
        // XCD-aware order: consecutive block ids go round-robin over the 8
        // XCDs; give each XCD a contiguous range of query slices instead
        const uint32_t G = gridDim.x, b = blockIdx.x;
        const uint32_t full = G / SPHIDX_NQUEUE, rem = G % SPHIDX_NQUEUE;
        const uint32_t x = b % SPHIDX_NQUEUE, i = b / SPHIDX_NQUEUE;
        const uint32_t lb = x * full + min(x, rem) + i;
        const uint64_t q0 = ((uint64_t)lb * nw + wave) * A.tile;
        for (uint32_t t = 0; t < A.tile; ++t) {
            uint64_t qi = q0 + t;
            if (qi >= A.Q) break;
            if (PASS == 0)
                count_query(L, T, tab_lds, A, (uint32_t)qi);
            else
                write_query(L, T, tab_lds, A, (uint32_t)qi, lds_base);
        }
    } else {
        // persistent: one work queue per XCD over a contiguous range of the
        // queries; drain the own queue, then take from the others
        uint32_t x = blockIdx.x % SPHIDX_NQUEUE;
        uint32_t misses = 0;
        while (misses < SPHIDX_NQUEUE) {
            const uint32_t qs = (uint32_t)(((uint64_t)x * A.Q) / SPHIDX_NQUEUE);
            const uint32_t qe = (uint32_t)(((uint64_t)(x + 1) * A.Q) / SPHIDX_NQUEUE);
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(&A.queues[x], A.tile);
            t = uni(t);
            if ((uint64_t)qs + t >= qe) {
                x = (x + 1) % SPHIDX_NQUEUE;
                ++misses;
                continue;
            }
            misses = 0;
            const uint32_t end = (uint32_t)min((uint64_t)qe, (uint64_t)qs + t + A.tile);
            for (uint32_t qi = qs + t; qi < end; ++qi) {
                if (PASS == 0)
                    count_query(L, T, tab_lds, A, qi);
                else
                    write_query(L, T, tab_lds, A, qi, lds_base);
            }
        }
    }
}

}  // namespace

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

hipError_t launch_query_pass(int pass, const LatArgs& L, const TabArgs& T, const QArgs& q,
                             uint32_t waves_per_block, uint32_t blocks_per_cu, hipStream_t st) {
    if (q.Q == 0) return hipSuccess;
    const uint32_t threads = waves_per_block * 64;
    size_t shmem = 0;
    if (T.lds) shmem += ((size_t)T.total * 4 + 15) & ~(size_t)15;
    if (pass == 1) shmem += (size_t)waves_per_block * wave_lds_bytes(q.sort_cap);
    uint32_t blocks;
    if (q.persistent) {
        blocks = (uint32_t)device_cu_count() * blocks_per_cu;
        hipError_t e = launch_fill_u32(q.queues, 0u, SPHIDX_NQUEUE, st);
        if (e != hipSuccess) return e;
    } else {
        uint64_t per_block = (uint64_t)waves_per_block * q.tile;
        blocks = (uint32_t)((q.Q + per_block - 1) / per_block);
    }
    if (pass == 0)
        hipLaunchKernelGGL(query_kernel<0>, dim3(blocks), dim3(threads), shmem, st, L, T, q);
    else
        hipLaunchKernelGGL(query_kernel<1>, dim3(blocks), dim3(threads), shmem, st, L, T, q);
    return hipGetLastError();
}

size_t query_wave_lds_bytes(uint32_t cap) { return wave_lds_bytes(cap); }
