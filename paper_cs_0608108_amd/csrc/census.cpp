// Cells walked under the table designs of the paper, against the sub-cell
// class tables of this library and the exact set (host only).
//
// All lengths are in fixed-point units, a cell being e = 2^F units wide.  A
// query sits at (fx, fy, fz) inside its home cell (0 <= f < e) with radius r.
//
//   exact      cells holding a position within r: per axis the gap to cell
//              offset o is 0 for o = 0, (o - 1) e + (e - f) above and
//              (|o| - 1) e + f + 1 below (integer positions, as everywhere in
//              the library); kept iff the squared gaps sum to <= r^2.
//   cube       the bin-lattice bounding cube, exact to the sub-cell: offsets
//              floor((f - r) / e) .. floor((f + r) / e) per axis.
//   unshaved   the Section II.A table: per axis b_o = max(|o| - 1, 0) cells,
//              entry b^2 = sum b_o^2, walked while b^2 e^2 <= r^2 (b^2 <=
//              floor(d^2) with d = r / e).
//   paper 64   Section III.A: below floor(d)^2 the unshaved table; from
//              floor(d)^2 to floor(d^2) one of 64 specialised tables, chosen
//              by six bits [frac(d) < zeta] for the six directions (zeta: the
//              distance from the centre to its cell's face, e - f up and f
//              down, the paper's real-valued model).  In that range floor(d)
//              is floor(b) of the entry itself, so table m can leave out, ahead
//              of time, every cell that (the one-direction rule) has an axis
//              with b_o = floor(b) whose direction is flagged in m, or (Eq. 2)
//              moves along at least one axis with all its directions flagged.
//   paper 64 + Eq. 1
//              the same, then the run-time test of Eq. 1 on the cells at or
//              above d - 1: reject when sum (b_o e + zeta)^2 > r^2 over the
//              axes the cell moves along.
//   sub-cell   the library's tables: the prefix key <= r^2 of the query's
//              sub-cell class (s bits per axis).
//
// The paper's model places the lower face at f rather than f + 1, so its
// rejections are never wrong for integer positions: the exact set is a subset
// of every walked or kept set.  The census counts the exact cells a design
// would drop (it must be none).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sphidx_internal.h"

namespace {

struct UnshavedEntry {
    uint32_t b2;    // sum of squared per-axis cell gaps
    int8_t o[3];    // offset
};

// The unshaved table for offsets |o| <= m, sorted by b^2 (Section II.A).
std::vector<UnshavedEntry> unshaved_table(int m) {
    std::vector<UnshavedEntry> t;
    for (int oz = -m; oz <= m; ++oz)
        for (int oy = -m; oy <= m; ++oy)
            for (int ox = -m; ox <= m; ++ox) {
                const int o[3] = {ox, oy, oz};
                uint32_t b2 = 0;
                for (int a = 0; a < 3; ++a) {
                    const int b = std::max(std::abs(o[a]) - 1, 0);
                    b2 += (uint32_t)(b * b);
                }
                t.push_back({b2, {(int8_t)ox, (int8_t)oy, (int8_t)oz}});
            }
    std::stable_sort(t.begin(), t.end(), [](const UnshavedEntry& x, const UnshavedEntry& y) { return x.b2 < y.b2; });
    return t;
}

// Direction bit of axis a and sign s (0: up, 1: down) in a 6-bit table index.
inline uint32_t dir_bit(int a, int down) { return 1u << (2 * a + down); }

// The cell directions an offset moves along, as a 6-bit mask (0: the home cell).
inline uint32_t dirs_of(const int8_t* o) {
    uint32_t m = 0;
    for (int a = 0; a < 3; ++a)
        if (o[a] != 0) m |= dir_bit(a, o[a] < 0 ? 1 : 0);
    return m;
}

struct PaperTables {
    std::vector<UnshavedEntry> base;                 // sorted by b^2
    std::vector<std::vector<UnshavedEntry>> spec;    // 64 specialised tables, each sorted by b^2
};

// floor(sqrt(v)) for the small entries of the tables.
inline uint32_t isqrt32(uint32_t v) {
    uint32_t x = (uint32_t)std::sqrt((double)v);
    while (x * x > v) --x;
    while ((x + 1) * (x + 1) <= v) ++x;
    return x;
}

// Whether table t (six flags [frac(d) < zeta]) leaves out an entry that lies
// between floor(d)^2 and floor(d^2), where floor(d) = floor(b) (Section III.A):
// along one direction, the cell's gap on an axis with b_o = floor(d) already
// exceeds d when that direction is flagged; with every direction it moves
// along flagged, Eq. 2 exceeds Eq. 1's bound.
inline bool left_out(const UnshavedEntry& en, uint32_t t) {
    const uint32_t d = dirs_of(en.o);
    if (d != 0 && (d & t) == d) return true;
    const int D0 = (int)isqrt32(en.b2);
    for (int a = 0; a < 3; ++a)
        if (en.o[a] != 0 && std::abs(en.o[a]) - 1 == D0 && (t & dir_bit(a, en.o[a] < 0 ? 1 : 0))) return true;
    return false;
}

// Section III.A: the 64 specialised tables, each the unshaved entries that
// its flags do not leave out.
PaperTables paper_tables(int m) {
    PaperTables p;
    p.base = unshaved_table(m);
    p.spec.resize(64);
    for (uint32_t t = 0; t < 64; ++t)
        for (const UnshavedEntry& en : p.base)
            if (!left_out(en, t)) p.spec[t].push_back(en);
    return p;
}

// Entries of a b^2-sorted table with lo <= b^2 <= hi.
template <typename V>
size_t count_range(const V& t, uint64_t lo, uint64_t hi) {
    auto lb = std::lower_bound(t.begin(), t.end(), lo, [](const UnshavedEntry& e, uint64_t v) { return e.b2 < v; });
    auto ub = std::upper_bound(t.begin(), t.end(), hi, [](uint64_t v, const UnshavedEntry& e) { return v < e.b2; });
    return ub > lb ? (size_t)(ub - lb) : 0u;
}

inline uint64_t sq(uint64_t v) { return v * v; }

// Exact per-axis gap (integer positions) from position f of the home cell to
// cell offset o.
inline uint64_t exact_gap(int o, uint64_t f, uint64_t e) {
    if (o == 0) return 0;
    if (o > 0) return (uint64_t)(o - 1) * e + (e - f);
    return (uint64_t)(-o - 1) * e + f + 1;
}

// The paper's per-axis distance to cell offset o: b_o cells plus zeta.
inline uint64_t paper_gap(int o, uint64_t f, uint64_t e) {
    if (o == 0) return 0;
    if (o > 0) return (uint64_t)(o - 1) * e + (e - f);
    return (uint64_t)(-o - 1) * e + f;
}

}  // namespace

// The paper's tables laid out for the device (Section III.A): the 64
// specialised tables, then the unshaved table, each sorted by b^2, as
// packed offsets (10 bits per axis, two's complement) with their b^2;
// start[t] .. start[t + 1] is table t (t = 64: the unshaved table).
void paper_tables_flat(int m, std::vector<uint32_t>& off, std::vector<uint32_t>& b2,
                       std::vector<uint32_t>& start) {
    const PaperTables pt = paper_tables(m);
    off.clear();
    b2.clear();
    start.assign(66, 0);
    auto put = [&](const std::vector<UnshavedEntry>& tab) {
        for (const UnshavedEntry& en : tab) {
            off.push_back(((uint32_t)en.o[0] & 0x3FFu) | (((uint32_t)en.o[1] & 0x3FFu) << 10) |
                          (((uint32_t)en.o[2] & 0x3FFu) << 20));
            b2.push_back(en.b2);
        }
    };
    for (uint32_t t = 0; t < 64; ++t) {
        start[t] = (uint32_t)off.size();
        put(pt.spec[t]);
    }
    start[64] = (uint32_t)off.size();
    put(pt.base);
    start[65] = (uint32_t)off.size();
}

extern "C" {

sphidx_status sphidx_table_census(const sphidx_tables* tab, uint32_t nq, const uint32_t* fx_host,
                                  const uint32_t* fy_host, const uint32_t* fz_host, const uint32_t* r_host,
                                  uint64_t* out_host) {
    if (!tab || (nq && (!fx_host || !fy_host || !fz_host || !r_host || !out_host))) return SPHIDX_ERR_INVALID_ARG;
    const uint64_t e = 1ull << tab->F;
    uint32_t rmax = 0;
    for (uint32_t i = 0; i < nq; ++i) {
        if (fx_host[i] >= e || fy_host[i] >= e || fz_host[i] >= e) return SPHIDX_ERR_INVALID_ARG;
        rmax = std::max(rmax, r_host[i]);
    }
    if (rmax > tab->rmax_fx) return SPHIDX_ERR_RADIUS;
    const int m = (int)((rmax + e - 1) / e) + 1;
    if (m > 32) return SPHIDX_ERR_RADIUS;  // 65 tables of (2m + 1)^3 entries
    const PaperTables pt = paper_tables(m);
    for (uint32_t i = 0; i < nq; ++i) {
        const uint64_t f[3] = {fx_host[i], fy_host[i], fz_host[i]};
        const uint64_t r = r_host[i], r2 = r * r;
        uint64_t* out = out_host + 7 * (size_t)i;
        // cube
        uint64_t cube = 1;
        for (int a = 0; a < 3; ++a) {
            const int64_t lo = ((int64_t)f[a] - (int64_t)r) >> tab->F, hi = ((int64_t)f[a] + (int64_t)r) >> tab->F;
            cube *= (uint64_t)(hi - lo + 1);
        }
        // unshaved: b^2 e^2 <= r^2
        const uint64_t b2max = r2 / (e * e);
        const size_t unshaved = count_range(pt.base, 0, b2max);
        // paper 64: floor(d) and frac(d) in units
        const uint64_t D0 = r / e, fu = r - D0 * e;
        uint32_t t = 0;
        for (int a = 0; a < 3; ++a) {
            if (fu < e - f[a]) t |= dir_bit(a, 0);
            if (fu < f[a]) t |= dir_bit(a, 1);
        }
        const std::vector<UnshavedEntry>& spec = pt.spec[t];
        const uint64_t lo2 = D0 * D0;
        size_t walked = (lo2 > 0 ? count_range(pt.base, 0, lo2 - 1) : 0u) + count_range(spec, lo2, b2max);
        // Eq. 1 on the walked cells at or above d - 1, and the exact cells
        // each design would drop
        size_t rejected = 0, dropped = 0, exact = 0;
        auto eq1_rejects = [&](const UnshavedEntry& en) {
            // only at or above d - 1: b e >= r - e, squared when r >= e
            const bool test = r < e || (uint64_t)en.b2 * e * e >= sq(r - e);
            if (!test) return false;
            uint64_t t2 = 0;
            for (int a = 0; a < 3; ++a) t2 += sq(paper_gap(en.o[a], f[a], e));
            return t2 > r2;
        };
        for (const UnshavedEntry& en : pt.base) {
            if (en.b2 > b2max) break;
            uint64_t g2 = 0;
            for (int a = 0; a < 3; ++a) g2 += sq(exact_gap(en.o[a], f[a], e));
            const bool need = g2 <= r2;
            exact += need ? 1u : 0u;
            const bool in_walk = en.b2 < lo2 || !left_out(en, t);
            const bool rej = in_walk && eq1_rejects(en);
            rejected += rej ? 1u : 0u;
            if (need && (!in_walk || rej)) ++dropped;
        }
        // sub-cell class table prefix
        const uint32_t cls = (uint32_t)((f[0] >> (tab->F - tab->s)) | ((f[1] >> (tab->F - tab->s)) << tab->s) |
                                        ((f[2] >> (tab->F - tab->s)) << (2 * tab->s)));
        const int64_t* kb = tab->h_key.data() + tab->h_class_start[cls];
        const int64_t* ke = tab->h_key.data() + tab->h_class_start[cls + 1];
        const size_t sub = (size_t)(std::upper_bound(kb, ke, (int64_t)r2) - kb);
        out[0] = cube;
        out[1] = unshaved;
        out[2] = walked;
        out[3] = walked - rejected;
        out[4] = sub;
        out[5] = exact;
        out[6] = dropped;
    }
    return SPHIDX_OK;
}

sphidx_status sphidx_table_census_nd(uint32_t dims, uint32_t frac_bits, uint32_t subcell_bits, uint32_t r_fx,
                                     double* sphere_cells, double* cube_cells, uint64_t* unshaved_hist,
                                     uint32_t hist_len) {
    if (dims < 2 || dims > 4 || subcell_bits > 3 || subcell_bits > frac_bits || frac_bits > 20)
        return SPHIDX_ERR_INVALID_ARG;
    if (!sphere_cells || !cube_cells || (hist_len && !unshaved_hist)) return SPHIDX_ERR_INVALID_ARG;
    const uint64_t e = 1ull << frac_bits, w = 1ull << (frac_bits - subcell_bits);
    const uint64_t r = r_fx, r2 = r * r;
    const int m = (int)((r + e - 1) / e) + 1;
    const uint64_t side = 2 * (uint64_t)m + 1;
    uint64_t offsets = 1, classes = 1;
    for (uint32_t a = 0; a < dims; ++a) {
        offsets *= side;
        classes <<= subcell_bits;
    }
    if (offsets * classes > (1ull << 34)) return SPHIDX_ERR_RADIUS;
    // per class along one axis: squared gaps of every offset from the class
    // box [c w, (c + 1) w - 1] (the smallest over the box), and the offsets of
    // the bounding interval (gap <= r)
    const uint32_t nsub = 1u << subcell_bits;
    std::vector<uint64_t> g2((size_t)nsub * side);
    std::vector<uint64_t> span(nsub, 0);
    for (uint32_t c = 0; c < nsub; ++c)
        for (int o = -m; o <= m; ++o) {
            uint64_t g = 0;
            if (o > 0) g = (uint64_t)o * e - ((c + 1) * w - 1);
            if (o < 0) g = c * w + (uint64_t)(-o - 1) * e + 1;
            g2[(size_t)c * side + (o + m)] = g * g;
            if (g * g <= r2) ++span[c];
        }
    double s_sum = 0, c_sum = 0;
    std::vector<uint32_t> cls(dims, 0), idx(dims, 0);
    for (uint64_t k = 0; k < classes; ++k) {
        uint64_t kk = k, box = 1;
        for (uint32_t a = 0; a < dims; ++a) {
            cls[a] = (uint32_t)(kk % nsub);
            kk /= nsub;
            box *= span[cls[a]];
        }
        uint64_t inside = 0;
        for (uint64_t p = 0; p < offsets; ++p) {
            uint64_t pp = p, sum = 0;
            for (uint32_t a = 0; a < dims && sum <= r2; ++a) {
                sum += g2[(size_t)cls[a] * side + (pp % side)];
                pp /= side;
            }
            inside += sum <= r2 ? 1u : 0u;
        }
        s_sum += (double)inside;
        c_sum += (double)box;
    }
    *sphere_cells = s_sum / (double)classes;
    *cube_cells = c_sum / (double)classes;
    if (hist_len) {
        // the unshaved table (Section II.A) in `dims` dimensions: offsets per
        // entry b^2 < hist_len
        std::fill(unshaved_hist, unshaved_hist + hist_len, 0ull);
        const int mh = (int)std::ceil(std::sqrt((double)hist_len)) + 1;
        const uint64_t sh = 2 * (uint64_t)mh + 1;
        uint64_t n = 1;
        for (uint32_t a = 0; a < dims; ++a) n *= sh;
        for (uint64_t p = 0; p < n; ++p) {
            uint64_t pp = p, b2 = 0;
            for (uint32_t a = 0; a < dims; ++a) {
                const int o = (int)(pp % sh) - mh;
                pp /= sh;
                const uint64_t b = (uint64_t)std::max(std::abs(o) - 1, 0);
                b2 += b * b;
            }
            if (b2 < hist_len) ++unshaved_hist[b2];
        }
    }
    return SPHIDX_OK;
}

}  // extern "C"
