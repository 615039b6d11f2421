// Sphere tables (Section II.A, sorted cell-offset array with a radius index;
// Section III.A, tables specialised on the query's sub-cell position).
//
// For sub-cell class c (s bits per axis: the query lies in the box of
// positions [c*w, (c+1)*w - 1] of its cell along each axis, w = 2^(F-s)),
// the key of cell offset o is the smallest squared distance between a
// position of that box and a position of cell o.  The distance separates
// over the axes and the box is a product, so the key is the sum over axes of
// the squared per-axis minimum gap:
//   o > 0: first position of cell o minus the box's last position
//   o < 0: box's first position minus the last position of cell o
//   o = 0: 0.
// A query of radius r in class c needs exactly the entries with key <= r^2;
// no other cell can hold an object within r.  Entries are sorted by key, so
// they run from the centre to the edge (Section II.A).  The radius index
// gives, per class and radius bucket j (bucket width 2^rshift units), the
// number of entries with key <= (j * 2^rshift)^2: an upper bound of the
// prefix that a single lookup returns (the paper indexes by floor(d^2)).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "sphidx_internal.h"

namespace {

const char kMagic[8] = {'S', 'P', 'H', 'I', 'D', 'X', 'T', '1'};
const uint32_t kVersion = 1;

uint32_t pack_offset(int ox, int oy, int oz) {
    return ((uint32_t)ox & 0x3FFu) | (((uint32_t)oy & 0x3FFu) << 10) | (((uint32_t)oz & 0x3FFu) << 20);
}

// FNV-1a, 64-bit.
uint64_t fnv1a(const void* data, size_t n, uint64_t h) {
    const unsigned char* p = (const unsigned char*)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

}  // namespace

// Copy the row table, and the full table's radius index (the cell counts
// the method choice compares), to device memory (once).
sphidx_status tables_upload(sphidx_tables* t) {
    if (t->d_rows) return SPHIDX_OK;
    t->device_bytes = 0;
    auto put = [&](void** dst, const void* src, size_t bytes) -> bool {
        size_t b = bytes ? bytes : 4;
        if (hipMalloc(dst, b) != hipSuccess) return false;
        t->device_bytes += b;
        if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return false;
        return true;
    };
    bool ok = put((void**)&t->d_rows, t->h_rows.data(), t->h_rows.size() * 4) &&
              put((void**)&t->d_rkey, t->h_rkey.data(), t->h_rkey.size() * 8) &&
              put((void**)&t->d_rclass_start, t->h_rclass_start.data(), t->h_rclass_start.size() * 4) &&
              put((void**)&t->d_rrindex, t->h_rrindex.data(), t->h_rrindex.size() * 4) &&
              put((void**)&t->d_vcount, t->h_rindex.data(), t->h_rindex.size() * 4);
    if (ok && t->pm)
        ok = put((void**)&t->d_poff, t->h_poff.data(), t->h_poff.size() * 4) &&
             put((void**)&t->d_pb2, t->h_pb2.data(), t->h_pb2.size() * 4) &&
             put((void**)&t->d_plo, t->h_plo.data(), t->h_plo.size() * 4);
    return ok ? SPHIDX_OK : SPHIDX_ERR_OUT_OF_MEMORY;
}

namespace {

void free_device(sphidx_tables* t) {
    if (t->d_rows) (void)hipFree(t->d_rows);
    if (t->d_rkey) (void)hipFree(t->d_rkey);
    if (t->d_rclass_start) (void)hipFree(t->d_rclass_start);
    if (t->d_rrindex) (void)hipFree(t->d_rrindex);
    if (t->d_vcount) (void)hipFree(t->d_vcount);
    if (t->d_poff) (void)hipFree(t->d_poff);
    if (t->d_pb2) (void)hipFree(t->d_pb2);
    if (t->d_plo) (void)hipFree(t->d_plo);
    t->d_poff = t->d_pb2 = t->d_plo = nullptr;
    t->d_vcount = nullptr;
    t->d_rows = nullptr;
    t->d_rkey = nullptr;
    t->d_rclass_start = nullptr;
    t->d_rrindex = nullptr;
}

}  // namespace

// Row table.  The packed cell index puts the cells of one x-row next to
// each other, so their objects are one contiguous range (Section II.B).  A
// query meets, in row (oy, oz), exactly the cells whose x-gap satisfies
// gx^2 <= r^2 - gy^2 - gz^2: a contiguous run found per query.  The table
// therefore lists rows instead of cells: for (y, z) sub-cell class (cy, cz)
// every row whose key -- the smallest gy^2 + gz^2 over the class box -- is
// <= rmax^2, sorted by key (centre to edge), with the same radius index.
void tables_build_rows(sphidx_tables* t) {
    const int64_t e = (int64_t)1 << t->F, w = (int64_t)1 << (t->F - t->s);
    const int m = (int)(((int64_t)t->rmax_fx + e - 1) / e) + 1;
    const uint64_t r2 = (uint64_t)t->rmax_fx * (uint64_t)t->rmax_fx;
    const uint32_t nsub = 1u << t->s;
    t->nrclasses = nsub * nsub;
    t->h_rows.clear();
    t->h_rkey.clear();
    t->h_rclass_start.assign(t->nrclasses + 1, 0);
    t->h_rrindex.assign((size_t)t->nrclasses * t->nr, 0);
    auto gap2 = [&](int64_t c, int o) -> uint64_t {
        int64_t g = 0;
        if (o > 0)
            g = (int64_t)o * e - ((c + 1) * w - 1);
        else if (o < 0)
            g = c * w + ((int64_t)(-o) - 1) * e + 1;
        return (uint64_t)(g * g);
    };
    struct Row {
        uint64_t key;
        uint32_t packed;
    };
    std::vector<Row> rows;
    for (uint32_t cls = 0; cls < t->nrclasses; ++cls) {
        const int64_t cy = cls & (nsub - 1), cz = cls >> t->s;
        rows.clear();
        for (int oz = -m; oz <= m; ++oz)
            for (int oy = -m; oy <= m; ++oy) {
                const uint64_t k = gap2(cy, oy) + gap2(cz, oz);
                if (k <= r2) rows.push_back({k, ((uint32_t)oy & 0xFFFFu) | ((uint32_t)oz << 16)});
            }
        std::sort(rows.begin(), rows.end(), [](const Row& x, const Row& y) {
            return x.key < y.key || (x.key == y.key && x.packed < y.packed);
        });
        t->h_rclass_start[cls] = (uint32_t)t->h_rows.size();
        for (const Row& r : rows) {
            t->h_rows.push_back(r.packed);
            t->h_rkey.push_back((int64_t)r.key);
        }
        size_t p = 0;
        for (uint32_t j = 0; j < t->nr; ++j) {
            const uint64_t rj = (uint64_t)j << t->rshift;
            while (p < rows.size() && rows[p].key <= rj * rj) ++p;
            t->h_rrindex[(size_t)cls * t->nr + j] = (uint32_t)p;
        }
    }
    t->h_rclass_start[t->nrclasses] = (uint32_t)t->h_rows.size();
}

// The paper's 64 specialised tables and the unshaved table (Section III.A)
// for offsets up to m = ceil(rmax / e) + 1 cells, with the per-table b^2
// index the query set-up reads; left unbuilt (pm = 0) beyond kPaperMaxOff.
void tables_build_paper(sphidx_tables* t) {
    const uint64_t e = 1ull << t->F;
    const uint64_t m = ((uint64_t)t->rmax_fx + e - 1) / e + 1;
    t->pm = 0;
    t->h_poff.clear();
    t->h_pb2.clear();
    t->h_pstart.clear();
    t->h_plo.clear();
    if (m > kPaperMaxOff) return;
    paper_tables_flat((int)m, t->h_poff, t->h_pb2, t->h_pstart);
    t->pm = (uint32_t)m;
    t->pnb2 = 3u * (uint32_t)(m * m) + 2u;
    t->h_plo.assign((size_t)65 * t->pnb2, 0);
    for (uint32_t tb = 0; tb < 65; ++tb) {
        uint32_t p = t->h_pstart[tb];
        const uint32_t end = t->h_pstart[tb + 1];
        for (uint32_t v = 0; v < t->pnb2; ++v) {
            while (p < end && t->h_pb2[p] < v) ++p;
            t->h_plo[(size_t)tb * t->pnb2 + v] = p;
        }
    }
}

// Build on the host (validation of s / F / rmax is done by the caller).
sphidx_status tables_build_host(uint32_t F, uint32_t s, uint32_t rmax_fx, sphidx_tables* t) {
    const int64_t e = (int64_t)1 << F, w = (int64_t)1 << (F - s);
    const int m = (int)(((int64_t)rmax_fx + e - 1) / e) + 1;
    const uint64_t r2 = (uint64_t)rmax_fx * (uint64_t)rmax_fx;
    const uint32_t ncls = 1u << (3 * s);
    const uint32_t nsub = 1u << s;
    t->s = s;
    t->F = F;
    t->rmax_fx = rmax_fx;
    t->nclasses = ncls;
    t->rshift = F > 6 ? F - 6 : 0;
    t->nr = (rmax_fx >> t->rshift) + 2;
    t->max_off = 0;
    // per-axis squared gap, indexed by [class along axis][o + m]
    std::vector<uint64_t> g2((size_t)nsub * (2 * m + 1));
    for (uint32_t c = 0; c < nsub; ++c)
        for (int o = -m; o <= m; ++o) {
            int64_t g = 0;
            if (o > 0)
                g = (int64_t)o * e - ((int64_t)(c + 1) * w - 1);
            else if (o < 0)
                g = (int64_t)c * w + ((int64_t)(-o) - 1) * e + 1;
            g2[(size_t)c * (2 * m + 1) + (o + m)] = (uint64_t)(g * g);
        }
    t->h_class_start.assign(ncls + 1, 0);
    t->h_off.clear();
    t->h_key.clear();
    t->h_rindex.assign((size_t)ncls * t->nr, 0);
    struct Ent {
        uint64_t key;
        uint32_t off;
    };
    std::vector<Ent> ents;
    for (uint32_t cls = 0; cls < ncls; ++cls) {
        const uint32_t cx = cls & (nsub - 1), cy = (cls >> s) & (nsub - 1), cz = (cls >> (2 * s)) & (nsub - 1);
        const uint64_t* gx = &g2[(size_t)cx * (2 * m + 1)];
        const uint64_t* gy = &g2[(size_t)cy * (2 * m + 1)];
        const uint64_t* gz = &g2[(size_t)cz * (2 * m + 1)];
        ents.clear();
        for (int oz = -m; oz <= m; ++oz) {
            uint64_t kz = gz[oz + m];
            if (kz > r2) continue;
            for (int oy = -m; oy <= m; ++oy) {
                uint64_t kyz = kz + gy[oy + m];
                if (kyz > r2) continue;
                for (int ox = -m; ox <= m; ++ox) {
                    uint64_t k = kyz + gx[ox + m];
                    if (k > r2) continue;
                    ents.push_back({k, pack_offset(ox, oy, oz)});
                    uint32_t a = (uint32_t)std::max(std::abs(ox), std::max(std::abs(oy), std::abs(oz)));
                    t->max_off = std::max(t->max_off, a);
                }
            }
        }
        // increasing key; equal keys in a fixed order (packed offset)
        std::sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) {
            return a.key < b.key || (a.key == b.key && a.off < b.off);
        });
        t->h_class_start[cls] = (uint32_t)t->h_off.size();
        for (const Ent& en : ents) {
            t->h_off.push_back(en.off);
            t->h_key.push_back((int64_t)en.key);
        }
        // radius index: entries with key <= (j << rshift)^2
        size_t p = 0;
        for (uint32_t j = 0; j < t->nr; ++j) {
            uint64_t rj = (uint64_t)j << t->rshift;
            uint64_t rj2 = rj * rj;
            while (p < ents.size() && ents[p].key <= rj2) ++p;
            t->h_rindex[(size_t)cls * t->nr + j] = (uint32_t)p;
        }
    }
    t->h_class_start[ncls] = (uint32_t)t->h_off.size();
    t->total = t->h_off.size();
    tables_build_rows(t);
    tables_build_paper(t);
    return SPHIDX_OK;
}

void tables_free(sphidx_tables* t) { free_device(t); }

sphidx_status tables_save_file(const sphidx_tables* t, const char* path) {
    FILE* f = std::fopen(path, "wb");
    if (!f) return SPHIDX_ERR_IO;
    uint64_t h = 0xcbf29ce484222325ull;
    bool ok = true;
    auto put = [&](const void* d, size_t n) {
        if (n && std::fwrite(d, 1, n, f) != n) ok = false;
        h = fnv1a(d, n, h);
    };
    uint32_t hdr[8] = {kVersion, t->s, t->F, t->rmax_fx, t->nclasses, t->nr, t->rshift, t->max_off};
    uint64_t total = t->total;
    put(kMagic, 8);
    put(hdr, sizeof(hdr));
    put(&total, 8);
    put(t->h_class_start.data(), t->h_class_start.size() * 4);
    put(t->h_off.data(), t->h_off.size() * 4);
    put(t->h_key.data(), t->h_key.size() * 8);
    put(t->h_rindex.data(), t->h_rindex.size() * 4);
    if (std::fwrite(&h, 1, 8, f) != 8) ok = false;
    if (std::fclose(f) != 0) ok = false;
    return ok ? SPHIDX_OK : SPHIDX_ERR_IO;
}

sphidx_status tables_load_file(const char* path, sphidx_tables* t) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return SPHIDX_ERR_IO;
    uint64_t h = 0xcbf29ce484222325ull;
    bool ok = true;
    auto get = [&](void* d, size_t n) {
        if (!ok) return;
        if (n && std::fread(d, 1, n, f) != n) {
            ok = false;
            return;
        }
        h = fnv1a(d, n, h);
    };
    char magic[8];
    uint32_t hdr[8];
    uint64_t total = 0;
    get(magic, 8);
    get(hdr, sizeof(hdr));
    get(&total, 8);
    if (!ok || std::memcmp(magic, kMagic, 8) != 0 || hdr[0] != kVersion || hdr[1] > 3 || hdr[4] != (1u << (3 * hdr[1])) ||
        hdr[5] == 0 || hdr[5] > (1u << 26) || total > (1ull << 32)) {
        std::fclose(f);
        return SPHIDX_ERR_IO;
    }
    t->s = hdr[1];
    t->F = hdr[2];
    t->rmax_fx = hdr[3];
    t->nclasses = hdr[4];
    t->nr = hdr[5];
    t->rshift = hdr[6];
    t->max_off = hdr[7];
    t->total = total;
    t->h_class_start.resize(t->nclasses + 1);
    t->h_off.resize(total);
    t->h_key.resize(total);
    t->h_rindex.resize((size_t)t->nclasses * t->nr);
    get(t->h_class_start.data(), t->h_class_start.size() * 4);
    get(t->h_off.data(), total * 4);
    get(t->h_key.data(), total * 8);
    get(t->h_rindex.data(), t->h_rindex.size() * 4);
    uint64_t stored = 0;
    if (ok && std::fread(&stored, 1, 8, f) != 8) ok = false;
    char extra;
    if (ok && std::fread(&extra, 1, 1, f) != 0) ok = false;  // trailing bytes
    std::fclose(f);
    if (!ok || stored != h) return SPHIDX_ERR_IO;
    // structural checks
    if (t->h_class_start[0] != 0 || t->h_class_start[t->nclasses] != total) return SPHIDX_ERR_IO;
    for (uint32_t c = 0; c < t->nclasses; ++c) {
        uint32_t b = t->h_class_start[c], en = t->h_class_start[c + 1];
        if (en < b) return SPHIDX_ERR_IO;
        for (uint32_t j = 0; j < t->nr; ++j)
            if (t->h_rindex[(size_t)c * t->nr + j] > en - b) return SPHIDX_ERR_IO;
    }
    if (t->s > t->F || t->F > 30) return SPHIDX_ERR_IO;
    tables_build_rows(t);
    tables_build_paper(t);
    return SPHIDX_OK;
}
