// C ABI of libsphidx: argument validation, workspace layout and dispatch.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "sphidx_internal.h"

sphidx_status tables_build_host(uint32_t F, uint32_t s, uint32_t rmax_fx, sphidx_tables* t);
void tables_free(sphidx_tables* t);
sphidx_status tables_save_file(const sphidx_tables* t, const char* path);
sphidx_status tables_upload(sphidx_tables* t);
sphidx_status tables_load_file(const char* path, sphidx_tables* t);
size_t scan_u32_tmp_words(size_t n);

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kMaxBlockLds = 64 * 1024;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

bool desc_ok(const sphidx_lattice_desc* d) {
    if (!d) return false;
    uint32_t sum = 0;
    for (int a = 0; a < 3; ++a) {
        if (d->log2_cells[a] > 10) return false;
        if (d->frac_bits + d->log2_cells[a] > 30) return false;
        sum += d->log2_cells[a];
    }
    return sum <= SPHIDX_MAX_LOG2_SUM && d->cyclic_mask <= 7u;
}

uint32_t ncells_of(const sphidx_lattice_desc* d) {
    return 1u << (d->log2_cells[0] + d->log2_cells[1] + d->log2_cells[2]);
}

struct Layout {
    size_t cell_start, pts, rank, scan_tmp, status, total;
};

Layout lattice_layout(const sphidx_lattice_desc* d, uint32_t max_points) {
    Layout L;
    size_t nc = (size_t)ncells_of(d);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes ? bytes : 4);
        return o;
    };
    L.cell_start = take((nc + 4) * 4);
    L.pts = take((size_t)max_points * 16);
    // per-object build scratch; also the flags of the non-empty cell list and
    // their scan (one word more for the total)
    L.rank = take(((size_t)max_points + 1) * 4);
    L.scan_tmp = take(scan_u32_tmp_words(std::max(nc + 2, (size_t)max_points)) * 4);
    L.status = take(64 * 4);
    L.total = off;
    return L;
}

LatArgs lat_args(const sphidx_lattice* lat) {
    LatArgs L;
    for (int a = 0; a < 3; ++a) L.lg[a] = lat->desc.log2_cells[a];
    L.F = lat->desc.frac_bits;
    L.cyc = lat->desc.cyclic_mask;
    L.ncells = lat->ncells;
    L.n = lat->n;
    L.cs = lat->cell_start;
    L.pts = lat->pts;
    L.status = lat->status;
    L.cells = lat->cell_list ? (const uint2*)(lat->cell_list + 16) : nullptr;
    L.ncl = lat->cell_list ? (const uint32_t*)lat->cell_list : nullptr;
    // queries look at the x-order word only on lattices built to keep it, so
    // that the others pay one uniform branch per row
    L.xsorted = lat->cell_order == SPHIDX_ORDER_X ? lat->status + 1 : nullptr;
    return L;
}

TabArgs tab_args(const sphidx_tables* t) {
    TabArgs T;
    std::memset(&T, 0, sizeof(T));
    if (!t) return T;
    T.rows = t->d_rows;
    T.rkey = t->d_rkey;
    T.cstart = t->d_rclass_start;
    T.rindex = t->d_rrindex;
    T.vcount = t->d_vcount;
    T.s = t->s;
    T.rshift = t->rshift;
    T.nr = t->nr;
    T.rmax = t->rmax_fx;
    T.total = (uint32_t)t->h_rows.size();
    T.nrcls = t->nrclasses;
    T.has = 1;
    T.p_off = t->d_poff;
    T.p_b2 = t->d_pb2;
    T.p_lo = t->d_plo;
    T.p_nb2 = t->pnb2;
    return T;
}

struct Launch {
    uint32_t method, persistent, waves, tile, bpc, cap, tab_lds, lds_chunk, interior, no_stash, grouped, long_waves;
    uint32_t weight, rev, knn_rev, model;
    uint32_t* stats;
    uint32_t* method_out;
    hipEvent_t ev_begin, ev_end;
};

sphidx_status resolve_launch(const sphidx_launch* in, const sphidx_tables* tab, Launch& o) {
    o.method = in ? in->method : SPHIDX_METHOD_SPHERE;
    o.persistent = in ? (in->schedule == SPHIDX_SCHED_PERSISTENT) : 1u;
    o.waves = (in && in->waves_per_block) ? in->waves_per_block : 4u;
    o.tile = (in && in->tile) ? in->tile : (o.persistent ? 64u : 1u);
    o.bpc = (in && in->blocks_per_cu) ? in->blocks_per_cu : 8u;
    o.cap = (in && in->sort_cap) ? in->sort_cap : 256u;
    o.tab_lds = in ? in->table_in_lds : 0u;
    o.lds_chunk = 0;
    if (o.tab_lds > 2) return SPHIDX_ERR_INVALID_ARG;
    o.interior = in ? in->interior : 0u;
    if (o.interior > 2) return SPHIDX_ERR_INVALID_ARG;
    o.no_stash = in ? in->no_stash : 0u;
    if (o.no_stash > 1) return SPHIDX_ERR_INVALID_ARG;
    o.grouped = in ? in->grouped : 0u;
    if (o.grouped > 1) return SPHIDX_ERR_INVALID_ARG;
    o.long_waves = (in && in->long_row_waves) ? in->long_row_waves : 4u;
    if (!(o.long_waves == 1 || o.long_waves == 2 || o.long_waves == 4 || o.long_waves == 8))
        return SPHIDX_ERR_INVALID_ARG;
    o.stats = in ? in->stats_dev : nullptr;
    o.method_out = in ? in->method_dev : nullptr;
    o.weight = (in && in->select_weight) ? in->select_weight : 256u;
    o.rev = in ? in->reversal_fx : 0u;
    o.knn_rev = in ? in->knn_reversal_fx : 0u;
    o.model = in ? in->select_model : 0u;
    if (o.model > 1) return SPHIDX_ERR_INVALID_ARG;
    if (o.weight > (1u << 16)) return SPHIDX_ERR_INVALID_ARG;
    o.ev_begin = in ? (hipEvent_t)in->event_begin : nullptr;
    o.ev_end = in ? (hipEvent_t)in->event_end : nullptr;
    if (in && in->schedule > SPHIDX_SCHED_PERSISTENT) return SPHIDX_ERR_INVALID_ARG;
    if (o.method > SPHIDX_METHOD_PAPER64) return SPHIDX_ERR_INVALID_ARG;
    if (!(o.waves == 1 || o.waves == 2 || o.waves == 4)) return SPHIDX_ERR_INVALID_ARG;
    if (o.cap < 64 || o.cap > 256 || (o.cap & (o.cap - 1))) return SPHIDX_ERR_INVALID_ARG;
    if (o.tile > 4096 || o.bpc > 64) return SPHIDX_ERR_INVALID_ARG;
    const bool tables = o.method == SPHIDX_METHOD_SPHERE || o.method == SPHIDX_METHOD_AUTO ||
                        o.method == SPHIDX_METHOD_PAPER64;
    if (tables && !tab) return SPHIDX_ERR_INVALID_ARG;
    // the paper's tables exist only for offsets up to kPaperMaxOff cells
    if (o.method == SPHIDX_METHOD_PAPER64 && !tab->pm) return SPHIDX_ERR_RADIUS;
    // the row table is what LDS staging holds; the paper's cell tables and
    // the other walks read device memory
    if (o.method != SPHIDX_METHOD_SPHERE && o.method != SPHIDX_METHOD_AUTO) o.tab_lds = 0;
    size_t tab_bytes = (o.tab_lds == 1 && tab) ? (tab->h_rows.size() * 4 + 15) / 16 * 16 : 0;
    if (o.tab_lds == 2 && tab) {
        // the first rows of every (y, z) class, as many as fit beside the
        // largest per-block buffer of the passes
        size_t worst = 0;
        for (int pass = 1; pass <= 5; ++pass) worst = std::max(worst, query_lds_bytes(pass, o.cap, o.waves, 0));
        const size_t room = kMaxBlockLds > worst ? kMaxBlockLds - worst : 0;
        uint32_t longest = 0;
        for (uint32_t c = 0; c < tab->nrclasses; ++c)
            longest = std::max(longest, tab->h_rclass_start[c + 1] - tab->h_rclass_start[c]);
        const uint32_t chunk = (uint32_t)std::min<size_t>(room / (4u * tab->nrclasses), longest) & ~3u;
        if (chunk < 16) return SPHIDX_ERR_CAPACITY;
        o.lds_chunk = chunk;
        tab_bytes = ((size_t)tab->nrclasses * chunk * 4 + 15) / 16 * 16;
    }
    for (int pass = 1; pass <= 5; ++pass) {
        if (query_lds_bytes(pass, o.cap, o.waves, 0) > kMaxBlockLds) return SPHIDX_ERR_INVALID_ARG;
        if (o.tab_lds && query_lds_bytes(pass, o.cap, o.waves, tab_bytes) > kMaxBlockLds) return SPHIDX_ERR_CAPACITY;
    }
    return SPHIDX_OK;
}

// Query workspace: counters | descriptors[Q] | longq[Q] | fbq[Q] | walkq[Q] |
// soff[Q] | xq[Q] | lq[Q] | scan partials, then the stash: every byte beyond
// the minimum.
struct QLayout {
    size_t counters, desc, longq, fbq, walkq, soff, xq, lq, scan, total;
};

QLayout query_layout(uint32_t Q) {
    QLayout l;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes ? bytes : 4);
        return o;
    };
    l.counters = take(SPHIDX_COUNTER_WORDS * 4);
    l.desc = take((size_t)Q * 64);
    l.longq = take((size_t)Q * 4);
    l.fbq = take((size_t)Q * 4);
    l.walkq = take((size_t)Q * 4);
    l.soff = take((size_t)Q * 4);
    l.xq = take((size_t)Q * 4);
    l.lq = take((size_t)Q * 4);
    l.scan = take(scan_i64_tmp_bytes(Q));
    l.total = off;
    return l;
}

size_t query_ws_bytes(uint32_t Q) { return query_layout(Q).total; }

sphidx_status check_queries(const sphidx_lattice* lat, const sphidx_queries* q, const sphidx_csr* csr) {
    if (!lat || !q || !csr || !csr->row_ptr_dev) return SPHIDX_ERR_INVALID_ARG;
    bool all = q->x_dev == nullptr;
    if (all != (q->y_dev == nullptr) || all != (q->z_dev == nullptr)) return SPHIDX_ERR_INVALID_ARG;
    if (all && q->count != lat->n) return SPHIDX_ERR_INVALID_ARG;
    if (q->mode > SPHIDX_MODE_MIXED) return SPHIDX_ERR_INVALID_ARG;
    if (q->flags & ~SPHIDX_EXCLUDE_SELF) return SPHIDX_ERR_INVALID_ARG;
    if (csr->capacity < 0) return SPHIDX_ERR_INVALID_ARG;
    if (!csr->workspace_dev || csr->workspace_bytes < query_ws_bytes(q->count)) return SPHIDX_ERR_CAPACITY;
    if (((uintptr_t)csr->workspace_dev) % kAlign) return SPHIDX_ERR_INVALID_ARG;
    return SPHIDX_OK;
}

QArgs q_args(const sphidx_queries* q, sphidx_csr* csr, const Launch& ln) {
    QArgs A;
    std::memset(&A, 0, sizeof(A));
    A.Q = q->count;
    A.qx = q->x_dev;
    A.qy = q->y_dev;
    A.qz = q->z_dev;
    A.rad = q->radius_fx_dev;
    A.rad_u = q->radius_fx;
    A.kk = q->k_dev;
    A.k_u = q->k;
    A.mode = q->mode;
    A.flags = q->flags;
    A.row_ptr = csr->row_ptr_dev;
    A.out_ids = csr->ids_dev;
    A.out_d2 = csr->dist2_dev;
    A.capacity = csr->capacity;
    const QLayout ql = query_layout(q->count);
    char* ws = (char*)csr->workspace_dev;
    A.queues = (uint32_t*)(ws + ql.counters);
    uint32_t* lists = A.queues + SPHIDX_NQSETS * SPHIDX_NQUEUE * SPHIDX_QSTRIDE;
    A.long_count = lists;
    A.fb_count = lists + SPHIDX_QSTRIDE;
    A.walk_count = lists + 2 * SPHIDX_QSTRIDE;
    A.stash_hdr = lists + 3 * SPHIDX_QSTRIDE;
    A.xq_count = lists + 4 * SPHIDX_QSTRIDE;
    A.lq_count = lists + 5 * SPHIDX_QSTRIDE;
    A.stash_ctr = lists + SPHIDX_NLISTS * SPHIDX_QSTRIDE;
    A.longq = (uint32_t*)(ws + ql.longq);
    A.fbq = (uint32_t*)(ws + ql.fbq);
    A.walkq = (uint32_t*)(ws + ql.walkq);
    A.soff = (uint32_t*)(ws + ql.soff);
    A.xq = (uint32_t*)(ws + ql.xq);
    A.lq = (uint32_t*)(ws + ql.lq);
    A.desc = (uint4*)(ws + ql.desc);
    A.stash_base = ws + ql.total;
    A.stats = ln.stats;
    A.method = ln.method;
    A.persistent = ln.persistent;
    A.tile = ln.tile;
    A.sort_cap = ln.cap;
    A.select = ln.method == SPHIDX_METHOD_AUTO ? 1u : ln.method == SPHIDX_METHOD_LIST ? 2u : 0u;
    A.weight = ln.weight;
    A.rev = ln.rev;
    A.knn_rev = ln.knn_rev;
    A.model = ln.model;
    A.method_out = ln.method_out;
    A.long_waves = ln.long_waves;
    return A;
}

// Count pass: size the stash from the bytes beyond the minimum workspace.
// Rows are kept as ids (plus dist^2 when this call asks for them) in
// NQUEUE regions, one per XCD, handed out to waves in chunks.
void plan_stash(QArgs& A, const sphidx_csr* csr, const Launch& ln, bool interior_forced) {
    A.stash = 0;
    // plain launches: a wave lives for `tile` queries only, too short to
    // fill a chunk of its own
    if (ln.no_stash || !ln.persistent || interior_forced) return;
    const size_t base = query_layout(A.Q).total;
    if (csr->workspace_bytes <= base + 4096) return;
    const size_t room = csr->workspace_bytes - base - 512;  // alignment slack
    const bool d2 = csr->dist2_dev != nullptr;
    uint64_t elems = d2 ? room / 12 : room / 4;
    elems = std::min<uint64_t>(elems, 0xFFFFFF00ull);
    const uint64_t region = elems / SPHIDX_NREGION;
    if (region < 4096) return;
    A.stash = 1;
    A.stash_region = (uint32_t)region;
    A.stash_ids = (uint32_t*)A.stash_base;
    A.stash_d2 = d2 ? (int64_t*)(A.stash_base + align_up(region * SPHIDX_NREGION * 4)) : nullptr;
    // about 8 grabs per resident wave and region: little tail left unused
    const uint64_t waves = (uint64_t)device_cu_count() * ln.bpc * ln.waves;
    const uint64_t per = std::max<uint64_t>(1, waves / SPHIDX_NREGION);
    A.stash_chunk = (uint32_t)std::min<uint64_t>(8192, std::max<uint64_t>(ln.cap, region / (per * 8)));
}

void* scan_tmp_of(sphidx_csr* csr, uint32_t Q) { return (char*)csr->workspace_dev + query_layout(Q).scan; }

sphidx_status dev_err(hipError_t e) { return e == hipSuccess ? SPHIDX_OK : SPHIDX_ERR_DEVICE; }

// Lattices whose status words a stream has touched since the last
// sphidx_stream_status on it: (stream, lattice) pairs, noted by every entry
// point that enqueues work on a lattice.
std::mutex g_touch_mu;
std::vector<std::pair<void*, const sphidx_lattice*>> g_touched;

void note_stream(const sphidx_lattice* lat, void* stream) {
    std::lock_guard<std::mutex> lk(g_touch_mu);
    for (const auto& t : g_touched)
        if (t.first == stream && t.second == lat) return;
    g_touched.emplace_back(stream, lat);
}

void forget_lattice(const sphidx_lattice* lat) {
    std::lock_guard<std::mutex> lk(g_touch_mu);
    g_touched.erase(std::remove_if(g_touched.begin(), g_touched.end(),
                                   [lat](const std::pair<void*, const sphidx_lattice*>& t) { return t.second == lat; }),
                    g_touched.end());
}

// Read and clear one lattice's status word in stream order (synchronises).
sphidx_status take_status(const sphidx_lattice* lat, hipStream_t st, uint32_t* v) {
    *v = 0;
    if (hipMemcpyAsync(v, lat->status, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return SPHIDX_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return SPHIDX_ERR_DEVICE;
    if (launch_fill_u32(lat->status, 0u, 1, st) != hipSuccess) return SPHIDX_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return SPHIDX_ERR_DEVICE;
    return SPHIDX_OK;
}

sphidx_status status_of_flags(uint32_t v) {
    if (v & SPHIDX_FLAG_RANGE) return SPHIDX_ERR_RANGE;
    if (v & SPHIDX_FLAG_CAPACITY) return SPHIDX_ERR_CAPACITY;
    return SPHIDX_OK;
}


// Upload freshly built or loaded tables when a device is present.  Without
// one (a CPU-only host) the tables stay host-only: they can be inspected,
// saved and loaded, and are uploaded on first use by a query.
sphidx_status attach_device(sphidx_tables* t) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return SPHIDX_OK;
    return tables_upload(t);
}

sphidx_status run_pass(int pass, const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                       sphidx_csr* csr, const sphidx_launch* launch, hipStream_t st) {
    sphidx_status s = check_queries(lat, q, csr);
    if (s != SPHIDX_OK) return s;
    Launch ln;
    s = resolve_launch(launch, tab, ln);
    if (s != SPHIDX_OK) return s;
    if (pass == 1 && csr->capacity > 0 && !csr->ids_dev) return SPHIDX_ERR_INVALID_ARG;
    if (tab && tab->F != lat->desc.frac_bits) return SPHIDX_ERR_INVALID_ARG;
    const bool tables = ln.method == SPHIDX_METHOD_SPHERE || ln.method == SPHIDX_METHOD_AUTO ||
                        ln.method == SPHIDX_METHOD_PAPER64;
    if (ln.method == SPHIDX_METHOD_LIST && !lat->cell_list) return SPHIDX_ERR_INVALID_ARG;
    if (tab && tables && !tab->d_rows) {
        s = tables_upload(const_cast<sphidx_tables*>(tab));
        if (s != SPHIDX_OK) return s;
    }
    note_stream(lat, (void*)st);
    LatArgs L = lat_args(lat);
    TabArgs T = tab_args(tables ? tab : nullptr);
    T.lds = ln.tab_lds ? 1u : 0u;
    T.lds_chunk = ln.lds_chunk;
    T.paper = ln.method == SPHIDX_METHOD_PAPER64 ? 1u : 0u;
    QArgs A = q_args(q, csr, ln);
    if (pass == 0) plan_stash(A, csr, ln, ln.interior == 2);
    // counting wholly-inside cells whole saves object reads but costs a
    // second extent per row: worth it once cells hold an object or more
    // (not with the stash, which needs every object of a row)
    A.interior = !A.stash &&
                 (ln.interior == 2 || (ln.interior == 0 && (uint64_t)lat->n >= (uint64_t)lat->ncells));
    // count pass: radius queries in groups of several per wavefront (the
    // persistent schedule; not with per-query statistics or the interior
    // shortcut, which the grouped kernel does not implement)
    // (the paper's cell tables are walked one query per wavefront)
    A.group = pass == 0 && ln.persistent && ln.grouped && !A.interior && !T.paper;
    if (pass == 0) {
        s = dev_err(launch_query_pass(0, L, T, A, ln.waves, ln.bpc, st, ln.ev_begin, ln.ev_end));
        if (s != SPHIDX_OK) return s;
        return dev_err(launch_scan_i64(csr->row_ptr_dev, q->count, scan_tmp_of(csr, q->count), st));
    }
    return dev_err(launch_query_pass(1, L, T, A, ln.waves, ln.bpc, st, ln.ev_begin, ln.ev_end));
}

}  // namespace

sphidx_status check_launch(const sphidx_launch* launch, const sphidx_tables* tab) {
    Launch ln{};
    return resolve_launch(launch, tab, ln);
}

void forget_stream(void* stream) {
    std::lock_guard<std::mutex> lk(g_touch_mu);
    g_touched.erase(std::remove_if(g_touched.begin(), g_touched.end(),
                                   [stream](const std::pair<void*, const sphidx_lattice*>& t) {
                                       return t.first == stream;
                                   }),
                    g_touched.end());
}

extern "C" {

size_t sphidx_lattice_workspace_bytes(const sphidx_lattice_desc* desc, uint32_t max_points) {
    if (!desc_ok(desc)) return 0;
    return lattice_layout(desc, max_points).total;
}

sphidx_status sphidx_lattice_create(const sphidx_lattice_desc* desc, uint32_t max_points, void* workspace_dev,
                                    size_t workspace_bytes, sphidx_lattice** out) {
    if (!out) return SPHIDX_ERR_INVALID_ARG;
    *out = nullptr;
    if (!desc_ok(desc) || !workspace_dev || ((uintptr_t)workspace_dev % kAlign)) return SPHIDX_ERR_INVALID_ARG;
    if (max_points > 0xFFFFFF00u) return SPHIDX_ERR_INVALID_ARG;
    Layout ly = lattice_layout(desc, max_points);
    if (workspace_bytes < ly.total) return SPHIDX_ERR_CAPACITY;
    sphidx_lattice* lat = new (std::nothrow) sphidx_lattice();
    if (!lat) return SPHIDX_ERR_OUT_OF_MEMORY;
    char* b = (char*)workspace_dev;
    lat->desc = *desc;
    lat->max_points = max_points;
    lat->n = 0;
    lat->ncells = ncells_of(desc);
    lat->cell_start = (uint32_t*)(b + ly.cell_start);
    lat->pts = (uint4*)(b + ly.pts);
    lat->rank = (uint32_t*)(b + ly.rank);
    lat->scan_tmp = (uint32_t*)(b + ly.scan_tmp);
    lat->status = (uint32_t*)(b + ly.status);
    lat->bytes = ly.total;
    lat->cell_order = SPHIDX_ORDER_ANY;
    lat->xbuf = nullptr;
    (void)hipGetDevice(&lat->device);
    // an empty lattice until the first build: every cell empty, status clear
    // (skipped on a host without a device, where only validation can run)
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0 &&
        (launch_fill_u32(lat->cell_start, 0u, (size_t)lat->ncells + 4, nullptr) != hipSuccess ||
         launch_fill_u32(lat->status, 0u, 64, nullptr) != hipSuccess)) {
        delete lat;
        return SPHIDX_ERR_DEVICE;
    }
    *out = lat;
    return SPHIDX_OK;
}

void sphidx_lattice_destroy(sphidx_lattice* lat) {
    if (!lat) return;
    forget_lattice(lat);
    if (lat->xbuf) (void)hipFree(lat->xbuf);
    delete lat;
}

sphidx_status sphidx_build_lattice(sphidx_lattice* lat, const uint32_t* x_dev, const uint32_t* y_dev,
                                   const uint32_t* z_dev, uint32_t n, void* stream) {
    if (!lat || n > lat->max_points) return lat ? SPHIDX_ERR_CAPACITY : SPHIDX_ERR_INVALID_ARG;
    if (n > 0 && (!x_dev || !y_dev || !z_dev)) return SPHIDX_ERR_INVALID_ARG;
    lat->n = n;
    note_stream(lat, stream);
    return dev_err(launch_build(lat, x_dev, y_dev, z_dev, n, (hipStream_t)stream));
}

size_t sphidx_cell_list_bytes(const sphidx_lattice* lat) {
    if (!lat) return 0;
    const size_t entries = (size_t)std::min(lat->max_points, lat->ncells) + 1;
    return 16 + entries * 8;
}

sphidx_status sphidx_lattice_attach_cell_list(sphidx_lattice* lat, void* list_dev, size_t bytes, void* stream) {
    if (!lat) return SPHIDX_ERR_INVALID_ARG;
    if (!list_dev) {
        lat->cell_list = nullptr;
        return SPHIDX_OK;
    }
    if ((uintptr_t)list_dev % kAlign) return SPHIDX_ERR_INVALID_ARG;
    if (bytes < sphidx_cell_list_bytes(lat)) return SPHIDX_ERR_CAPACITY;
    lat->cell_list = (char*)list_dev;
    note_stream(lat, stream);
    const sphidx_status s = dev_err(launch_cell_list(lat, (hipStream_t)stream));
    if (s != SPHIDX_OK) lat->cell_list = nullptr;
    return s;
}

sphidx_status sphidx_lattice_get_view(const sphidx_lattice* lat, sphidx_lattice_view* out) {
    if (!lat || !out) return SPHIDX_ERR_INVALID_ARG;
    out->cell_start = lat->cell_start;
    out->points = (const uint32_t*)lat->pts;
    out->n = lat->n;
    out->ncells = lat->ncells;
    return SPHIDX_OK;
}

sphidx_status sphidx_lattice_set_cell_order(sphidx_lattice* lat, uint32_t order) {
    if (!lat || order > SPHIDX_ORDER_X) return SPHIDX_ERR_INVALID_ARG;
    if (order == SPHIDX_ORDER_X && !lat->xbuf && lat->max_points > 0) {
        // the counting sort's records, before the x ranking places them
        void* p = nullptr;
        if (hipMalloc(&p, (size_t)lat->max_points * sizeof(uint4)) != hipSuccess) return SPHIDX_ERR_OUT_OF_MEMORY;
        lat->xbuf = (uint4*)p;
    }
    lat->cell_order = order;
    return SPHIDX_OK;
}

sphidx_status sphidx_lattice_status(sphidx_lattice* lat, void* stream, uint32_t* flags_out) {
    if (!lat) return SPHIDX_ERR_INVALID_ARG;
    uint32_t v = 0;
    const sphidx_status s = take_status(lat, (hipStream_t)stream, &v);
    if (s != SPHIDX_OK) return s;
    if (flags_out) *flags_out = v;
    return status_of_flags(v);
}

sphidx_status sphidx_stream_status(void* stream, uint32_t* flags_out) {
    std::vector<const sphidx_lattice*> lats;
    {
        std::lock_guard<std::mutex> lk(g_touch_mu);
        for (auto it = g_touched.begin(); it != g_touched.end();) {
            if (it->first == stream) {
                lats.push_back(it->second);
                it = g_touched.erase(it);
            } else {
                ++it;
            }
        }
    }
    hipStream_t st = (hipStream_t)stream;
    if (lats.empty() && hipStreamSynchronize(st) != hipSuccess) return SPHIDX_ERR_DEVICE;
    uint32_t all = 0;
    for (const sphidx_lattice* lat : lats) {
        uint32_t v = 0;
        const sphidx_status s = take_status(lat, st, &v);
        if (s != SPHIDX_OK) return s;
        all |= v;
    }
    if (flags_out) *flags_out = all;
    return status_of_flags(all);
}

sphidx_status sphidx_build_sphere_tables(const sphidx_lattice_desc* desc, uint32_t subcell_bits,
                                         uint32_t rmax_fx, sphidx_tables** out) {
    if (!out) return SPHIDX_ERR_INVALID_ARG;
    *out = nullptr;
    if (!desc_ok(desc)) return SPHIDX_ERR_INVALID_ARG;
    const uint32_t F = desc->frac_bits;
    if (subcell_bits > 3 || subcell_bits > F) return SPHIDX_ERR_INVALID_ARG;
    if (F + 2 >= 31 || (uint64_t)rmax_fx > (1ull << 31) - (1ull << (F + 2))) return SPHIDX_ERR_RADIUS;
    uint64_t m = (((uint64_t)rmax_fx + (1ull << F) - 1) >> F) + 1;
    if (m > 511) return SPHIDX_ERR_RADIUS;
    sphidx_tables* t = new (std::nothrow) sphidx_tables();
    if (!t) return SPHIDX_ERR_OUT_OF_MEMORY;
    sphidx_status s = tables_build_host(F, subcell_bits, rmax_fx, t);
    if (s == SPHIDX_OK) s = attach_device(t);
    if (s != SPHIDX_OK) {
        tables_free(t);
        delete t;
        return s;
    }
    *out = t;
    return SPHIDX_OK;
}

void sphidx_tables_destroy(sphidx_tables* tab) {
    if (!tab) return;
    tables_free(tab);
    delete tab;
}

sphidx_status sphidx_tables_get_info(const sphidx_tables* tab, sphidx_tables_info* out) {
    if (!tab || !out) return SPHIDX_ERR_INVALID_ARG;
    out->subcell_bits = tab->s;
    out->frac_bits = tab->F;
    out->rmax_fx = tab->rmax_fx;
    out->nclasses = tab->nclasses;
    out->total_entries = tab->total;
    out->device_bytes = tab->device_bytes;
    return SPHIDX_OK;
}

sphidx_status sphidx_tables_export(const sphidx_tables* tab, uint32_t cls, int32_t* offsets_host,
                                   int64_t* keys_host, uint64_t* n_inout) {
    if (!tab || !n_inout || cls >= tab->nclasses) return SPHIDX_ERR_INVALID_ARG;
    uint32_t b = tab->h_class_start[cls], e = tab->h_class_start[cls + 1];
    uint64_t n = e - b, cap = *n_inout;
    *n_inout = n;
    if ((offsets_host || keys_host) && cap < n) return SPHIDX_ERR_CAPACITY;
    for (uint64_t i = 0; i < n && (offsets_host || keys_host); ++i) {
        uint32_t w = tab->h_off[b + i];
        if (offsets_host) {
            offsets_host[3 * i + 0] = ((int32_t)(w << 22)) >> 22;
            offsets_host[3 * i + 1] = ((int32_t)(w << 12)) >> 22;
            offsets_host[3 * i + 2] = ((int32_t)(w << 2)) >> 22;
        }
        if (keys_host) keys_host[i] = tab->h_key[b + i];
    }
    return SPHIDX_OK;
}

sphidx_status sphidx_tables_save(const sphidx_tables* tab, const char* path) {
    if (!tab || !path) return SPHIDX_ERR_INVALID_ARG;
    return tables_save_file(tab, path);
}

sphidx_status sphidx_tables_load(const char* path, sphidx_tables** out) {
    if (!path || !out) return SPHIDX_ERR_INVALID_ARG;
    *out = nullptr;
    sphidx_tables* t = new (std::nothrow) sphidx_tables();
    if (!t) return SPHIDX_ERR_OUT_OF_MEMORY;
    sphidx_status s = tables_load_file(path, t);
    if (s == SPHIDX_OK) s = attach_device(t);
    if (s != SPHIDX_OK) {
        tables_free(t);
        delete t;
        return s;
    }
    *out = t;
    return SPHIDX_OK;
}

size_t sphidx_query_workspace_bytes(uint32_t Q) { return query_ws_bytes(Q); }

size_t sphidx_query_stash_bytes(uint64_t pairs, int want_dist2) {
    // the rows, plus the tails left unused in each wave's last chunk (a
    // chunk is at most an eighth of a region per resident wave, at least
    // 256 objects) and the alignment slack
    const uint64_t waves = (uint64_t)device_cu_count() * 64u;
    const uint64_t elems = pairs + pairs / 4 + waves * 256u + 4096u * SPHIDX_NREGION;
    return (size_t)(elems * (want_dist2 ? 12u : 4u) + 1024u);
}

sphidx_status sphidx_count(const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                           sphidx_csr* csr, const sphidx_launch* launch, void* stream) {
    return run_pass(0, lat, tab, q, csr, launch, (hipStream_t)stream);
}

sphidx_status sphidx_write(const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                           sphidx_csr* csr, const sphidx_launch* launch, void* stream) {
    return run_pass(1, lat, tab, q, csr, launch, (hipStream_t)stream);
}

sphidx_status sphidx_query(const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                           sphidx_csr* csr, const sphidx_launch* launch, void* stream) {
    sphidx_status s = run_pass(0, lat, tab, q, csr, launch, (hipStream_t)stream);
    if (s != SPHIDX_OK) return s;
    return run_pass(1, lat, tab, q, csr, launch, (hipStream_t)stream);
}

static sphidx_status with_mode(const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                               sphidx_csr* csr, uint32_t mode, uint32_t method, void* stream) {
    if (!q) return SPHIDX_ERR_INVALID_ARG;
    sphidx_queries qq = *q;
    qq.mode = mode;
    sphidx_launch ln;
    std::memset(&ln, 0, sizeof(ln));
    ln.method = method;
    ln.schedule = SPHIDX_SCHED_PERSISTENT;
    return sphidx_query(lat, tab, &qq, csr, &ln, stream);
}

sphidx_status sphidx_radius_count(const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                                  sphidx_csr* csr, void* stream) {
    if (!q) return SPHIDX_ERR_INVALID_ARG;
    sphidx_queries qq = *q;
    qq.mode = SPHIDX_MODE_RADIUS;
    sphidx_launch ln;
    std::memset(&ln, 0, sizeof(ln));
    ln.schedule = SPHIDX_SCHED_PERSISTENT;
    return sphidx_count(lat, tab, &qq, csr, &ln, stream);
}

sphidx_status sphidx_radius_query(const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                                  sphidx_csr* csr, void* stream) {
    return with_mode(lat, tab, q, csr, SPHIDX_MODE_RADIUS, SPHIDX_METHOD_SPHERE, stream);
}

sphidx_status sphidx_knn_query(const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                               sphidx_csr* csr, void* stream) {
    return with_mode(lat, tab, q, csr, SPHIDX_MODE_KNN, SPHIDX_METHOD_SPHERE, stream);
}

sphidx_status sphidx_cube_scan_radius(const sphidx_lattice* lat, const sphidx_queries* q, sphidx_csr* csr,
                                      void* stream) {
    return with_mode(lat, nullptr, q, csr, SPHIDX_MODE_RADIUS, SPHIDX_METHOD_CUBE, stream);
}

sphidx_status sphidx_cube_scan_knn(const sphidx_lattice* lat, const sphidx_queries* q, sphidx_csr* csr,
                                   void* stream) {
    return with_mode(lat, nullptr, q, csr, SPHIDX_MODE_KNN, SPHIDX_METHOD_CUBE, stream);
}

sphidx_status sphidx_move_agents(const sphidx_lattice_desc* desc, uint64_t seed, uint32_t step, uint32_t* x_dev,
                                 uint32_t* y_dev, uint32_t* z_dev, uint32_t n, void* stream) {
    if (!desc_ok(desc)) return SPHIDX_ERR_INVALID_ARG;
    if (n > 0 && (!x_dev || !y_dev || !z_dev)) return SPHIDX_ERR_INVALID_ARG;
    return dev_err(launch_move_agents(*desc, seed, step, nullptr, x_dev, y_dev, z_dev, n, (hipStream_t)stream));
}

sphidx_status sphidx_move_agents_counted(const sphidx_lattice_desc* desc, uint64_t seed, uint32_t* step_dev,
                                         uint32_t* x_dev, uint32_t* y_dev, uint32_t* z_dev, uint32_t n,
                                         void* stream) {
    if (!desc_ok(desc) || !step_dev) return SPHIDX_ERR_INVALID_ARG;
    if (n > 0 && (!x_dev || !y_dev || !z_dev)) return SPHIDX_ERR_INVALID_ARG;
    return dev_err(launch_move_agents(*desc, seed, 0, step_dev, x_dev, y_dev, z_dev, n, (hipStream_t)stream));
}

sphidx_status sphidx_move_resident(sphidx_lattice* lat, uint64_t seed, uint32_t step, uint32_t* step_dev,
                                   void* scratch_dev, size_t scratch_bytes, void* stream) {
    if (!lat) return SPHIDX_ERR_INVALID_ARG;
    const uint32_t n = lat->n;
    if (n > 0 && (!scratch_dev || (uintptr_t)scratch_dev % 16)) return SPHIDX_ERR_INVALID_ARG;
    if (scratch_bytes < (size_t)n * sizeof(uint4)) return SPHIDX_ERR_CAPACITY;
    const hipStream_t st = (hipStream_t)stream;
    note_stream(lat, stream);
    uint4* moved = (uint4*)scratch_dev;
    hipError_t e = hipSuccess;
    if (step_dev) {
        e = launch_move_records(lat->desc, seed, step_dev, lat->pts, moved, n, st);
    } else {
        // a host step: the same kernel with the step as an argument
        e = launch_move_records_at(lat->desc, seed, step, lat->pts, moved, n, st);
    }
    if (e == hipSuccess) e = launch_build_records(lat, moved, n, st);
    return dev_err(e);
}

size_t sphidx_move_incremental_scratch_bytes(const sphidx_lattice* lat) {
    return lat ? move_incremental_scratch_bytes(lat) : 0;
}

sphidx_status sphidx_move_incremental(sphidx_lattice* lat, uint64_t seed, uint32_t step, uint32_t* step_dev,
                                      void* scratch_dev, size_t scratch_bytes, void* stream) {
    if (!lat) return SPHIDX_ERR_INVALID_ARG;
    if (!scratch_dev || (uintptr_t)scratch_dev % kAlign) return SPHIDX_ERR_INVALID_ARG;
    if (scratch_bytes < move_incremental_scratch_bytes(lat)) return SPHIDX_ERR_CAPACITY;
    note_stream(lat, stream);
    return dev_err(launch_move_incremental(lat, seed, step, step_dev, scratch_dev, (hipStream_t)stream));
}

sphidx_status sphidx_lattice_positions(const sphidx_lattice* lat, uint32_t* x_dev, uint32_t* y_dev, uint32_t* z_dev,
                                       void* stream) {
    if (!lat) return SPHIDX_ERR_INVALID_ARG;
    if (lat->n > 0 && (!x_dev || !y_dev || !z_dev)) return SPHIDX_ERR_INVALID_ARG;
    return dev_err(launch_records_to_ids(lat->pts, lat->n, x_dev, y_dev, z_dev, (hipStream_t)stream));
}

sphidx_status sphidx_count_checksum(const int64_t* row_ptr_dev, uint32_t Q, uint64_t* out_dev, void* stream) {
    if (!row_ptr_dev || !out_dev) return SPHIDX_ERR_INVALID_ARG;
    return dev_err(launch_count_checksum(row_ptr_dev, Q, out_dev, (hipStream_t)stream));
}

const char* sphidx_status_string(sphidx_status s) {
    switch (s) {
        case SPHIDX_OK: return "ok";
        case SPHIDX_ERR_INVALID_ARG: return "invalid argument";
        case SPHIDX_ERR_RANGE: return "coordinate out of range";
        case SPHIDX_ERR_RADIUS: return "radius out of range";
        case SPHIDX_ERR_CAPACITY: return "capacity exceeded";
        case SPHIDX_ERR_OUT_OF_MEMORY: return "out of memory";
        case SPHIDX_ERR_DEVICE: return "device error";
        case SPHIDX_ERR_IO: return "table file error";
    }
    return "unknown status";
}

const char* sphidx_version(void) { return "sphidx 1.0 gfx950"; }

}  // extern "C"
