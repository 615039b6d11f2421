/*
 * oracle.c -- plain, slow CPU oracle for spherical-indexing neighbourhood
 * queries (N. Brodu, "Spherical Indexing for Neighborhood Queries",
 * arXiv cs/0608108).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library under
 * paper_cs_0608108_amd/ may link, load or call this file; only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg do.  It shares
 * no code, header, table or constant generator with the HIP path.
 *
 * What it computes is the plain definition of the query (Section II.A):
 * the neighbours of a centre C for radius d are the objects X whose distance
 * x to C satisfies x <= d; the K-nearest variant keeps only the K closest
 * (Section I, Section II.A last paragraph).  The spherical index is an
 * acceleration that reaches exactly this set, so the oracle never uses
 * sphere tables for query results: tier 0 is an O(n) scan per query
 * (Section I, "naive algorithm"), tier 1 a plain bin-lattice scan of every
 * cell of the sphere's bounding cube (Section I, Section III.C).
 *
 * Number format (reading of the paper, which used float32): coordinates are
 * unsigned fixed point with `frac_bits` fractional bits per cell edge, so a
 * cell is the set of integer positions [k*2^F, (k+1)*2^F - 1] along each
 * axis; all distances are exact int64 squares.  A result row is ordered by
 * (squared distance, id), both ascending.
 *
 * Table keys (Sections II.A and III.A): the key of cell offset o for a query
 * whose sub-cell position lies in class box B is the minimum, over positions
 * in B, of the squared distance to the nearest position of cell o.  The
 * closed form and an exhaustive brute force are both given here so that
 * tests can pin one against the other and against Fig. 2.
 *
 * Every function is self-contained C99; OpenMP only spreads independent
 * queries over host threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Lattice description (the oracle's own; not shared with the library).      */

typedef struct {
    uint32_t log2_cells[3]; /* cells per axis L_a = 2^log2_cells[a] (Section II.B: power of two) */
    uint32_t frac_bits;     /* F: a cell edge is 2^F fixed-point units */
    uint32_t cyclic_mask;   /* bit a set: axis a wraps (Section II.B, cyclic case) */
} orc_desc;

#define ORC_EXCLUDE_SELF 1u

static int64_t axis_cells(const orc_desc *d, int a) { return (int64_t)1 << d->log2_cells[a]; }
static int64_t cell_edge(const orc_desc *d) { return (int64_t)1 << d->frac_bits; }
static int64_t axis_width(const orc_desc *d, int a) { return axis_cells(d, a) * cell_edge(d); }
static int is_cyclic(const orc_desc *d, int a) { return (int)((d->cyclic_mask >> a) & 1u); }

static int64_t floor_mod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

static int64_t floor_div(int64_t a, int64_t b) {
    /* b > 0 */
    if (a >= 0) return a / b;
    return -((-a + b - 1) / b);
}

/* A coordinate is usable on a clipped axis when below 2^30; any value is
 * usable on a cyclic axis, where it is reduced modulo the world width. */
static int coord_valid(const orc_desc *d, int a, uint32_t v) {
    return is_cyclic(d, a) || v < (1u << 30);
}

static int64_t coord_norm(const orc_desc *d, int a, uint32_t v) {
    return is_cyclic(d, a) ? floor_mod((int64_t)v, axis_width(d, a)) : (int64_t)v;
}

/* Signed separation p - q along axis a; on a cyclic axis the minimum image
 * in [-W/2, W/2) (a wrapping world has no boundary, Section III.C). */
static int64_t axis_delta(const orc_desc *d, int a, int64_t p, int64_t q) {
    int64_t dd = p - q;
    if (is_cyclic(d, a)) {
        int64_t w = axis_width(d, a);
        dd = floor_mod(dd + w / 2, w) - w / 2;
    }
    return dd;
}

/* ------------------------------------------------------------------------ */
/* Result rows.                                                              */

typedef struct {
    int64_t d2;
    uint32_t id;
} orc_pair;

typedef struct {
    orc_pair *v;
    int64_t n, cap;
} orc_row;

static void row_push(orc_row *r, int64_t d2, uint32_t id) {
    if (r->n == r->cap) {
        int64_t nc = r->cap ? 2 * r->cap : 16;
        orc_pair *nv = (orc_pair *)realloc(r->v, (size_t)nc * sizeof(orc_pair));
        if (!nv) abort();
        r->v = nv;
        r->cap = nc;
    }
    r->v[r->n].d2 = d2;
    r->v[r->n].id = id;
    r->n++;
}

static int pair_cmp(const void *a, const void *b) {
    const orc_pair *x = (const orc_pair *)a, *y = (const orc_pair *)b;
    if (x->d2 != y->d2) return x->d2 < y->d2 ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

static void row_sort(orc_row *r) {
    if (r->n > 1) qsort(r->v, (size_t)r->n, sizeof(orc_pair), pair_cmp);
}

typedef struct {
    int64_t nq;
    int64_t *row_ptr; /* nq + 1 */
    uint32_t *ids;
    int64_t *d2;
} orc_result;

/* Concatenate per-query rows into CSR and release them. */
static orc_result *rows_to_result(orc_row *rows, int64_t nq) {
    orc_result *res = (orc_result *)calloc(1, sizeof(orc_result));
    res->nq = nq;
    res->row_ptr = (int64_t *)malloc((size_t)(nq + 1) * sizeof(int64_t));
    int64_t tot = 0;
    for (int64_t i = 0; i < nq; ++i) {
        res->row_ptr[i] = tot;
        tot += rows[i].n;
    }
    res->row_ptr[nq] = tot;
    res->ids = (uint32_t *)malloc((size_t)(tot ? tot : 1) * sizeof(uint32_t));
    res->d2 = (int64_t *)malloc((size_t)(tot ? tot : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < nq; ++i) {
        int64_t o = res->row_ptr[i];
        for (int64_t k = 0; k < rows[i].n; ++k) {
            res->ids[o + k] = rows[i].v[k].id;
            res->d2[o + k] = rows[i].v[k].d2;
        }
        free(rows[i].v);
    }
    free(rows);
    return res;
}

int64_t orc_result_total(const orc_result *r) { return r->row_ptr[r->nq]; }

void orc_result_copy(const orc_result *r, int64_t *row_ptr, uint32_t *ids, int64_t *d2) {
    int64_t tot = r->row_ptr[r->nq];
    if (row_ptr) memcpy(row_ptr, r->row_ptr, (size_t)(r->nq + 1) * sizeof(int64_t));
    if (ids) memcpy(ids, r->ids, (size_t)tot * sizeof(uint32_t));
    if (d2) memcpy(d2, r->d2, (size_t)tot * sizeof(int64_t));
}

void orc_result_free(orc_result *r) {
    if (!r) return;
    free(r->row_ptr);
    free(r->ids);
    free(r->d2);
    free(r);
}

/* Threads of the OpenMP loops from now on (1 = serial). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Points and queries.                                                       */

typedef struct {
    int64_t c[3];
    int ok;
} orc_center;

static orc_center make_center(const orc_desc *d, uint32_t x, uint32_t y, uint32_t z) {
    orc_center q;
    uint32_t v[3] = {x, y, z};
    q.ok = 1;
    for (int a = 0; a < 3; ++a) {
        q.ok &= coord_valid(d, a, v[a]);
        q.c[a] = coord_norm(d, a, v[a]);
    }
    return q;
}

/* Squared distance per the definition: sum of squared (minimum-image) axis
 * separations, exact in int64 (each |delta| < 2^30). */
static int64_t dist2(const orc_desc *d, const int64_t *p, const int64_t *q) {
    int64_t s = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t t = axis_delta(d, a, p[a], q[a]);
        s += t * t;
    }
    return s;
}

/* Center of query i: explicit arrays, or point i in all-agents mode. */
static orc_center query_center(const orc_desc *d, int64_t i, const uint32_t *qx, const uint32_t *qy,
                               const uint32_t *qz, const uint32_t *px, const uint32_t *py,
                               const uint32_t *pz) {
    if (qx) return make_center(d, qx[i], qy[i], qz[i]);
    return make_center(d, px[i], py[i], pz[i]);
}

/* ------------------------------------------------------------------------ */
/* Tier 0: every query against every point (the O(n) query of Section I).    */

orc_result *orc_radius_brute(const orc_desc *d, uint32_t n, const uint32_t *px, const uint32_t *py,
                             const uint32_t *pz, uint32_t nq, const uint32_t *qx,
                             const uint32_t *qy, const uint32_t *qz, const uint32_t *r_fx,
                             uint32_t flags) {
    orc_center *pts = (orc_center *)malloc((size_t)(n ? n : 1) * sizeof(orc_center));
    for (uint32_t j = 0; j < n; ++j) pts[j] = make_center(d, px[j], py[j], pz[j]);
    orc_row *rows = (orc_row *)calloc((size_t)(nq ? nq : 1), sizeof(orc_row));
    int all_agents = (qx == NULL);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < (int64_t)nq; ++i) {
        orc_center q = query_center(d, i, qx, qy, qz, px, py, pz);
        if (!q.ok) continue;
        uint64_t r2 = (uint64_t)r_fx[i] * (uint64_t)r_fx[i];
        for (uint32_t j = 0; j < n; ++j) {
            if (!pts[j].ok) continue;
            if (all_agents && (flags & ORC_EXCLUDE_SELF) && (int64_t)j == i) continue;
            int64_t s = dist2(d, pts[j].c, q.c);
            if ((uint64_t)s <= r2) row_push(&rows[i], s, j);
        }
        row_sort(&rows[i]);
    }
    free(pts);
    return rows_to_result(rows, nq);
}

/* Tier 0 without the minimum-image formula: on cyclic axes, try the three
 * periodic images p - W, p, p + W of every point and keep the smallest
 * squared distance.  Valid because normalised coordinates lie in [0, W). */
orc_result *orc_radius_images(const orc_desc *d, uint32_t n, const uint32_t *px,
                              const uint32_t *py, const uint32_t *pz, uint32_t nq,
                              const uint32_t *qx, const uint32_t *qy, const uint32_t *qz,
                              const uint32_t *r_fx, uint32_t flags) {
    orc_row *rows = (orc_row *)calloc((size_t)(nq ? nq : 1), sizeof(orc_row));
    int all_agents = (qx == NULL);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < (int64_t)nq; ++i) {
        orc_center q = query_center(d, i, qx, qy, qz, px, py, pz);
        if (!q.ok) continue;
        uint64_t r2 = (uint64_t)r_fx[i] * (uint64_t)r_fx[i];
        for (uint32_t j = 0; j < n; ++j) {
            orc_center p = make_center(d, px[j], py[j], pz[j]);
            if (!p.ok) continue;
            if (all_agents && (flags & ORC_EXCLUDE_SELF) && (int64_t)j == i) continue;
            int64_t best = INT64_MAX;
            for (int sx = -1; sx <= 1; ++sx)
                for (int sy = -1; sy <= 1; ++sy)
                    for (int sz = -1; sz <= 1; ++sz) {
                        int sh[3] = {sx, sy, sz};
                        int64_t s = 0, skip = 0;
                        for (int a = 0; a < 3; ++a) {
                            if (sh[a] != 0 && !is_cyclic(d, a)) skip = 1;
                            int64_t t = p.c[a] + sh[a] * axis_width(d, a) - q.c[a];
                            s += t * t;
                        }
                        if (!skip && s < best) best = s;
                    }
            if ((uint64_t)best <= r2) row_push(&rows[i], best, j);
        }
        row_sort(&rows[i]);
    }
    return rows_to_result(rows, nq);
}

/* ------------------------------------------------------------------------ */
/* Tier 1: a plain cell grid (its own counting sort) and the bin-lattice     */
/* scan of the query's bounding cube (Section I; Section III.C for the       */
/* parallelepiped clipped to the region and the unique outside cell, II.B).  */

typedef struct {
    orc_desc d;
    uint32_t n;
    int64_t ncells;  /* cells in the region; index ncells is the outside cell */
    int64_t *start;  /* ncells + 2 */
    uint32_t *order; /* point ids grouped by cell, ascending id within a cell */
    orc_center *pts; /* normalised coordinates by id */
} orc_grid;

static int64_t grid_cell_of(const orc_desc *d, const orc_center *p) {
    int64_t c[3];
    for (int a = 0; a < 3; ++a) {
        if (!is_cyclic(d, a) && p->c[a] >= axis_width(d, a)) return -1; /* outside */
        c[a] = p->c[a] >> d->frac_bits;
    }
    return (c[2] * axis_cells(d, 1) + c[1]) * axis_cells(d, 0) + c[0];
}

orc_grid *orc_grid_build(const orc_desc *d, uint32_t n, const uint32_t *px, const uint32_t *py,
                         const uint32_t *pz) {
    orc_grid *g = (orc_grid *)calloc(1, sizeof(orc_grid));
    g->d = *d;
    g->n = n;
    g->ncells = axis_cells(d, 0) * axis_cells(d, 1) * axis_cells(d, 2);
    g->start = (int64_t *)calloc((size_t)(g->ncells + 2), sizeof(int64_t));
    g->order = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    g->pts = (orc_center *)malloc((size_t)(n ? n : 1) * sizeof(orc_center));
    int64_t *cell = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    for (uint32_t j = 0; j < n; ++j) {
        g->pts[j] = make_center(d, px[j], py[j], pz[j]);
        if (!g->pts[j].ok) {
            cell[j] = -2; /* unusable point: in no cell */
            continue;
        }
        int64_t c = grid_cell_of(d, &g->pts[j]);
        cell[j] = c < 0 ? g->ncells : c;
        g->start[cell[j] + 1]++;
    }
    for (int64_t k = 0; k < g->ncells + 1; ++k) g->start[k + 1] += g->start[k];
    int64_t *cur = (int64_t *)malloc((size_t)(g->ncells + 1) * sizeof(int64_t));
    memcpy(cur, g->start, (size_t)(g->ncells + 1) * sizeof(int64_t));
    for (uint32_t j = 0; j < n; ++j)
        if (cell[j] >= 0) g->order[cur[cell[j]]++] = j;
    free(cur);
    free(cell);
    return g;
}

void orc_grid_free(orc_grid *g) {
    if (!g) return;
    free(g->start);
    free(g->order);
    free(g->pts);
    free(g);
}

/* Cell counts per cell of the grid (ncells + 1 entries, the last being the
 * outside cell): the histogram a lattice rebuild must reproduce. */
void orc_grid_counts(const orc_grid *g, uint32_t *out) {
    for (int64_t k = 0; k < g->ncells + 1; ++k) out[k] = (uint32_t)(g->start[k + 1] - g->start[k]);
}

/* The cells of the bounding cube of a sphere, per axis: every cell index
 * between floor((q-r)/2^F) and floor((q+r)/2^F); wrapped on a cyclic axis
 * (the whole axis once when the span reaches L, so nothing repeats), and
 * clipped to [0, L) on a non-cyclic one. */
static int64_t axis_cube_cells(const orc_desc *d, int a, int64_t q, int64_t r, int64_t *list) {
    int64_t L = axis_cells(d, a), e = cell_edge(d);
    int64_t lo = floor_div(q - r, e), hi = floor_div(q + r, e), m = 0;
    if (is_cyclic(d, a)) {
        if (hi - lo + 1 >= L) {
            for (int64_t k = 0; k < L; ++k) list[m++] = k;
        } else {
            for (int64_t k = lo; k <= hi; ++k) list[m++] = floor_mod(k, L);
        }
    } else {
        if (lo < 0) lo = 0;
        if (hi > L - 1) hi = L - 1;
        for (int64_t k = lo; k <= hi; ++k) list[m++] = k;
    }
    return m;
}

/* Number of distinct cells of the bounding cube of the sphere (q, r). */
int64_t orc_cube_cells(const orc_desc *d, const uint32_t *q, uint32_t r_fx) {
    int64_t M = 0, n = 1;
    for (int a = 0; a < 3; ++a)
        if (axis_cells(d, a) + 2 > M) M = axis_cells(d, a) + 2;
    int64_t *list = (int64_t *)malloc((size_t)M * sizeof(int64_t));
    for (int a = 0; a < 3; ++a) n *= axis_cube_cells(d, a, coord_norm(d, a, q[a]), r_fx, list);
    free(list);
    return n;
}

static int any_clipped(const orc_desc *d) { return (d->cyclic_mask & 7u) != 7u; }

static void grid_scan_cell(const orc_grid *g, int64_t cell, const orc_center *q, uint64_t r2,
                           int64_t skip_id, orc_row *row) {
    for (int64_t k = g->start[cell]; k < g->start[cell + 1]; ++k) {
        uint32_t j = g->order[k];
        if ((int64_t)j == skip_id) continue;
        int64_t s = dist2(&g->d, g->pts[j].c, q->c);
        if ((uint64_t)s <= r2) row_push(row, s, j);
    }
}

static void grid_radius_one(const orc_grid *g, const orc_center *q, uint32_t r_fx, int64_t skip_id,
                            int64_t *lx, int64_t *ly, int64_t *lz, orc_row *row) {
    const orc_desc *d = &g->d;
    uint64_t r2 = (uint64_t)r_fx * (uint64_t)r_fx;
    int64_t nx = axis_cube_cells(d, 0, q->c[0], r_fx, lx);
    int64_t ny = axis_cube_cells(d, 1, q->c[1], r_fx, ly);
    int64_t nz = axis_cube_cells(d, 2, q->c[2], r_fx, lz);
    for (int64_t iz = 0; iz < nz; ++iz)
        for (int64_t iy = 0; iy < ny; ++iy)
            for (int64_t ix = 0; ix < nx; ++ix) {
                int64_t cell = (lz[iz] * axis_cells(d, 1) + ly[iy]) * axis_cells(d, 0) + lx[ix];
                grid_scan_cell(g, cell, q, r2, skip_id, row);
            }
    /* Objects outside a non-cyclic region all live in one extra cell
     * (Section II.B); the oracle simply tests them for every query. */
    if (any_clipped(d)) grid_scan_cell(g, g->ncells, q, r2, skip_id, row);
    row_sort(row);
}

static int64_t max_axis_cells(const orc_desc *d) {
    int64_t m = 0;
    for (int a = 0; a < 3; ++a)
        if (axis_cells(d, a) > m) m = axis_cells(d, a);
    return m;
}

orc_result *orc_grid_radius(const orc_grid *g, uint32_t nq, const uint32_t *qx,
                            const uint32_t *qy, const uint32_t *qz, const uint32_t *r_fx,
                            uint32_t flags) {
    const orc_desc *d = &g->d;
    orc_row *rows = (orc_row *)calloc((size_t)(nq ? nq : 1), sizeof(orc_row));
    int all_agents = (qx == NULL);
    int64_t M = max_axis_cells(d) + 2;
#pragma omp parallel
    {
        int64_t *lx = (int64_t *)malloc((size_t)M * 3 * sizeof(int64_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < (int64_t)nq; ++i) {
            orc_center q = all_agents ? g->pts[i] : make_center(d, qx[i], qy[i], qz[i]);
            if (!q.ok) continue;
            int64_t skip = (all_agents && (flags & ORC_EXCLUDE_SELF)) ? i : -1;
            grid_radius_one(g, &q, r_fx[i], skip, lx, lx + M, lx + 2 * M, &rows[i]);
        }
        free(lx);
    }
    return rows_to_result(rows, nq);
}

/* Objects of one grid cell within r of q (skip_id excluded). */
static int64_t cell_count_within(const orc_grid *g, int64_t cell, const orc_center *q, uint64_t r2,
                                 int64_t skip_id) {
    int64_t cnt = 0;
    for (int64_t k = g->start[cell]; k < g->start[cell + 1]; ++k) {
        uint32_t j = g->order[k];
        if ((int64_t)j == skip_id) continue;
        if ((uint64_t)dist2(&g->d, g->pts[j].c, q->c) <= r2) ++cnt;
    }
    return cnt;
}

/* Row sizes only: for each query, the number of objects within r (Section
 * II.A), the same cube-set scan as orc_grid_radius without keeping the
 * pairs.  out[i] = |R(q_i)|, 0 for an unusable centre.  This is what a
 * neighbour-count checksum over many queries needs, without the memory of
 * every row. */
void orc_grid_radius_counts(const orc_grid *g, uint32_t nq, const uint32_t *qx, const uint32_t *qy,
                            const uint32_t *qz, const uint32_t *r_fx, uint32_t flags, int64_t *out) {
    const orc_desc *d = &g->d;
    int all_agents = (qx == NULL);
    int64_t M = max_axis_cells(d) + 2;
#pragma omp parallel
    {
        int64_t *l = (int64_t *)malloc((size_t)M * 3 * sizeof(int64_t));
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < (int64_t)nq; ++i) {
            orc_center q = all_agents ? g->pts[i] : make_center(d, qx[i], qy[i], qz[i]);
            out[i] = 0;
            if (!q.ok) continue;
            int64_t skip = (all_agents && (flags & ORC_EXCLUDE_SELF)) ? i : -1;
            uint64_t r2 = (uint64_t)r_fx[i] * (uint64_t)r_fx[i];
            int64_t nx = axis_cube_cells(d, 0, q.c[0], r_fx[i], l);
            int64_t ny = axis_cube_cells(d, 1, q.c[1], r_fx[i], l + M);
            int64_t nz = axis_cube_cells(d, 2, q.c[2], r_fx[i], l + 2 * M);
            int64_t cnt = 0;
            for (int64_t iz = 0; iz < nz; ++iz)
                for (int64_t iy = 0; iy < ny; ++iy)
                    for (int64_t ix = 0; ix < nx; ++ix) {
                        int64_t cell = (l[2 * M + iz] * axis_cells(d, 1) + l[M + iy]) * axis_cells(d, 0) + l[ix];
                        cnt += cell_count_within(g, cell, &q, r2, skip);
                    }
            /* objects outside a non-cyclic region: the one outside cell */
            if (any_clipped(d)) cnt += cell_count_within(g, g->ncells, &q, r2, skip);
            out[i] = cnt;
        }
        free(l);
    }
}

/* ------------------------------------------------------------------------ */
/* K nearest (Section II.A, last paragraph): the first min(K, |R|) entries   */
/* of the radius result R at the search cap rmax, in (dist2, id) order.      */

/* Tier 0: sort every candidate within rmax and truncate. */
orc_result *orc_knn_brute(const orc_desc *d, uint32_t n, const uint32_t *px, const uint32_t *py,
                          const uint32_t *pz, uint32_t nq, const uint32_t *qx, const uint32_t *qy,
                          const uint32_t *qz, const uint32_t *k, const uint32_t *rmax_fx,
                          uint32_t flags) {
    orc_result *full = orc_radius_brute(d, n, px, py, pz, nq, qx, qy, qz, rmax_fx, flags);
    orc_row *rows = (orc_row *)calloc((size_t)(nq ? nq : 1), sizeof(orc_row));
    for (int64_t i = 0; i < (int64_t)nq; ++i) {
        int64_t b = full->row_ptr[i], e = full->row_ptr[i + 1];
        int64_t m = e - b < (int64_t)k[i] ? e - b : (int64_t)k[i];
        for (int64_t t = 0; t < m; ++t) row_push(&rows[i], full->d2[b + t], full->ids[b + t]);
    }
    orc_result_free(full);
    return rows_to_result(rows, nq);
}

/* Tier 1: grow a search radius rho (1 cell, doubling, capped at rmax) until
 * at least K objects lie within rho or rho = rmax.  Every object closer than
 * the K-th one is within rho, so the prefix of R_rho is the prefix of R_rmax. */
orc_result *orc_grid_knn(const orc_grid *g, uint32_t nq, const uint32_t *qx, const uint32_t *qy,
                         const uint32_t *qz, const uint32_t *k, const uint32_t *rmax_fx,
                         uint32_t flags) {
    const orc_desc *d = &g->d;
    orc_row *rows = (orc_row *)calloc((size_t)(nq ? nq : 1), sizeof(orc_row));
    int all_agents = (qx == NULL);
    int64_t M = max_axis_cells(d) + 2;
#pragma omp parallel
    {
        int64_t *lx = (int64_t *)malloc((size_t)M * 3 * sizeof(int64_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < (int64_t)nq; ++i) {
            orc_center q = all_agents ? g->pts[i] : make_center(d, qx[i], qy[i], qz[i]);
            if (!q.ok || k[i] == 0) continue;
            int64_t skip = (all_agents && (flags & ORC_EXCLUDE_SELF)) ? i : -1;
            uint64_t rho = (uint64_t)cell_edge(d);
            orc_row tmp = {0, 0, 0};
            for (;;) {
                uint32_t re = rho >= rmax_fx[i] ? rmax_fx[i] : (uint32_t)rho;
                tmp.n = 0;
                grid_radius_one(g, &q, re, skip, lx, lx + M, lx + 2 * M, &tmp);
                if (tmp.n >= (int64_t)k[i] || re == rmax_fx[i]) break;
                rho *= 2;
            }
            int64_t m = tmp.n < (int64_t)k[i] ? tmp.n : (int64_t)k[i];
            for (int64_t t = 0; t < m; ++t) row_push(&rows[i], tmp.v[t].d2, tmp.v[t].id);
            free(tmp.v);
        }
        free(lx);
    }
    return rows_to_result(rows, nq);
}

/* Mixed batch: query i is a K-NN query with cap r_fx[i] when k[i] > 0,
 * otherwise a radius query with radius r_fx[i]. */
orc_result *orc_grid_mixed(const orc_grid *g, uint32_t nq, const uint32_t *qx, const uint32_t *qy,
                           const uint32_t *qz, const uint32_t *k, const uint32_t *r_fx,
                           uint32_t flags) {
    orc_result *rad = orc_grid_radius(g, nq, qx, qy, qz, r_fx, flags);
    orc_result *nn = orc_grid_knn(g, nq, qx, qy, qz, k, r_fx, flags);
    orc_row *rows = (orc_row *)calloc((size_t)(nq ? nq : 1), sizeof(orc_row));
    for (int64_t i = 0; i < (int64_t)nq; ++i) {
        const orc_result *src = k[i] > 0 ? nn : rad;
        for (int64_t t = src->row_ptr[i]; t < src->row_ptr[i + 1]; ++t)
            row_push(&rows[i], src->d2[t], src->ids[t]);
    }
    orc_result_free(rad);
    orc_result_free(nn);
    return rows_to_result(rows, nq);
}

/* ------------------------------------------------------------------------ */
/* Cells touched by one query (Sections I, II.A, III.A).                     */
/* For each cell u of the bounding cube (unwrapped indices, clipped to the   */
/* region on non-cyclic axes): the minimum squared distance from q to the    */
/* cell's positions and the maximum one.  kept = cells with min <= r^2       */
/* (the cells the sphere intersects), interior = cells with max <= r^2       */
/* (wholly inside), cube = all cells of the clipped cube.  On a cyclic axis  */
/* the radius must satisfy ceil(r / 2^F) <= L/2 - 1 so that no cell repeats; */
/* queries violating this get -1.                                            */

static int64_t gap_lo(int64_t q, int64_t u, int64_t e) {
    int64_t lo = u * e, hi = u * e + e - 1;
    int64_t g = 0;
    if (lo - q > g) g = lo - q;
    if (q - hi > g) g = q - hi;
    return g;
}

static int64_t gap_hi(int64_t q, int64_t u, int64_t e) {
    int64_t lo = u * e, hi = u * e + e - 1;
    int64_t a = q - lo, b = hi - q;
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    return a > b ? a : b;
}

void orc_cells_touched(const orc_desc *d, uint32_t nq, const uint32_t *qx, const uint32_t *qy,
                       const uint32_t *qz, const uint32_t *r_fx, int64_t *kept, int64_t *interior,
                       int64_t *cube) {
    int64_t e = cell_edge(d);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < (int64_t)nq; ++i) {
        orc_center q = make_center(d, qx[i], qy[i], qz[i]);
        int64_t r = r_fx[i];
        uint64_t r2 = (uint64_t)r * (uint64_t)r;
        int64_t lo[3], hi[3], bad = !q.ok;
        for (int a = 0; a < 3; ++a) {
            lo[a] = floor_div(q.c[a] - r, e);
            hi[a] = floor_div(q.c[a] + r, e);
            if (is_cyclic(d, a)) {
                int64_t m = (r + e - 1) / e;
                if (m > axis_cells(d, a) / 2 - 1) bad = 1;
            } else {
                if (lo[a] < 0) lo[a] = 0;
                if (hi[a] > axis_cells(d, a) - 1) hi[a] = axis_cells(d, a) - 1;
            }
        }
        if (bad) {
            kept[i] = interior[i] = cube[i] = -1;
            continue;
        }
        int64_t nk = 0, ni = 0, nc = 0;
        for (int64_t uz = lo[2]; uz <= hi[2]; ++uz)
            for (int64_t uy = lo[1]; uy <= hi[1]; ++uy)
                for (int64_t ux = lo[0]; ux <= hi[0]; ++ux) {
                    int64_t u[3] = {ux, uy, uz};
                    uint64_t mn = 0, mx = 0;
                    for (int a = 0; a < 3; ++a) {
                        int64_t g0 = gap_lo(q.c[a], u[a], e), g1 = gap_hi(q.c[a], u[a], e);
                        mn += (uint64_t)(g0 * g0);
                        mx += (uint64_t)(g1 * g1);
                    }
                    nc++;
                    if (mn <= r2) nk++;
                    if (mx <= r2) ni++;
                }
        kept[i] = nk;
        interior[i] = ni;
        cube[i] = nc;
    }
}

/* ------------------------------------------------------------------------ */
/* Sphere-table keys (Section II.A, Fig. 2; Section III.A, Fig. 3).          */

/* Fig. 2's bound in cell units: a cell offset by o_i along each axis is at
 * least max(|o_i| - 1, 0) cells away along that axis from any position of
 * the centre cell, so the squared bound is the sum of their squares. */
int64_t orc_base_minbound2(int dim, const int32_t *o) {
    int64_t s = 0;
    for (int i = 0; i < dim; ++i) {
        int64_t a = o[i] < 0 ? -(int64_t)o[i] : o[i];
        int64_t b = a > 0 ? a - 1 : 0;
        s += b * b;
    }
    return s;
}

/* Fixed-point key of offset o for sub-cell class `cls` (s bits per axis):
 * the class box along an axis holds positions [c*w, (c+1)*w - 1] of the
 * centre cell, w = 2^(F-s).  Nearest position of the target cell:
 *   o > 0: o*2^F - ((c+1)*w - 1)      (target's first position, box's last)
 *   o < 0: c*w + (|o|-1)*2^F + 1      (box's first position, target's last)
 *   o = 0: 0.                                                              */
int64_t orc_table_key(uint32_t F, uint32_t s, const uint32_t *cls, const int32_t *o) {
    int64_t e = (int64_t)1 << F, w = (int64_t)1 << (F - s), key = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t c = cls[a], g;
        if (o[a] > 0)
            g = (int64_t)o[a] * e - ((c + 1) * w - 1);
        else if (o[a] < 0)
            g = c * w + (-(int64_t)o[a] - 1) * e + 1;
        else
            g = 0;
        if (g < 0) g = 0;
        key += g * g;
    }
    return key;
}

/* The same key by exhaustion over every position of the class box
 * (only for small F). */
int64_t orc_table_key_brute(uint32_t F, uint32_t s, const uint32_t *cls, const int32_t *o) {
    int64_t e = (int64_t)1 << F, w = (int64_t)1 << (F - s);
    int64_t best = INT64_MAX;
    for (int64_t qz = cls[2] * w; qz < (cls[2] + 1) * w; ++qz)
        for (int64_t qy = cls[1] * w; qy < (cls[1] + 1) * w; ++qy)
            for (int64_t qx = cls[0] * w; qx < (cls[0] + 1) * w; ++qx) {
                int64_t q[3] = {qx, qy, qz}, s2 = 0;
                for (int a = 0; a < 3; ++a) {
                    int64_t g = gap_lo(q[a], o[a], e);
                    s2 += g * g;
                }
                if (s2 < best) best = s2;
            }
    return best;
}

/* All offsets o with key <= r^2 for one class, by enumerating the cube
 * [-(m+1), m+1]^3, m = ceil(r / 2^F).  Returns the count; when `out` is not
 * NULL it receives (ox, oy, oz) triples and `keys` the keys, in enumeration
 * order (z slowest, x fastest). */
int64_t orc_table_set(uint32_t F, uint32_t s, const uint32_t *cls, uint32_t r_fx, int32_t *out,
                      int64_t *keys) {
    int64_t e = (int64_t)1 << F;
    int64_t m = ((int64_t)r_fx + e - 1) / e + 1;
    uint64_t r2 = (uint64_t)r_fx * (uint64_t)r_fx;
    int64_t cnt = 0;
    for (int64_t z = -m; z <= m; ++z)
        for (int64_t y = -m; y <= m; ++y)
            for (int64_t x = -m; x <= m; ++x) {
                int32_t o[3] = {(int32_t)x, (int32_t)y, (int32_t)z};
                int64_t k = orc_table_key(F, s, cls, o);
                if ((uint64_t)k <= r2) {
                    if (out) {
                        out[3 * cnt + 0] = o[0];
                        out[3 * cnt + 1] = o[1];
                        out[3 * cnt + 2] = o[2];
                    }
                    if (keys) keys[cnt] = k;
                    cnt++;
                }
            }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Counter-based generator (SplitMix64 finaliser, Steele, Lea and Flood,     */
/* OOPSLA 2014) for the moving-agent workload, and the count checksum.       */

uint64_t orc_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_hash(uint64_t seed, uint64_t tag, uint64_t i) {
    return orc_mix64(seed ^ orc_mix64((tag << 40) ^ i));
}

/* Agents move (dynamic objects, Section I): each coordinate of agent i at
 * step t is displaced by delta in [-2^F/4, 2^F/4] drawn from
 * hash(seed, 1000 + 3t + axis, i), then wrapped (cyclic) or clamped. */
void orc_move(const orc_desc *d, uint64_t seed, uint32_t step, uint32_t n, uint32_t *x,
              uint32_t *y, uint32_t *z) {
    int64_t dmax = cell_edge(d) / 4;
    uint32_t *v[3] = {x, y, z};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        for (int a = 0; a < 3; ++a) {
            uint64_t h = orc_hash(seed, 1000u + 3u * (uint64_t)step + (uint64_t)a, (uint64_t)i);
            int64_t delta = (int64_t)(((h >> 32) * (uint64_t)(2 * dmax + 1)) >> 32) - dmax;
            int64_t w = axis_width(d, a);
            int64_t nv = (int64_t)v[a][i] + delta;
            if (is_cyclic(d, a))
                nv = floor_mod(nv, w);
            else
                nv = nv < 0 ? 0 : (nv > w - 1 ? w - 1 : nv);
            v[a][i] = (uint32_t)nv;
        }
    }
}

/* Order-independent checksum of per-row counts: out[0] = sum of counts,
 * out[1] = sum over rows of mix64((i << 32) | count_i) (mod 2^64). */
void orc_count_checksum(const int64_t *row_ptr, uint32_t nq, uint64_t *out) {
    uint64_t s = 0, h = 0;
    for (int64_t i = 0; i < (int64_t)nq; ++i) {
        uint64_t c = (uint64_t)(row_ptr[i + 1] - row_ptr[i]);
        s += c;
        h += orc_mix64(((uint64_t)i << 32) | (c & 0xffffffffULL));
    }
    out[0] = s;
    out[1] = h;
}
