/*
 * sphidx.h -- C ABI of libsphidx: spherical-indexing neighbourhood queries
 * (N. Brodu, "Spherical Indexing for Neighborhood Queries", arXiv
 * cs/0608108) on one AMD Instinct MI355X (gfx950).
 *
 * Conventions for every entry point:
 *   - "dev" pointers are device memory (for instance torch.Tensor.data_ptr()
 *     of a CUDA/HIP tensor), "host" pointers are host memory.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *   - A call validates its host-visible arguments synchronously, enqueues its
 *     kernels on `stream` and returns without synchronising, unless its
 *     comment says otherwise.  Argument errors are returned as a status and
 *     nothing is enqueued.
 *   - Conditions found in device arrays (coordinates out of range, output
 *     capacity exceeded) set bits of the lattice's device status word, read
 *     with sphidx_lattice_status().  The affected rows are left empty; no
 *     out-of-bounds write happens.
 *   - The caller owns every device buffer it passes (coordinates, queries,
 *     outputs, workspaces).  The library owns only the opaque handles and the
 *     sphere-table storage.  No C++ type or exception crosses the ABI.
 *
 * Geometry (Section II.B): a lattice of 2^log2_cells[a] cubic cells per axis,
 * each cell 2^frac_bits fixed-point units wide, each axis cyclic or clipped.
 * Coordinates are uint32 fixed point.  On a cyclic axis any value is accepted
 * and reduced modulo the world width W_a = 2^(log2_cells[a] + frac_bits); on
 * a clipped axis values must be below 2^30; values >= W_a lie outside the
 * region of interest and are kept in the one "outside" cell (Section II.B,
 * non-cyclic case), whose index is the number of region cells.
 *
 * Query semantics (Section II.A): the neighbours of centre q for radius r are
 * the objects p with |p - q| <= r (inclusive), distances measured with the
 * minimum image on cyclic axes; each object appears at most once.  The K
 * nearest are the first min(K, |R|) of those within the search cap r.  Every
 * output row lists ids ordered by (squared distance, id) ascending; squared
 * distances are exact int64 in fixed-point units^2.
 */
#ifndef SPHIDX_H
#define SPHIDX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPHIDX_OK = 0,
    SPHIDX_ERR_INVALID_ARG = 1,   /* bad pointer, size or descriptor */
    SPHIDX_ERR_RANGE = 2,         /* coordinate out of the accepted range (device-detected) */
    SPHIDX_ERR_RADIUS = 3,        /* radius beyond what the call accepts */
    SPHIDX_ERR_CAPACITY = 4,      /* output or workspace too small */
    SPHIDX_ERR_OUT_OF_MEMORY = 5, /* library-owned allocation failed */
    SPHIDX_ERR_DEVICE = 6,        /* a HIP call failed */
    SPHIDX_ERR_IO = 7             /* table file missing, truncated or corrupt */
} sphidx_status;

/* Device status word bits (sphidx_lattice_status). */
#define SPHIDX_FLAG_RANGE 1u    /* a clipped-axis coordinate >= 2^30 was seen; that point/query was skipped */
#define SPHIDX_FLAG_CAPACITY 2u /* row_ptr[Q] exceeded csr.capacity; the write pass wrote nothing */
#define SPHIDX_FLAG_FALLBACK 4u /* informational: some queries used the cube scan (radius beyond the
                                   tables' cap or the cyclic limit, or centre outside the region) */

/* ---------------------------------------------------------------------- */
/* Lattice (Section II.B): power-of-two cells per axis, per-axis cyclicity. */

typedef struct {
    uint32_t log2_cells[3]; /* 0..10 per axis; sum <= 30 */
    uint32_t frac_bits;     /* F: cell edge = 2^F units; F + log2_cells[a] <= 30 */
    uint32_t cyclic_mask;   /* bit a set: axis a wraps (minimum image) */
} sphidx_lattice_desc;

typedef struct sphidx_lattice sphidx_lattice; /* opaque, host-side handle */
typedef struct sphidx_tables sphidx_tables;   /* opaque, host-side handle */

/* Device workspace needed by a lattice of up to max_points objects. */
size_t sphidx_lattice_workspace_bytes(const sphidx_lattice_desc* desc, uint32_t max_points);

/* Bind a lattice handle to a caller-owned device workspace (>= the size
 * above, 256-byte aligned).  Returns INVALID_ARG for a descriptor outside the
 * limits, CAPACITY for a short workspace.  Synchronous; launches nothing. */
sphidx_status sphidx_lattice_create(const sphidx_lattice_desc* desc, uint32_t max_points,
                                    void* workspace_dev, size_t workspace_bytes,
                                    sphidx_lattice** out);
void sphidx_lattice_destroy(sphidx_lattice* lat);

/* Rebuild the cell lists from n objects (dev x, y, z: uint32[n]) as a
 * counting sort: cell-id histogram, exclusive scan, scatter of one 16-byte
 * record {x, y, z, id} per object in packed-cell order (each object is in
 * exactly one cell, Section I).  Object ids are their input indices.  Objects with a clipped-axis coordinate >= 2^30 set
 * SPHIDX_FLAG_RANGE and are left out.  n <= max_points.  The lattice must not
 * be read by queries still in flight on other streams. */
sphidx_status sphidx_build_lattice(sphidx_lattice* lat, const uint32_t* x_dev, const uint32_t* y_dev,
                                   const uint32_t* z_dev, uint32_t n, void* stream);

/* Device views of the lattice, for inspection: cell_start has ncells + 3
 * entries (region cells, then the outside cell, then the cell of skipped
 * objects), cell k holding sorted positions [cell_start[k], cell_start[k+1]);
 * points holds 4 uint32 per sorted position: the normalised x, y, z and the
 * object id.  Valid after the build's kernels complete. */
typedef struct {
    const uint32_t* cell_start;
    const uint32_t* points;
    uint32_t n;
    uint32_t ncells;
} sphidx_lattice_view;
sphidx_status sphidx_lattice_get_view(const sphidx_lattice* lat, sphidx_lattice_view* out);

/* The non-empty cell list (Section III.B): the region cells that hold at
 * least one object, in increasing packed-cell order.  A caller-owned buffer
 * of at least sphidx_cell_list_bytes(lat) bytes (256-byte aligned) holds
 *   bytes [0, 4):   uint32 count
 *   bytes [16, ..): count + 1 entries {uint32 cell, uint32 first}: the packed
 *                   cell index and the sorted position of its first object;
 *                   the last entry is {0xFFFFFFFF, cell_start[ncells]}, so
 *                   entry j's objects are [first_j, first_{j+1}).
 * Attaching enqueues the list of the current contents on `stream`; from then
 * on every sphidx_build_lattice rebuilds it after the cell lists, in stream
 * order.  list_dev = NULL detaches (no list kept; METHOD_AUTO stops choosing
 * it).  The buffer must outlive the attachment. */
size_t sphidx_cell_list_bytes(const sphidx_lattice* lat);
sphidx_status sphidx_lattice_attach_cell_list(sphidx_lattice* lat, void* list_dev, size_t bytes, void* stream);

/* Order of the objects inside each cell after a build.  ANY: the order the
 * counting sort's atomics give (the default).  X: by x coordinate, then id,
 * for every cell of at most 4,096 objects; queries then narrow a row of
 * cells with many objects to those whose x lies within the sphere's x-slab
 * on that row, by a search on the sorted x values, instead of testing every
 * object of the row's cells (results are the same; the order costs one more
 * pass of the build, quadratic in a cell's objects).  A build that finds a
 * larger cell keeps it in the counting sort's order and queries then test
 * whole rows.  Applies to sphidx_build_lattice; sphidx_move_resident and
 * sphidx_move_incremental leave cells unordered.  INVALID_ARG for another
 * value.  Host only; the order is made by the next build, and queries narrow
 * rows only while the order set is X and the last build ordered every cell.
 * The first call with X allocates a second record array of 16 bytes per
 * point (max_points), which the build's counting sort fills before the x
 * ranking writes each record into the lattice; the library owns it and
 * sphidx_lattice_destroy frees it (OUT_OF_MEMORY when it cannot be had). */
#define SPHIDX_ORDER_ANY 0u
#define SPHIDX_ORDER_X 1u
sphidx_status sphidx_lattice_set_cell_order(sphidx_lattice* lat, uint32_t order);

/* Synchronise `stream`, return the device status word in *flags_out (may be
 * NULL) and clear it.  Returns RANGE or CAPACITY when those bits were set. */
sphidx_status sphidx_lattice_status(sphidx_lattice* lat, void* stream, uint32_t* flags_out);

/* The same by stream: synchronise `stream`, then read and clear the status
 * words of every lattice that calls on this stream (builds, moves, queries,
 * cell-list attachment) have touched since the last sphidx_stream_status
 * for it, and return their bits OR-ed in *flags_out (may be NULL).  Returns
 * RANGE or CAPACITY when those bits were set, DEVICE when a HIP call fails.
 * A destroyed lattice is forgotten.  Thread-safe. */
sphidx_status sphidx_stream_status(void* stream, uint32_t* flags_out);

/* ---------------------------------------------------------------------- */
/* Sphere tables (Section II.A; sub-cell specialisation, Section III.A).    */
/*                                                                          */
/* For each sub-cell class (subcell_bits s per axis: the query's position    */
/* inside its cell, truncated to s bits per axis) the table lists every cell */
/* offset o whose key -- the minimum squared distance from any position of  */
/* the class box to the nearest position of cell o -- is <= rmax_fx^2,      */
/* sorted by increasing key.  A query of radius r <= rmax walks the prefix  */
/* with key <= r^2, centre to edge (Section II.A).                          */

/* Build on the host and upload (allocates device memory; synchronous).
 * s <= 3 and s <= frac_bits; rmax_fx <= 2^31 - 2^(frac_bits+2); the
 * offset bound ceil(rmax/2^F) + 1 must be <= 511. */
sphidx_status sphidx_build_sphere_tables(const sphidx_lattice_desc* desc, uint32_t subcell_bits,
                                         uint32_t rmax_fx, sphidx_tables** out);
void sphidx_tables_destroy(sphidx_tables* tab);

typedef struct {
    uint32_t subcell_bits;
    uint32_t frac_bits;
    uint32_t rmax_fx;
    uint32_t nclasses;      /* 2^(3s) */
    uint64_t total_entries; /* over all classes */
    uint64_t device_bytes;
} sphidx_tables_info;
sphidx_status sphidx_tables_get_info(const sphidx_tables* tab, sphidx_tables_info* out);

/* Copy class `cls`'s entries to host: offsets_host int32[3*n] as (ox, oy, oz)
 * triples, keys_host int64[n] (either may be NULL).  *n_inout holds the
 * capacity on entry and the class's entry count on return; CAPACITY if short. */
sphidx_status sphidx_tables_export(const sphidx_tables* tab, uint32_t cls, int32_t* offsets_host,
                                   int64_t* keys_host, uint64_t* n_inout);

/* Save/load (Section II.A: the table may come from an external file).  The
 * file holds a header (magic, version, s, F, rmax), the entries and a 64-bit
 * checksum; load returns IO for a missing, truncated or corrupt file. */
sphidx_status sphidx_tables_save(const sphidx_tables* tab, const char* path);
sphidx_status sphidx_tables_load(const char* path, sphidx_tables** out);

/* Table designs compared (host only; Section II.A, III.A).  For nq query
 * positions inside the home cell (fx, fy, fz < 2^F, host arrays) and radii
 * r <= the tables' cap (and <= 31 cells), out_host[7*i + k] (uint64) counts
 * the cells query i walks under each design:
 *   0 the bin-lattice bounding cube (exact to the sub-cell);
 *   1 the unshaved table: entries b^2 = sum max(|o|-1, 0)^2 <= floor(d^2),
 *     d = r / 2^F;
 *   2 the paper's 64 specialised tables: the unshaved entries below floor(d)^2,
 *     then, up to floor(d^2), the table chosen by the six bits
 *     [frac(d) < zeta] (zeta = 2^F - f up, f down), which leaves out each cell
 *     with an axis at b_o = floor(b) in a flagged direction (the one-direction
 *     rule) or moving along some axis with all its directions flagged (Eq. 2);
 *   3 those left after the run-time test of Eq. 1 on the cells at or above
 *     d - 1;
 *   4 the prefix key <= r^2 of `tab`'s sub-cell class (this library's tables);
 *   5 the exact set: cells holding an integer position within r;
 *   6 exact cells that design 3 leaves out (always 0: the paper's tests are
 *     conservative for integer positions).
 * RADIUS when a radius exceeds those limits. */
sphidx_status sphidx_table_census(const sphidx_tables* tab, uint32_t nq, const uint32_t* fx_host,
                                  const uint32_t* fy_host, const uint32_t* fz_host, const uint32_t* r_host,
                                  uint64_t* out_host);

/* The sub-cell class tables in `dims` = 2, 3 or 4 dimensions (Section I: the
 * method generalises; Section V: more dimensions): over the 2^(dims*s) classes
 * of s sub-cell bits per axis, the mean number of cells whose key (the
 * smallest squared distance from the class box, integer positions) is <= r^2
 * (*sphere_cells) and of the bounding box exact to the class (*cube_cells).
 * Their ratio tends to the ball/cube volume ratio (pi/4, pi/6, pi^2/32).
 * With hist_len > 0, unshaved_hist[k] (k < hist_len) receives the number of
 * cells of the unshaved table (Section II.A) with entry b^2 = k.  RADIUS when
 * the enumeration would exceed 2^34 cell visits. */
sphidx_status sphidx_table_census_nd(uint32_t dims, uint32_t frac_bits, uint32_t subcell_bits, uint32_t r_fx,
                                     double* sphere_cells, double* cube_cells, uint64_t* unshaved_hist,
                                     uint32_t hist_len);

/* ---------------------------------------------------------------------- */
/* Queries.                                                                */

#define SPHIDX_MODE_RADIUS 0u /* every query: all objects within radius_fx */
#define SPHIDX_MODE_KNN 1u    /* every query: K nearest within the cap radius_fx */
#define SPHIDX_MODE_MIXED 2u  /* query i: K-NN when k_i > 0, else radius */

#define SPHIDX_EXCLUDE_SELF 1u /* all-agents mode: leave out the query's own id */

typedef struct {
    uint32_t count;          /* Q */
    const uint32_t* x_dev;   /* query centres (uint32[Q] each); all NULL = all agents: */
    const uint32_t* y_dev;   /*   query i is object i of the lattice (Q must equal its n) */
    const uint32_t* z_dev;
    const uint32_t* radius_fx_dev; /* per-query radius (K-NN: search cap); NULL = use radius_fx */
    uint32_t radius_fx;
    const uint32_t* k_dev; /* per-query K; NULL = use k */
    uint32_t k;
    uint32_t mode;  /* SPHIDX_MODE_* */
    uint32_t flags; /* SPHIDX_EXCLUDE_SELF */
} sphidx_queries;

typedef struct {
    int64_t* row_ptr_dev; /* Q + 1 entries */
    uint32_t* ids_dev;    /* capacity entries */
    int64_t* dist2_dev;   /* capacity entries, or NULL when not wanted */
    int64_t capacity;     /* entries available in ids (and dist2) */
    void* workspace_dev;  /* at least sphidx_query_workspace_bytes(Q) bytes, 256-byte aligned; */
    size_t workspace_bytes; /* bytes beyond that minimum are the stash (below) */
} sphidx_csr;

/* The stash.  Workspace bytes beyond the minimum let the count pass keep
 * each radius row of at most sort_cap objects, and each K-NN row of K <= 64
 * (searched there to the end), already sorted, so that the write pass copies
 * it into place instead of walking the tables again.  A
 * row needs 4 bytes per object (12 when the count call passes dist2_dev).
 * Rows that do not fit are walked again by the write pass, so any size is
 * correct; sphidx_query_stash_bytes gives the size that keeps every row.
 * The write pass must use the workspace the count pass used, unchanged.
 * Only the persistent schedule stashes (a plain launch's waves are too
 * short-lived to fill allocation chunks). */
size_t sphidx_query_stash_bytes(uint64_t pairs, int want_dist2);

#define SPHIDX_METHOD_SPHERE 0u /* sphere-table walk (falls back to the cube where the tables do not apply) */
#define SPHIDX_METHOD_CUBE 1u   /* bin-lattice bounding-cube scan: the paper's baseline */
#define SPHIDX_METHOD_AUTO 2u   /* per query, the walk with the fewest cells (Section III.B, III.C):
                                   the sphere table (cells of its prefix for the query's sub-cell class
                                   and radius), the bounding cube clipped to the region, or the lattice's
                                   non-empty cell list when one is attached; see select_weight and the
                                   reversal distances below.  Needs tables. */
#define SPHIDX_METHOD_LIST 3u   /* every query walks the non-empty cell list (needs an attached list;
                                   tables unused) */
#define SPHIDX_METHOD_PAPER64 4u /* the paper's own table design (Section III.A): per cell entries
                                   sorted by b^2 = sum max(|o|-1, 0)^2, the unshaved table below
                                   floor(d)^2 and, up to floor(d^2), one of 64 tables specialised on
                                   the six flags [frac(d) < zeta] (zeta = e - f up, f down), which leave
                                   out ahead of time the cells the one-direction rule and Eq. 2
                                   reject; the run-time test of Eq. 1 on the cells at or above d - 1;
                                   every object of a kept cell tested.  One cell per lane, one query
                                   per wavefront (grouped ignored, no LDS staging).  Needs tables whose
                                   cap is at most 31 cells (RADIUS otherwise); queries the tables do
                                   not serve take the cube scan, as with SPHERE.  For comparing the
                                   designs: the row walk of SPHERE keeps exactly the same cells' objects
                                   with fewer, longer rows */

#define SPHIDX_SCHED_PLAIN 0u      /* one launch, each wave owns a fixed slice of queries */
#define SPHIDX_SCHED_PERSISTENT 1u /* resident waves pull query tiles from per-XCD work queues */

typedef struct {
    uint32_t method;          /* SPHIDX_METHOD_* */
    uint32_t schedule;        /* SPHIDX_SCHED_* */
    uint32_t waves_per_block; /* 1, 2 or 4; 0 = default (4) */
    uint32_t tile;            /* queries per wave slice / per queue grab; 0 = default */
    uint32_t blocks_per_cu;   /* persistent residency; 0 = default */
    uint32_t sort_cap;        /* per-wave LDS row buffer (64, 128 or 256); longer rows take the
                                 windowed top-M path; 0 = 256 */
    uint32_t table_in_lds;    /* 1: stage the whole row table in LDS (CAPACITY if it does not fit);
                                 2: stage in chunks: the first rows of every (y, z) class table, as
                                 many as fit the LDS beside the passes' buffers (CAPACITY below 16),
                                 the rest read from device memory */
    uint32_t interior;        /* count pass, sphere method: 0 = auto (on when objects per cell >= 1),
                                 1 = off, 2 = on: cells wholly inside the sphere are counted whole */
    uint32_t* stats_dev; /* optional uint32[4*Q], zeroed by the caller: per query, the count
                            pass adds the table entries (rows) walked, the cells kept and the
                            candidate objects tested, over every walk the query took (a grouped
                            K-NN row searched again, a K-NN search restarted at a larger bound),
                            and stores the bounding cube's cells.  Costs atomics: for
                            measurement, not for timed runs */
    void* event_begin;   /* optional hipEvent_t, recorded on the stream just before the pass's main
                            kernel (count pass: the count kernel; write pass: the stash copy and
                            the write kernel, or the top-K kernel when every row is K-NN) */
    void* event_end;     /* optional hipEvent_t, recorded just after that kernel (neither event is
                            recorded when Q = 0) */
    uint32_t no_stash;   /* 1: never keep rows in the workspace stash (see sphidx_csr) */
    uint32_t grouped;    /* 1: the count pass takes radius queries in groups of several per
                            wavefront (persistent schedule), and K-NN queries of the sphere
                            tables with 2K <= sort_cap as radius rows at a first search
                            radius (expected to hold min(1.7K, K + 3 sqrt(K) + 3) objects),
                            keeping the first K when it holds K (rows short of K are searched
                            again in groups at a larger radius, then one query per
                            wavefront; the stash needs K pairs per such row);
                            0: one query per wavefront */
    /* METHOD_AUTO (Appendix: weighting factor and reversal distances).  A radius query takes
     * the sphere when select_weight/256 * (sphere cells) <= (cube cells), else the cube; then
     * the non-empty list instead if it holds fewer cells than the one chosen (plain counts).
     * (Model 0 below; model 1 compares estimated work instead of cells.)
     * Sphere cells: the entries of the query's sub-cell class with key <= (j * 2^b)^2,
     * j = ceil(r / 2^b), b = max(F - 6, 0) -- the one lookup of the radius index.  Cube
     * cells: the bounding cube's cells inside the region (the whole axis once it spans it).
     * K-NN queries take the sphere or, below knn_reversal_fx, the cube (their final radius is
     * not known in advance, Section IV.B).  Queries the tables cannot serve choose between the
     * cube and the list. */
    uint32_t select_weight;   /* Q8 fixed point; 0 = 256 (the plain volume comparison) */
    uint32_t reversal_fx;     /* radius queries with r < reversal_fx never take the sphere; 0 = off */
    uint32_t knn_reversal_fx; /* K-NN queries with cap < knn_reversal_fx take the cube; 0 = off */
    uint32_t select_model;    /* what the comparisons count: 0 = cells (the paper's volumes);
                                 1 = estimated lane work of each walk: the rows it visits (sphere:
                                 table rows with key <= (j * 2^b)^2, i.e. cells of that prefix with
                                 ox = 0; cube: its y-z rows; list: its entries) plus the mean objects
                                 per region cell times the cells whose objects it tests (sphere and
                                 list: floor(sphere cells * cube cells / unclipped cube cells), or
                                 the cube cells when the sphere is left out; cube: the cube cells),
                                 in 1/256 units with the mean taken as
                                 min(floor(256 * n / region cells), 2^24); the unclipped cube spans
                                 floor((q - r) / 2^F) .. floor((q + r) / 2^F) per axis, at most the
                                 axis on a cyclic one */
    uint32_t* method_dev;     /* optional uint32[Q], written by the count pass: the walk each query
                                 used (SPHIDX_METHOD_SPHERE, _CUBE or _LIST), or 0xFFFFFFFF for a
                                 query with an empty row by definition (invalid centre, K = 0) */
    uint32_t long_row_waves;  /* write pass, radius rows longer than sort_cap and at most 3072 pairs:
                                 the wavefronts that walk and order one such row together, as one
                                 block (2, 4 or 8; 0 = 4); 1 = one wavefront per row, which takes
                                 the row in windows of sort_cap, walking it once per window */
} sphidx_launch;

/* Bytes of device scratch a query call on Q queries needs. */
size_t sphidx_query_workspace_bytes(uint32_t Q);

/* Pass 1: per-query row sizes, then an exclusive scan into row_ptr (so
 * row_ptr[Q] = total pairs).  For K-NN rows the size is min(K, objects
 * within the cap).  `tab` may be NULL with method CUBE.  `launch` may be
 * NULL for the defaults (sphere, persistent).  Outputs other than row_ptr
 * are untouched. */
sphidx_status sphidx_count(const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                           sphidx_csr* csr, const sphidx_launch* launch, void* stream);

/* Pass 2: fill ids (and dist2) of every row using row_ptr and the query
 * descriptors and lists that sphidx_count left in the workspace: same
 * inputs, same launch method, same workspace, unchanged in between.  If
 * row_ptr[Q] > capacity it sets SPHIDX_FLAG_CAPACITY and writes nothing
 * (checked on the device, so it can run under capture). */
sphidx_status sphidx_write(const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                           sphidx_csr* csr, const sphidx_launch* launch, void* stream);

/* Both passes. */
sphidx_status sphidx_query(const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                           sphidx_csr* csr, const sphidx_launch* launch, void* stream);

/* For callers that cannot allocate device memory (work under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * as sphidx_query, with the query workspace taken from a fixed array of
 * SPHIDX_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  The call allocates nothing and calls no
 * allocating routine.
 *   csr    outputs as for sphidx_query; workspace_dev must be NULL and
 *          workspace_bytes 0 (INVALID_ARG otherwise)
 *   q      at most SPHIDX_NOALLOC_MAX_QUERIES queries (CAPACITY otherwise,
 *          nothing enqueued)
 *   tab    must already be on the device (tables built or loaded on a host
 *          with a device are); INVALID_ARG otherwise
 * The array beyond the minimum workspace is the stash, so rows that do not
 * fit it are walked again by the write pass (any batch is correct).  Every
 * call on a GPU uses that GPU's one array and leaves its contents there:
 * calls that overlap on one GPU (other streams, other host threads) race and
 * must be serialised by the caller.  Device selection: the current device. */
#define SPHIDX_NOALLOC_MAX_QUERIES 65536u
#define SPHIDX_NOALLOC_SCRATCH_BYTES (32u << 20)
sphidx_status sphidx_query_noalloc(const sphidx_lattice* lat, const sphidx_tables* tab, const sphidx_queries* q,
                                   sphidx_csr* csr, const sphidx_launch* launch, void* stream);

/* Pass 1 of a radius query with the default launch (mode forced to
 * RADIUS): the row sizes of Section II.A's neighbourhoods, scanned into
 * csr->row_ptr_dev (row_ptr[Q] = total pairs).  The workspace of `csr` is
 * required (the count pass keeps its query descriptors there for the write
 * pass); its ids, dist2 and capacity are not touched. */
sphidx_status sphidx_radius_count(const sphidx_lattice* lat, const sphidx_tables* tab,
                                  const sphidx_queries* q, sphidx_csr* csr, void* stream);

/* Named forms of sphidx_query with the default launch: radius (mode forced
 * to RADIUS), K nearest (mode forced to KNN), and the bin-lattice baseline
 * (method forced to CUBE, tables unused). */
sphidx_status sphidx_radius_query(const sphidx_lattice* lat, const sphidx_tables* tab,
                                  const sphidx_queries* q, sphidx_csr* csr, void* stream);
sphidx_status sphidx_knn_query(const sphidx_lattice* lat, const sphidx_tables* tab,
                               const sphidx_queries* q, sphidx_csr* csr, void* stream);
sphidx_status sphidx_cube_scan_radius(const sphidx_lattice* lat, const sphidx_queries* q, sphidx_csr* csr,
                                      void* stream);
sphidx_status sphidx_cube_scan_knn(const sphidx_lattice* lat, const sphidx_queries* q, sphidx_csr* csr,
                                   void* stream);

/* ---------------------------------------------------------------------- */
/* Moving agents (dynamic objects, Section I).                             */

/* Displace each coordinate of object i by delta in [-2^F/4, 2^F/4], drawn
 * from hash(seed, 1000 + 3*step + axis, i) with hash(s, t, i) =
 * mix64(s ^ mix64((t << 40) ^ i)), mix64 = the SplitMix64 finaliser; wrap on
 * cyclic axes, clamp to [0, W-1] on clipped ones.  In place on x, y, z. */
sphidx_status sphidx_move_agents(const sphidx_lattice_desc* desc, uint64_t seed, uint32_t step,
                                 uint32_t* x_dev, uint32_t* y_dev, uint32_t* z_dev, uint32_t n, void* stream);

/* The same with the step read from *step_dev (uint32, device) and the
 * counter advanced by one after the move, in stream order: a timestep
 * captured once in a HIP graph draws new displacements on every replay. */
sphidx_status sphidx_move_agents_counted(const sphidx_lattice_desc* desc, uint64_t seed, uint32_t* step_dev,
                                         uint32_t* x_dev, uint32_t* y_dev, uint32_t* z_dev, uint32_t n,
                                         void* stream);

/* Incremental maintenance of a lattice of moving objects (Section I: the
 * objects' cells are kept up to date as they move, instead of indexing them
 * again from their coordinates).  The lattice's own records are moved in
 * place, in their sorted order, by the displacement of sphidx_move_agents
 * (keyed by each record's object id), written to scratch_dev, and the
 * lattice is rebuilt from them by the same counting sort.  Objects that stay
 * in their cell, most of them at small steps, keep their place in memory
 * order, so the rebuild's atomics and stores fall on neighbouring addresses,
 * and no by-id coordinate array is read or written.
 *   lat          a lattice built with sphidx_build_lattice (its object ids
 *                are 0 .. n-1); after the call it holds the moved objects
 *   step, step_dev  as in sphidx_move_agents(_counted): with step_dev the
 *                step is read there and the counter advanced afterwards
 *   scratch_dev  device buffer of at least 16 * n bytes, 16-byte aligned,
 *                owned by the caller (free for other use between calls)
 * The object ids, cell starts and cell contents equal those of
 * sphidx_move_agents followed by sphidx_build_lattice on by-id arrays
 * (the order inside a cell can differ, as between any two builds).
 * Errors: SPHIDX_ERR_INVALID_ARG (null lattice, missing or misaligned
 * scratch), SPHIDX_ERR_CAPACITY (scratch too small). */
sphidx_status sphidx_move_resident(sphidx_lattice* lat, uint64_t seed, uint32_t step, uint32_t* step_dev,
                                   void* scratch_dev, size_t scratch_bytes, void* stream);

/* Incremental maintenance restricted to the objects that change cell
 * (Section I: the objects' cells are kept up to date as they move).  The
 * lattice's records are moved by the displacement of sphidx_move_agents
 * (keyed by object id); an object that stays in its cell keeps its rank
 * among its cell's stayers, found by one scan of stay flags over the sorted
 * records, and takes no atomic; only an object that changes cell takes one,
 * for its rank among its new cell's arrivals, which follow the stayers.
 *   lat, step, step_dev  as in sphidx_move_resident
 *   scratch_dev  device buffer of at least
 *                sphidx_move_incremental_scratch_bytes(lat) bytes (the moved
 *                records, arrival ranks, the previous cell starts and the
 *                new counts), 256-byte aligned, owned by the caller
 * Cell starts and cell contents equal those of sphidx_move_agents followed
 * by sphidx_build_lattice (the order inside a cell can differ: stayers keep
 * their order, arrivals follow in any order).  Every object stays usable:
 * clipped axes clamp to the region.
 * Errors: SPHIDX_ERR_INVALID_ARG (null lattice, missing or misaligned
 * scratch), SPHIDX_ERR_CAPACITY (scratch too small). */
size_t sphidx_move_incremental_scratch_bytes(const sphidx_lattice* lat);
sphidx_status sphidx_move_incremental(sphidx_lattice* lat, uint64_t seed, uint32_t step, uint32_t* step_dev,
                                      void* scratch_dev, size_t scratch_bytes, void* stream);

/* The lattice's objects as by-id coordinates: x_dev[id] = record x (normalised:
 * cyclic axes wrapped), and so on, for the n objects of the last build. */
sphidx_status sphidx_lattice_positions(const sphidx_lattice* lat, uint32_t* x_dev, uint32_t* y_dev, uint32_t* z_dev,
                                       void* stream);

/* out_dev[0] = sum of row sizes, out_dev[1] = sum_i mix64((i << 32) | size_i)
 * (mod 2^64), from row_ptr (Q + 1 entries).  out_dev is uint64[2]. */
sphidx_status sphidx_count_checksum(const int64_t* row_ptr_dev, uint32_t Q, uint64_t* out_dev, void* stream);

/* ---------------------------------------------------------------------- *
 * Serving: batches of queries against a device-resident lattice, with
 * continuous batching (many independent query sets against one maintained
 * index, the use Section I describes).
 *
 * A server holds `slots` batches in flight, each on its own stream (default
 * priority) with its own inputs, row_ptr and workspace (stash included), so
 * their kernels overlap on the device.  A batch is started when a slot is
 * free: its host inputs are staged through pinned memory and its count pass
 * runs.  When the count is done its exact output size is known, and it is
 * admitted to the write pass only when that many bytes fit in the server's
 * output pool (first fit; admission by memory, in arrival order); otherwise
 * it waits.  Its ids then stay in the pool until the batch is seen complete.
 * With slots = 1 and a SPHIDX_SCHED_PLAIN launch this is one plain launch
 * per batch: count, size, write, then the next batch.
 *
 * sphidx_server_run replays a schedule: batch i arrives arrival_s seconds
 * after the call starts (batches sorted by arrival), and the call returns when
 * every batch is complete.  The lattice must be complete before the call
 * (its build's stream synchronised) and stay unchanged during it.  Times
 * are host steady-clock seconds from the start of the call.  The server
 * allocates its device and pinned memory once, in sphidx_server_create;
 * runs allocate nothing. */
typedef struct sphidx_server sphidx_server;

typedef struct {
    uint32_t count;             /* queries, at most the server's max_batch */
    const uint32_t* x;          /* host arrays of `count` entries, read when the batch starts */
    const uint32_t* y;
    const uint32_t* z;
    const uint32_t* radius_fx;  /* per query: the radius, or the K-NN cap */
    const uint32_t* k;          /* per query: K (0 = a radius query); NULL = every query a radius query */
    double arrival_s;           /* seconds after the run starts */
    int64_t* row_ptr_out;       /* optional host int64[count + 1]: the batch's row_ptr */
    uint32_t* ids_out;          /* optional host uint32[ids_capacity]: its ids (rows ordered by
                                   (dist^2, id)), copied when it completes if they fit */
    uint64_t ids_capacity;
} sphidx_batch;

typedef struct {
    double start_s;             /* its count pass was launched */
    double admit_s;             /* its write pass was launched (its pool range reserved) */
    double done_s;              /* its write pass was seen complete (or it was rejected) */
    int64_t pairs;              /* its output pairs */
    uint64_t pool_in_use;       /* pool bytes reserved just after its admission */
    uint32_t rejected;          /* 1: its output alone is larger than the whole pool (nothing written) */
    uint32_t status;            /* SPHIDX_OK, or the error of one of its launches */
} sphidx_batch_result;

/* lat, tab: the lattice and tables every batch queries (kept by the caller
 * for the server's life; tab NULL for a cube-only launch).  slots >= 1,
 * max_batch >= 1, pool_bytes: the output pool (ids only), stash_pairs: the
 * stash per slot (0: none).  launch: the launch of every pass (NULL:
 * defaults; its statistics, method and event outputs are ignored).  Errors:
 * INVALID_ARG (null lattice or out, zero sizes, a pool under 256 bytes, a
 * launch that sphidx_count would refuse, e.g. null tables with a method
 * other than CUBE), SPHIDX_ERR_OUT_OF_MEMORY (device or pinned allocation
 * failed), DEVICE. */
sphidx_status sphidx_server_create(const sphidx_lattice* lat, const sphidx_tables* tab, uint32_t slots,
                                   uint32_t max_batch, size_t pool_bytes, uint64_t stash_pairs,
                                   const sphidx_launch* launch, sphidx_server** out);
void sphidx_server_destroy(sphidx_server* s);
/* Replay nbatch batches (sorted by arrival_s; INVALID_ARG otherwise, or for a
 * batch above max_batch or with a null input array) and fill results[i] for
 * batch i.  Returns the first launch error (later batches are not started)
 * or SPHIDX_OK; the lattice's status word collects device-side flags as for
 * any query. */
sphidx_status sphidx_server_run(sphidx_server* s, uint32_t nbatch, const sphidx_batch* batches,
                                sphidx_batch_result* results);

/* ---------------------------------------------------------------------- */

const char* sphidx_status_string(sphidx_status s);
/* Library version, e.g. "sphidx 1.0 gfx950". */
const char* sphidx_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPHIDX_H */
