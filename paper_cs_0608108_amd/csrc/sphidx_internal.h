// Internal types of libsphidx shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "sphidx.h"

// ---------------------------------------------------------------------------
// Host-side handles (opaque to callers).

struct sphidx_lattice {
    sphidx_lattice_desc desc;
    uint32_t max_points;
    uint32_t n;       // objects of the last build
    uint32_t ncells;  // region cells; index ncells = outside cell, ncells + 1 = skipped objects
    uint32_t* cell_start;  // ncells + 3
    uint4* pts;         // by sorted position: normalised x, y, z and the object id
    uint32_t* rank;     // per input object: its slot inside its cell (build scratch)
    uint32_t* scan_tmp; // scan partial sums
    uint32_t* status;   // device status word; status[1]: 1 while every cell's objects are in x order
    uint32_t cell_order; // SPHIDX_ORDER_*: the order builds give the objects inside a cell
    uint4* xbuf;         // ORDER_X: library-owned records (max_points x 16 B) the counting sort
                         // fills before the x ranking places them; NULL until that order is set
    size_t bytes;
    int device;
    // attached non-empty cell list (caller-owned): count word, then entries
    // {cell, first sorted position} from byte 16; NULL when none
    char* cell_list;
};

struct sphidx_tables {
    uint32_t s;        // sub-cell bits per axis
    uint32_t F;        // frac bits of the lattice the tables were built for
    uint32_t rmax_fx;  // radius cap
    uint32_t nclasses; // 2^(3s) cell-table classes
    uint32_t rshift;   // radius-index bucket = 2^rshift units
    uint32_t nr;       // radius-index entries per class
    uint32_t max_off;  // largest |offset| component
    uint64_t total;
    // cell table (host; what export, save and load use): packed offsets,
    // class-major, key-sorted, with their keys
    std::vector<uint32_t> h_off;
    std::vector<int64_t> h_key;
    std::vector<uint32_t> h_class_start; // nclasses + 1
    std::vector<uint32_t> h_rindex;      // nclasses * nr
    // row table (what the kernels walk): per (y, z) sub-cell class, the
    // x-rows (oy, oz) of cells, sorted by the row's key
    uint32_t nrclasses;                   // 2^(2s)
    std::vector<uint32_t> h_rows;         // (oy & 0xffff) | (oz << 16)
    std::vector<int64_t> h_rkey;
    std::vector<uint32_t> h_rclass_start; // nrclasses + 1
    std::vector<uint32_t> h_rrindex;      // nrclasses * nr
    // the paper's tables (Section III.A), built when the offsets stay within
    // kPaperMaxOff cells: 64 specialised tables, then the unshaved table,
    // each sorted by b^2 (packed offsets and b^2), and per table and value v
    // the absolute index of its first entry with b^2 >= v
    uint32_t pm = 0;    // offset bound m (0: not built)
    uint32_t pnb2 = 0;  // values v per table in the index (3 m^2 + 2)
    std::vector<uint32_t> h_poff, h_pb2, h_pstart, h_plo;
    uint32_t* d_poff = nullptr;
    uint32_t* d_pb2 = nullptr;
    uint32_t* d_plo = nullptr;
    // device copies of the row table
    uint32_t* d_rows = nullptr;
    int64_t* d_rkey = nullptr;
    uint32_t* d_rclass_start = nullptr;
    uint32_t* d_rrindex = nullptr;
    uint32_t* d_vcount = nullptr;  // copy of h_rindex: cells per class and radius bucket
    size_t device_bytes = 0;
};

// ---------------------------------------------------------------------------
// Kernel argument blocks (passed by value).

struct LatArgs {
    uint32_t lg[3];     // log2 cells per axis
    uint32_t F;         // frac bits
    uint32_t cyc;       // cyclic mask
    uint32_t ncells;
    uint32_t n;
    const uint32_t* cs;   // cell_start
    const uint4* pts;     // sorted objects {x, y, z, id}
    uint32_t* status;
    const uint2* cells;   // non-empty cell list {cell, first} (NULL: none kept)
    const uint32_t* ncl;  // its length (device)
    const uint32_t* xsorted;  // device word: 1 when the objects inside every cell are in x order (NULL: not kept)
};

struct TabArgs {
    const uint32_t* rows;   // packed (oy, oz), class-major, key-sorted
    const int64_t* rkey;    // row keys, same order
    const uint32_t* cstart; // first row of each class
    const uint32_t* rindex; // per class and radius bucket: rows with key <= bucket^2
    const uint32_t* vcount; // per 3-D sub-cell class and radius bucket: cells with key <= bucket^2
    uint32_t s;
    uint32_t rshift;
    uint32_t nr;
    uint32_t rmax;
    uint32_t total;  // rows over all classes
    uint32_t has;    // 0: no tables (cube only)
    uint32_t lds;    // 1: stage the row table in LDS
    uint32_t lds_chunk;  // with lds: rows staged per (y, z) class, the first of each (0: the whole table)
    uint32_t nrcls;      // (y, z) classes of the row table
    // the paper's tables (METHOD_PAPER64)
    uint32_t paper;         // 1: walk them instead of the row table
    const uint32_t* p_off;  // packed offsets, tables 0..63 then the unshaved table
    const uint32_t* p_b2;   // b^2 of each entry
    const uint32_t* p_lo;   // [65][p_nb2]: first entry of table t with b^2 >= v
    uint32_t p_nb2;
};

struct QArgs {
    uint32_t Q;
    const uint32_t* qx;  // NULL: all agents
    const uint32_t* qy;
    const uint32_t* qz;
    const uint32_t* rad;
    uint32_t rad_u;
    const uint32_t* kk;
    uint32_t k_u;
    uint32_t mode;
    uint32_t flags;
    int64_t* row_ptr;
    uint32_t* out_ids;
    int64_t* out_d2;
    int64_t capacity;
    uint32_t* queues;   // work counters: NQSETS x NQUEUE, then the list counters
    uint32_t* long_count;
    uint32_t* longq;    // rows handed from the write kernels to the top-M kernel
    uint32_t* fb_count;
    uint32_t* fbq;      // sphere method: queries the tables do not cover (cube scan)
    uint32_t* walk_count;
    uint32_t* walkq;    // stash mode: queries the count pass did not stash
    uint32_t* xq_count;
    uint32_t* xq;       // grouped count: queries left to the one-query-per-wave kernel
    uint32_t* lq_count;
    uint32_t* lq;       // stash mode: radius rows expected to be long, counted one block per row
    uint32_t* soff;     // stash mode: per output row, first stash element of its sorted row
    uint32_t* stash_hdr;  // stash header written by the count pass (see StashHdr)
    uint32_t* stash_ctr;  // NQUEUE per-region allocation counters
    char* stash_base;     // start of the stash area of the workspace
    uint32_t* stash_ids;  // count pass: stash arrays (ids, optional dist^2)
    int64_t* stash_d2;
    uint32_t stash;       // count pass: 1 = keep sorted rows in the stash
    uint32_t stash_region;  // elements per region
    uint32_t stash_chunk;   // elements per allocation grab
    const uint32_t* list;       // list-driven launches: the query list,
    const uint32_t* list_count; // its length (device)
    uint32_t list_set;          // and its work-queue set
    uint4* desc;        // per query (processing order): 4 x uint4 set up by the setup kernel
    uint32_t* stats;
    uint32_t method;
    uint32_t persistent;
    uint32_t tile;
    uint32_t sort_cap;
    uint32_t interior;  // count pass: count wholly-inside cells without reading them
    uint32_t group;     // count pass: radius queries in groups per wavefront
    uint32_t select;    // setup: 0 = the kernel's method, 1 = choose by volume, 2 = cell list
    uint32_t weight;    // volume choice: sphere cells x weight / 256 against cube cells
    uint32_t rev;       // volume choice: radius queries below this skip the sphere
    uint32_t knn_rev;   // volume choice: K-NN queries below this take the cube
    uint32_t model;     // volume choice: 0 = cells, 1 = estimated lane work
    uint32_t* method_out;  // optional per query row: the walk used
    uint32_t long_waves;   // write pass: waves per long radius row (one block each); <= 1: one wave, windowed
};

// Stash header words (in the counter block): written by the count pass,
// read by the write pass, which therefore needs no host-side state.
enum : uint32_t { kHdrMode = 0, kHdrElems = 1, kHdrHasD2 = 2, kHdrD2Off = 3 };

#define SPHIDX_NXCD 8           // XCDs of the MI355X: blocks are dispatched to them in turn
#define SPHIDX_NQUEUE 64        // work queues per set, 8 per XCD: queue q is served by the blocks of XCD q mod 8
#define SPHIDX_NREGION SPHIDX_NXCD  // stash regions, one per XCD
#define SPHIDX_QSTRIDE 32       // counters 128 bytes apart: one L2 line each
#define SPHIDX_NQSETS 7         // count, write, top-M, fallback count, fallback write, walk list, extra list
#define SPHIDX_NLISTS 6         // long_count, fb_count, walk_count, stash header, xq_count, lq_count
#define SPHIDX_COUNTER_WORDS \
    ((SPHIDX_NQSETS * SPHIDX_NQUEUE + SPHIDX_NLISTS + SPHIDX_NREGION) * SPHIDX_QSTRIDE)
#define SPHIDX_MAX_LOG2_SUM 30
static_assert(SPHIDX_NQUEUE <= 64 && SPHIDX_NQUEUE % SPHIDX_NXCD == 0, "a wave looks at every queue at once");

constexpr uint32_t kPaperMaxOff = 32;

// LDS bytes of the staged row table: the whole table, or the first
// lds_chunk rows of every (y, z) class.
inline size_t tab_lds_bytes(const TabArgs& T) {
    if (!T.lds) return 0;
    const size_t words = T.lds_chunk ? (size_t)T.nrcls * T.lds_chunk : (size_t)T.total;
    return (words * 4 + 15) & ~(size_t)15;
}
void paper_tables_flat(int m, std::vector<uint32_t>& off, std::vector<uint32_t>& b2, std::vector<uint32_t>& start);

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files).

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t st);
hipError_t launch_build(const sphidx_lattice* lat, const uint32_t* x, const uint32_t* y, const uint32_t* z,
                        uint32_t n, hipStream_t st);
hipError_t launch_cell_list(const sphidx_lattice* lat, hipStream_t st);
hipError_t launch_scan_i64(int64_t* data, uint32_t n, void* tmp, hipStream_t st);
size_t scan_i64_tmp_bytes(uint32_t n);
hipError_t launch_query_pass(int pass, const LatArgs& L, const TabArgs& T, const QArgs& q,
                             uint32_t waves_per_block, uint32_t blocks_per_cu, hipStream_t st,
                             hipEvent_t ev_begin, hipEvent_t ev_end);
hipError_t launch_build_records(const sphidx_lattice* lat, const uint4* recs, uint32_t n, hipStream_t st);
hipError_t launch_move_records(const sphidx_lattice_desc& d, uint64_t seed, uint32_t* step_dev, const uint4* src,
                               uint4* dst, uint32_t n, hipStream_t st);
hipError_t launch_move_records_at(const sphidx_lattice_desc& d, uint64_t seed, uint32_t step, const uint4* src,
                                  uint4* dst, uint32_t n, hipStream_t st);
hipError_t launch_records_to_ids(const uint4* pts, uint32_t n, uint32_t* x, uint32_t* y, uint32_t* z,
                                 hipStream_t st);
hipError_t launch_move_agents(const sphidx_lattice_desc& d, uint64_t seed, uint32_t step, uint32_t* step_dev,
                              uint32_t* x, uint32_t* y, uint32_t* z, uint32_t n, hipStream_t st);
size_t move_incremental_scratch_bytes(const sphidx_lattice* lat);
hipError_t launch_move_incremental(sphidx_lattice* lat, uint64_t seed, uint32_t step, uint32_t* step_dev,
                                   void* scratch, hipStream_t st);
hipError_t launch_scan_u32(uint32_t* data, size_t n, uint32_t* tmp, hipStream_t st);
hipError_t launch_scan_u32_to(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp, hipStream_t st);
hipError_t launch_count_checksum(const int64_t* row_ptr, uint32_t Q, uint64_t* out, hipStream_t st);
int device_cu_count();
size_t query_lds_bytes(int pass, uint32_t cap, uint32_t waves, size_t table_bytes);
size_t long_lds_bytes(uint32_t waves);
// Drop a stream from the record of streams that touched a lattice (called
// before the stream is destroyed).
void forget_stream(void* stream);
// The checks every query call makes of a launch descriptor (with these
// tables), without launching anything.
sphidx_status check_launch(const sphidx_launch* launch, const sphidx_tables* tab);
