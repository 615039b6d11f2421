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
    uint32_t* xs;
    uint32_t* ys;
    uint32_t* zs;
    uint32_t* ids;
    uint32_t* rank;     // per input object: its slot inside its cell (build scratch)
    uint32_t* scan_tmp; // scan partial sums
    uint32_t* status;   // device status word
    size_t bytes;
    int device;
};

struct sphidx_tables {
    uint32_t s;        // sub-cell bits per axis
    uint32_t F;        // frac bits of the lattice the tables were built for
    uint32_t rmax_fx;  // radius cap
    uint32_t nclasses; // 2^(3s)
    uint32_t rshift;   // radius-index bucket = 2^rshift units
    uint32_t nr;       // radius-index entries per class
    uint32_t max_off;  // largest |offset| component
    uint64_t total;
    // host copies (also what save/load serialise)
    std::vector<uint32_t> h_off;         // packed offsets, class-major, key-sorted
    std::vector<int64_t> h_key;          // keys, same order
    std::vector<uint32_t> h_class_start; // nclasses + 1
    std::vector<uint32_t> h_rindex;      // nclasses * nr
    // device copies
    uint32_t* d_off = nullptr;
    int64_t* d_key = nullptr;
    uint32_t* d_class_start = nullptr;
    uint32_t* d_rindex = nullptr;
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
    const uint32_t* xs;
    const uint32_t* ys;
    const uint32_t* zs;
    const uint32_t* ids;
    uint32_t* status;
};

struct TabArgs {
    const uint32_t* off;
    const int64_t* key;
    const uint32_t* cstart;
    const uint32_t* rindex;
    uint32_t s;
    uint32_t rshift;
    uint32_t nr;
    uint32_t rmax;
    uint32_t total;
    uint32_t has;   // 0: no tables (cube only)
    uint32_t lds;   // 1: stage off[] in LDS
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
    uint32_t* queues;   // persistent work counters (NQUEUE)
    uint32_t* stats;
    uint32_t method;
    uint32_t persistent;
    uint32_t tile;
    uint32_t sort_cap;
};

#define SPHIDX_NQUEUE 8  // one work queue per XCD of the MI355X
#define SPHIDX_MAX_LOG2_SUM 30

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files).

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t st);
hipError_t launch_build(const sphidx_lattice* lat, const uint32_t* x, const uint32_t* y, const uint32_t* z,
                        uint32_t n, hipStream_t st);
hipError_t launch_scan_i64(int64_t* data, uint32_t n, void* tmp, hipStream_t st);
size_t scan_i64_tmp_bytes(uint32_t n);
hipError_t launch_query_pass(int pass, const LatArgs& L, const TabArgs& T, const QArgs& q,
                             uint32_t waves_per_block, uint32_t blocks_per_cu, hipStream_t st);
hipError_t launch_move_agents(const sphidx_lattice_desc& d, uint64_t seed, uint32_t step, uint32_t* x,
                              uint32_t* y, uint32_t* z, uint32_t n, hipStream_t st);
hipError_t launch_count_checksum(const int64_t* row_ptr, uint32_t Q, uint64_t* out, hipStream_t st);
int device_cu_count();
