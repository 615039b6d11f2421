// Moving agents (dynamic objects whose positions change every step,
// Section I) and the order-independent checksum of per-row neighbour counts.
#include <algorithm>

#include "sphidx_internal.h"

namespace {

// SplitMix64 output finaliser (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t counter_hash(uint64_t seed, uint64_t tag, uint64_t i) {
    return mix64(seed ^ mix64((tag << 40) ^ i));
}

struct MoveArgs {
    uint32_t wbits[3];
    uint32_t cyc;
    uint32_t dmax;
    uint64_t seed;
    uint32_t step;
    const uint32_t* step_dev;  // when set, the step is read here
    uint32_t n;
    uint32_t* v[3];
};

// One coordinate of object `id` after the step's displacement (wrap on a
// cyclic axis, clamp on a clipped one).
__device__ __forceinline__ uint32_t moved(const MoveArgs& a, uint32_t step, int k, uint32_t id, uint32_t v) {
    const uint64_t span = 2ull * a.dmax + 1ull;
    const uint64_t h = counter_hash(a.seed, 1000ull + 3ull * step + (uint64_t)k, id);
    const int64_t delta = (int64_t)(((h >> 32) * span) >> 32) - (int64_t)a.dmax;
    const int64_t w = (int64_t)1 << a.wbits[k];
    int64_t nv = (int64_t)v + delta;
    if ((a.cyc >> k) & 1u)
        nv &= w - 1;
    else
        nv = nv < 0 ? 0 : (nv > w - 1 ? w - 1 : nv);
    return (uint32_t)nv;
}

__global__ __launch_bounds__(256) void move_kernel(MoveArgs a) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint32_t step = a.step_dev ? *a.step_dev : a.step;
#pragma unroll
    for (int k = 0; k < 3; ++k) a.v[k][i] = moved(a, step, k, i, a.v[k][i]);
}

// The same displacement applied to the lattice's own records, in their
// sorted order: record p of src, moved, is record p of dst.
__global__ __launch_bounds__(256) void move_records_kernel(MoveArgs a, const uint4* __restrict__ src,
                                                           uint4* __restrict__ dst) {
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const uint32_t step = a.step_dev ? *a.step_dev : a.step;
    const uint4 P = src[p];
    dst[p] = make_uint4(moved(a, step, 0, P.w, P.x), moved(a, step, 1, P.w, P.y), moved(a, step, 2, P.w, P.z), P.w);
}

// By-id coordinates from the records (object ids are 0 .. n-1).
__global__ __launch_bounds__(256) void records_to_ids_kernel(const uint4* __restrict__ pts, uint32_t n, uint32_t* x,
                                                             uint32_t* y, uint32_t* z) {
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint4 P = pts[p];
    x[P.w] = P.x;
    y[P.w] = P.y;
    z[P.w] = P.z;
}

__global__ void advance_step_kernel(uint32_t* step) { *step += 1u; }

__global__ __launch_bounds__(256) void checksum_kernel(const int64_t* __restrict__ row_ptr, uint32_t Q,
                                                       unsigned long long* out) {
    __shared__ uint64_t part[2][4];
    uint64_t s = 0, h = 0;
    // four consecutive rows per thread and step: five row_ptr loads in flight
    const uint64_t stride = 4ull * gridDim.x * blockDim.x;
    for (uint64_t i0 = 4ull * (blockIdx.x * blockDim.x + threadIdx.x); i0 < Q; i0 += stride) {
        int64_t v[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) v[k] = i0 + k <= Q ? row_ptr[i0 + k] : 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < Q) {
                const uint64_t c = (uint64_t)(v[k + 1] - v[k]);
                s += c;
                h += mix64(((i0 + k) << 32) | (c & 0xffffffffull));
            }
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        s += __shfl_xor(s, d);
        h += __shfl_xor(h, d);
    }
    // one pair of atomics per block: the same two words take every block's
    // sums, so their count is what bounds the kernel
    const uint32_t wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        part[0][wave] = s;
        part[1][wave] = h;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t w = 1; w < (blockDim.x >> 6); ++w) {
            s += part[0][w];
            h += part[1][w];
        }
        atomicAdd(&out[0], (unsigned long long)s);
        atomicAdd(&out[1], (unsigned long long)h);
    }
}

// ---------------------------------------------------------------------------
// Incremental lattice update (Section I: the objects' cells are kept up to
// date as they move).  Objects that stay in their cell keep their order and
// take no atomic; only the movers count themselves into their new cells.
//   move     record p moved; stay flag = (new cell == old cell); a mover
//            takes its rank among its new cell's arrivals (one atomic)
//   scan     exclusive scan of the stay flags: S
//   count    per cell c: its stayers' base SB[c] = S[cs[c]] (old starts),
//            new count = S[cs[c+1]] - S[cs[c]] + arrivals
//   scan     the new counts -> the lattice's new cell starts
//   place    a stayer keeps its rank among its cell's stayers, S[p] - SB[c];
//            a mover goes after its new cell's stayers, at its arrival rank

struct IncArgs {
    uint32_t lg[3];
    uint32_t F;
    uint32_t cyc;
    uint32_t ncells;
    uint32_t n;
    const uint4* old_pts;  // the lattice's records before the step (sorted)
    uint4* moved;          // the same records moved, in the old order
    uint4* new_pts;        // the lattice's records after the step
    uint32_t* cs;          // the lattice's cell starts: old ones, then new ones (ncells + 3)
    uint32_t* sb;          // per cell: stayers before its first object (ncells + 3)
    uint32_t* cnt;         // arrivals per cell, then new counts
    uint32_t* stay;        // n + 1: stay flags, then their exclusive scan
    uint32_t* arank;       // per mover: rank among its new cell's arrivals
};

// Cell of a normalised record: region cells packed z-major, ncells for a
// clipped coordinate at or beyond the world width (the outside cell),
// ncells + 1 for a clipped coordinate >= 2^30 (left out of queries).
__device__ __forceinline__ uint32_t inc_cell(const IncArgs& a, const uint4& P) {
    const uint32_t v[3] = {P.x, P.y, P.z};
    bool out = false, bad = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (!((a.cyc >> k) & 1u)) {
            bad |= v[k] >= (1u << 30);
            out |= (v[k] >> (a.lg[k] + a.F)) != 0u;
        }
    }
    if (bad) return a.ncells + 1u;
    if (out) return a.ncells;
    return ((v[2] >> a.F) << (a.lg[0] + a.lg[1])) | ((v[1] >> a.F) << a.lg[0]) | (v[0] >> a.F);
}

__global__ __launch_bounds__(256) void inc_move_kernel(MoveArgs m, IncArgs a) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const uint32_t step = m.step_dev ? *m.step_dev : m.step;
    const uint4 P = a.old_pts[p];
    const uint4 N = make_uint4(moved(m, step, 0, P.w, P.x), moved(m, step, 1, P.w, P.y), moved(m, step, 2, P.w, P.z),
                               P.w);
    a.moved[p] = N;
    const uint32_t c = inc_cell(a, P), c2 = inc_cell(a, N);
    const bool st = c == c2;
    a.stay[p] = st ? 1u : 0u;
    if (!st) a.arank[p] = atomicAdd(&a.cnt[c2], 1u);
}

__global__ __launch_bounds__(256) void inc_count_kernel(IncArgs a) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ncells + 2u) return;
    const uint32_t b = a.stay[a.cs[c]], e = a.stay[a.cs[c + 1]];
    a.sb[c] = b;
    if (c == a.ncells + 1u) a.sb[c + 1] = e;
    a.cnt[c] += e - b;
}

__global__ __launch_bounds__(256) void inc_place_kernel(IncArgs a) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const uint4 N = a.moved[p];
    const uint32_t c = inc_cell(a, N);
    const uint32_t s0 = a.stay[p];
    uint32_t pos;
    if (a.stay[p + 1] != s0)
        pos = a.cs[c] + (s0 - a.sb[c]);  // stayer: rank among its cell's stayers
    else
        pos = a.cs[c] + (a.sb[c + 1] - a.sb[c]) + a.arank[p];
    a.new_pts[pos] = N;
}

}  // namespace

namespace {

MoveArgs move_args(const sphidx_lattice_desc& d, uint64_t seed, uint32_t step, uint32_t* step_dev, uint32_t n) {
    MoveArgs a;
    a.step_dev = step_dev;
    for (int k = 0; k < 3; ++k) a.wbits[k] = d.log2_cells[k] + d.frac_bits;
    a.cyc = d.cyclic_mask;
    a.dmax = (1u << d.frac_bits) / 4u;
    a.seed = seed;
    a.step = step;
    a.n = n;
    for (int k = 0; k < 3; ++k) a.v[k] = nullptr;
    return a;
}

}  // namespace

hipError_t launch_move_records(const sphidx_lattice_desc& d, uint64_t seed, uint32_t* step_dev, const uint4* src,
                               uint4* dst, uint32_t n, hipStream_t st) {
    const MoveArgs a = move_args(d, seed, 0, step_dev, n);
    if (n > 0) move_records_kernel<<<(n + 255) / 256, 256, 0, st>>>(a, src, dst);
    if (step_dev) advance_step_kernel<<<1, 1, 0, st>>>(step_dev);
    return hipGetLastError();
}

hipError_t launch_move_records_at(const sphidx_lattice_desc& d, uint64_t seed, uint32_t step, const uint4* src,
                                  uint4* dst, uint32_t n, hipStream_t st) {
    const MoveArgs a = move_args(d, seed, step, nullptr, n);
    if (n > 0) move_records_kernel<<<(n + 255) / 256, 256, 0, st>>>(a, src, dst);
    return hipGetLastError();
}

hipError_t launch_records_to_ids(const uint4* pts, uint32_t n, uint32_t* x, uint32_t* y, uint32_t* z,
                                 hipStream_t st) {
    if (n > 0) records_to_ids_kernel<<<(n + 255) / 256, 256, 0, st>>>(pts, n, x, y, z);
    return hipGetLastError();
}

hipError_t launch_move_agents(const sphidx_lattice_desc& d, uint64_t seed, uint32_t step, uint32_t* step_dev,
                              uint32_t* x, uint32_t* y, uint32_t* z, uint32_t n, hipStream_t st) {
    MoveArgs a;
    a.step_dev = step_dev;
    for (int k = 0; k < 3; ++k) a.wbits[k] = d.log2_cells[k] + d.frac_bits;
    a.cyc = d.cyclic_mask;
    a.dmax = (1u << d.frac_bits) / 4u;
    a.seed = seed;
    a.step = step;
    a.n = n;
    a.v[0] = x;
    a.v[1] = y;
    a.v[2] = z;
    if (n > 0) move_kernel<<<(n + 255) / 256, 256, 0, st>>>(a);
    // stream order: the counter advances after every object has moved
    if (step_dev) advance_step_kernel<<<1, 1, 0, st>>>(step_dev);
    return hipGetLastError();
}

hipError_t launch_count_checksum(const int64_t* row_ptr, uint32_t Q, uint64_t* out, hipStream_t st) {
    hipError_t e = launch_fill_u32((uint32_t*)out, 0u, 4, st);
    if (e != hipSuccess) return e;
    uint32_t blocks = (Q + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks == 0) blocks = 1;
    checksum_kernel<<<blocks, 256, 0, st>>>(row_ptr, Q, (unsigned long long*)out);
    return hipGetLastError();
}

// Incremental update of a lattice of moving objects: scratch holds the moved
// records (16 B per object), the movers' arrival ranks (4 B per object), the
// per-cell stayer bases and counts (4 B per cell each); the lattice's rank
// array holds the stay flags and their scan.
size_t move_incremental_scratch_bytes(const sphidx_lattice* lat) {
    const size_t n = lat->max_points, nc = (size_t)lat->ncells + 4;
    return 16 * n + 4 * n + 4 * nc + 4 * nc + 1024;
}

hipError_t launch_move_incremental(sphidx_lattice* lat, uint64_t seed, uint32_t step, uint32_t* step_dev,
                                   void* scratch, hipStream_t st) {
    const uint32_t n = lat->n;
    const size_t nc = (size_t)lat->ncells + 4;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    char* b = (char*)scratch;
    IncArgs a;
    for (int k = 0; k < 3; ++k) a.lg[k] = lat->desc.log2_cells[k];
    a.F = lat->desc.frac_bits;
    a.cyc = lat->desc.cyclic_mask;
    a.ncells = lat->ncells;
    a.n = n;
    a.old_pts = lat->pts;
    a.new_pts = lat->pts;
    a.moved = (uint4*)b;
    a.arank = (uint32_t*)(b + al(16 * (size_t)n));
    a.sb = (uint32_t*)(b + al(16 * (size_t)n) + al(4 * (size_t)n));
    a.cnt = (uint32_t*)((char*)a.sb + al(4 * nc));
    a.cs = lat->cell_start;
    a.stay = lat->rank;
    const MoveArgs m = move_args(lat->desc, seed, step, step_dev, n);
    hipError_t e = launch_fill_u32(a.cnt, 0u, (size_t)lat->ncells + 3, st);
    if (e != hipSuccess) return e;
    // arrivals follow the stayers: cells in no particular order
    if ((e = launch_fill_u32(lat->status + 1, 0u, 1, st)) != hipSuccess) return e;
    const uint32_t blocks = (n + 255) / 256;
    if (n > 0) inc_move_kernel<<<blocks, 256, 0, st>>>(m, a);
    if (step_dev) advance_step_kernel<<<1, 1, 0, st>>>(step_dev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_scan_u32(a.stay, n, lat->scan_tmp, st)) != hipSuccess) return e;
    inc_count_kernel<<<(lat->ncells + 2u + 255u) / 256u, 256, 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the new counts' scan is written straight into the lattice's cell starts
    if ((e = launch_scan_u32_to(a.cnt, lat->cell_start, (size_t)lat->ncells + 2, lat->scan_tmp, st)) != hipSuccess)
        return e;
    if (n > 0) inc_place_kernel<<<blocks, 256, 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_cell_list(lat, st);
}
