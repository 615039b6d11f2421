// Lattice rebuild as a counting sort (each object in exactly one cell,
// Section I; packed ZYX cell index and the unique outside cell, Section II.B):
//   fill    count[0 .. ncells+2) = 0
//   hist    per object: normalise, cell id, slot = atomicAdd(count[cell], 1)
//   scan    exclusive prefix over ncells + 2 counts -> cell_start (+ total)
//   scatter per object: position = cell_start[cell] + slot; one 16-byte
//           record {x, y, z, id} per object, so a candidate is one load
//   list    (when a list is attached) the non-empty cells in cell order,
//           Section III.B: flag the first object of each region cell, scan
//           the flags, write {cell, first position} at the flag's rank
// plus the reduce-then-scan used for cell_start and for query row pointers.
#include "sphidx_internal.h"

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;  // per thread
constexpr int kScanBlock = kScanThreads * kScanItems;

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

struct BuildArgs {
    uint32_t lg[3];
    uint32_t F;
    uint32_t cyc;
    uint32_t ncells;
    uint32_t n;
    const uint32_t* x;
    const uint32_t* y;
    const uint32_t* z;
    const uint4* recs;  // rebuild from records: {x, y, z, id} by position
    uint32_t* count;  // == cell_start storage
    uint32_t* rank;
    uint4* pts;
    uint32_t* status;
    uint4* out;  // x order: where the ranking places the records (pts holds the counting sort's)
};

// Normalise one object and return its cell: region cells are packed ZYX
// (z << (lx+ly) | y << lx | x), ncells is the outside cell and ncells + 1
// holds objects with an unusable clipped coordinate (>= 2^30).
__device__ __forceinline__ uint32_t object_cell(const BuildArgs& a, uint32_t& vx, uint32_t& vy,
                                                uint32_t& vz, bool& bad) {
    uint32_t v[3] = {vx, vy, vz};
    uint32_t c[3];
    bool out = false;
    bad = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        uint32_t wbits = a.lg[k] + a.F;
        if ((a.cyc >> k) & 1u) {
            v[k] &= (1u << wbits) - 1u;
        } else {
            bad |= v[k] >= (1u << 30);
            out |= (v[k] >> wbits) != 0u;
        }
        c[k] = v[k] >> a.F;
    }
    vx = v[0];
    vy = v[1];
    vz = v[2];
    if (bad) return a.ncells + 1u;
    if (out) return a.ncells;
    return (c[2] << (a.lg[0] + a.lg[1])) | (c[1] << a.lg[0]) | c[0];
}

__global__ __launch_bounds__(256) void hist_kernel(BuildArgs a) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    uint32_t vx = a.x[i], vy = a.y[i], vz = a.z[i];
    bool bad;
    uint32_t cell = object_cell(a, vx, vy, vz, bad);
    if (bad) atomicOr(a.status, SPHIDX_FLAG_RANGE);
    a.rank[i] = atomicAdd(&a.count[cell], 1u);
}

__global__ __launch_bounds__(256) void scatter_kernel(BuildArgs a) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    uint32_t vx = a.x[i], vy = a.y[i], vz = a.z[i];
    bool bad;
    uint32_t cell = object_cell(a, vx, vy, vz, bad);
    uint32_t pos = a.count[cell] + a.rank[i];
    a.pts[pos] = make_uint4(vx, vy, vz, i);
}

// The same two steps over records {x, y, z, id} (the lattice's own, moved in
// place): the rank is kept per record position, and the record keeps its id.
__global__ __launch_bounds__(256) void hist_records_kernel(BuildArgs a) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint4 P = a.recs[i];
    uint32_t vx = P.x, vy = P.y, vz = P.z;
    bool bad;
    uint32_t cell = object_cell(a, vx, vy, vz, bad);
    if (bad) atomicOr(a.status, SPHIDX_FLAG_RANGE);
    a.rank[i] = atomicAdd(&a.count[cell], 1u);
}

__global__ __launch_bounds__(256) void scatter_records_kernel(BuildArgs a) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint4 P = a.recs[i];
    uint32_t vx = P.x, vy = P.y, vz = P.z;
    bool bad;
    uint32_t cell = object_cell(a, vx, vy, vz, bad);
    a.pts[a.count[cell] + a.rank[i]] = make_uint4(vx, vy, vz, P.w);
}

// Objects inside a cell in x order (then id), for cells of at most
// kXSortCap objects: after the scatter (into a second record array), every
// object counts the objects of its cell that come before it and is written
// to the lattice's records at its cell's start plus that rank.  In a larger
// cell an object keeps its place and the lattice's x-order word is cleared.  A block's 256 positions
// cover a run of whole or partial cells; when the cells' objects number at
// most kXStage they are staged in LDS as (x, id) keys and counted there,
// else every thread reads its cell from device memory.
constexpr uint32_t kXSortCap = 4096;
constexpr uint32_t kXStage = 2048;

__global__ __launch_bounds__(256) void xrank_kernel(BuildArgs a) {
    __shared__ uint64_t keys[kXStage];
    __shared__ uint32_t span[2];
    const uint32_t p0 = blockIdx.x * blockDim.x, p = p0 + threadIdx.x;
    const uint32_t last = min(a.n, p0 + blockDim.x) - 1u;
    const bool act = p < a.n;
    uint4 P = make_uint4(0, 0, 0, 0);
    uint32_t lo = 0, hi = 0;  // the cell's positions (the last two cells: no x)
    if (act) {
        P = a.pts[p];
        uint32_t vx = P.x, vy = P.y, vz = P.z;
        bool bad;
        const uint32_t cell = object_cell(a, vx, vy, vz, bad);
        lo = a.count[cell];
        hi = a.count[cell + 1];
    }
    // positions are in cell order: the block's cells span [lo of its first
    // position, hi of its last)
    if (p == p0) span[0] = lo;
    if (p == last) span[1] = hi;
    __syncthreads();
    const uint32_t s0 = span[0], s1 = span[1];
    const bool staged = s1 - s0 <= kXStage;
    if (staged) {
        for (uint32_t q = s0 + threadIdx.x; q < s1; q += blockDim.x) {
            const uint4 Q = a.pts[q];
            keys[q - s0] = ((uint64_t)Q.x << 32) | Q.w;
        }
    }
    __syncthreads();
    if (!act) return;
    uint32_t r = p - lo;
    if (hi - lo > kXSortCap) {
        if (p == lo) a.status[1] = 0u;
    } else if (staged) {
        const uint64_t mine = ((uint64_t)P.x << 32) | P.w;
        r = 0;
        for (uint32_t q = lo - s0; q < hi - s0; ++q) r += keys[q] < mine ? 1u : 0u;
    } else {
        r = 0;
        for (uint32_t q = lo; q < hi; ++q) {
            const uint4 Q = a.pts[q];
            r += (Q.x < P.x || (Q.x == P.x && Q.w < P.w)) ? 1u : 0u;
        }
    }
    a.out[lo + r] = P;
}

// Packed region cell of a sorted record (normalised, inside the region).
__device__ __forceinline__ uint32_t record_cell(const BuildArgs& a, const uint4& P) {
    return ((P.z >> a.F) << (a.lg[0] + a.lg[1])) | ((P.y >> a.F) << a.lg[0]) | (P.x >> a.F);
}

// flag[i] = 1 when sorted position i holds the first object of a region cell.
__global__ __launch_bounds__(256) void cell_flag_kernel(BuildArgs a, uint32_t* __restrict__ flag) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    uint32_t f = 0;
    if (i < a.count[a.ncells]) f = a.count[record_cell(a, a.pts[i])] == i ? 1u : 0u;
    flag[i] = f;
}

// After the exclusive scan of the flags (pos[n] = their total): entry
// pos[i] = {cell, i} for each flagged i, then the count and the closing entry.
__global__ __launch_bounds__(256) void cell_list_kernel(BuildArgs a, const uint32_t* __restrict__ pos,
                                                        uint32_t* __restrict__ hdr, uint2* __restrict__ list) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.n && pos[i + 1] != pos[i]) list[pos[i]] = make_uint2(record_cell(a, a.pts[i]), i);
    if (i == 0) {
        const uint32_t cnt = pos[a.n];
        hdr[0] = cnt;
        list[cnt] = make_uint2(0xFFFFFFFFu, a.count[a.ncells]);
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan, reduce-then-scan over blocks of kScanBlock elements.
// No inter-block waiting: three launches, each block independent.

template <typename T>
__device__ T block_exclusive_scan(T v, T* sh, T& total) {
    // wave-level inclusive scan
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T t = __shfl_up(x, d);
        if (lane >= d) x += t;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) {
            T s = sh[w];
            sh[w] = acc;
            acc += s;
        }
        sh[kScanThreads / 64] = acc;
    }
    __syncthreads();
    total = sh[kScanThreads / 64];
    T r = x - v + sh[wave];
    __syncthreads();
    return r;
}

// Block totals (the order of a sum is free: lanes read consecutive elements).
template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const T* __restrict__ in, size_t n,
                                                                   T* __restrict__ partial) {
    __shared__ T sh[kScanThreads / 64 + 1];
    const size_t base = (size_t)blockIdx.x * kScanBlock + threadIdx.x;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + (size_t)k * kScanThreads < n) s += in[base + (size_t)k * kScanThreads];
    T tot;
    block_exclusive_scan<T>(s, sh, tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_partials_kernel(T* __restrict__ partial, uint32_t nb) {
    __shared__ T sh[kScanThreads / 64 + 1];
    // each thread owns a contiguous run of ceil(nb / threads) partials;
    // partial[nb] receives the grand total
    uint32_t per = (nb + kScanThreads - 1) / kScanThreads;
    uint32_t b0 = threadIdx.x * per;
    T s = 0;
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < nb) s += partial[b0 + k];
    T tot;
    T off = block_exclusive_scan<T>(s, sh, tot);
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < nb) {
            T t = partial[b0 + k];
            partial[b0 + k] = off;
            off += t;
        }
    if (threadIdx.x == 0) partial[nb] = tot;
}

// Each thread scans its own run of kScanItems elements of `in` into `out`
// (the same array for an in-place scan); with VEC (both 16-byte aligned) a
// whole run is moved with 16-byte loads and stores.
template <typename T, bool VEC>
__global__ __launch_bounds__(kScanThreads) void scan_down_kernel(const T* in, T* out, size_t n,
                                                                 const T* __restrict__ partial, uint32_t nb) {
    __shared__ T sh[kScanThreads / 64 + 1];
    constexpr int kVec = kScanItems * (int)sizeof(T) / 16;
    const size_t base = (size_t)blockIdx.x * kScanBlock + (size_t)threadIdx.x * kScanItems;
    const bool whole = VEC && base + kScanItems <= n;
    T v[kScanItems];
    if (whole) {
        const uint4* p = (const uint4*)(in + base);
        uint4 w[kVec];
#pragma unroll
        for (int k = 0; k < kVec; ++k) w[k] = p[k];
        __builtin_memcpy(v, w, sizeof(v));
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < n) ? in[base + k] : (T)0;
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    T tot;
    T off = block_exclusive_scan<T>(s, sh, tot) + partial[blockIdx.x];
    T o[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = off;
        off += v[k];
    }
    if (whole) {
        uint4 w[kVec];
        __builtin_memcpy(w, o, sizeof(o));
        uint4* p = (uint4*)(out + base);
#pragma unroll
        for (int k = 0; k < kVec; ++k) p[k] = w[k];
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < n) out[base + k] = o[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = partial[nb];
}

// Short arrays in one launch: one block takes the chunks of kScanBlock
// elements in order, carrying the running total (each chunk is read whole
// before any of it is written, so the scan can be in place).  A query batch
// of a few thousand rows then costs one launch instead of three.
constexpr uint32_t kScanSingleChunks = 4;

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_single_kernel(const T* in, T* out, size_t n) {
    __shared__ T sh[kScanThreads / 64 + 1];
    T carry = 0;
    for (size_t c0 = 0; c0 < n; c0 += kScanBlock) {
        const size_t base = c0 + (size_t)threadIdx.x * kScanItems;
        T v[kScanItems];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < n) ? in[base + k] : (T)0;
        T s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) s += v[k];
        T tot;
        T off = block_exclusive_scan<T>(s, sh, tot) + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (base + k < n) out[base + k] = off;
            off += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

// Exclusive scan of in[0..n) into out[0..n) (in place when in == out);
// out[n] receives the total.  `partial` needs ceil(n / kScanBlock) + 1
// elements.
template <typename T>
hipError_t scan_exclusive_to(const T* in, T* out, size_t n, T* partial, hipStream_t st) {
    uint32_t nb = (uint32_t)((n + kScanBlock - 1) / kScanBlock);
    if (nb <= kScanSingleChunks) {
        scan_single_kernel<T><<<1, kScanThreads, 0, st>>>(in, out, n);
        return hipGetLastError();
    }
    scan_reduce_kernel<T><<<nb, kScanThreads, 0, st>>>(in, n, partial);
    scan_partials_kernel<T><<<1, kScanThreads, 0, st>>>(partial, nb);
    if ((((uintptr_t)in | (uintptr_t)out) & 15u) == 0)
        scan_down_kernel<T, true><<<nb, kScanThreads, 0, st>>>(in, out, n, partial, nb);
    else
        scan_down_kernel<T, false><<<nb, kScanThreads, 0, st>>>(in, out, n, partial, nb);
    return hipGetLastError();
}

template <typename T>
hipError_t scan_exclusive(T* data, size_t n, T* partial, hipStream_t st) {
    return scan_exclusive_to<T>(data, data, n, partial, st);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    fill_u32_kernel<<<(uint32_t)blocks, 256, 0, st>>>(p, value, n);
    return hipGetLastError();
}

namespace {

BuildArgs build_args(const sphidx_lattice* lat, const uint32_t* x, const uint32_t* y, const uint32_t* z, uint32_t n) {
    BuildArgs a;
    for (int k = 0; k < 3; ++k) a.lg[k] = lat->desc.log2_cells[k];
    a.F = lat->desc.frac_bits;
    a.cyc = lat->desc.cyclic_mask;
    a.ncells = lat->ncells;
    a.n = n;
    a.x = x;
    a.y = y;
    a.z = z;
    a.recs = nullptr;
    a.count = lat->cell_start;
    a.rank = lat->rank;
    a.pts = lat->pts;
    a.status = lat->status;
    a.out = nullptr;
    return a;
}

}  // namespace

// The attached non-empty cell list of the lattice's current contents (the
// rank array, build scratch, holds the flags and their scan).
hipError_t launch_cell_list(const sphidx_lattice* lat, hipStream_t st) {
    if (!lat->cell_list) return hipSuccess;
    const BuildArgs a = build_args(lat, nullptr, nullptr, nullptr, lat->n);
    const uint32_t blocks = (a.n + 255) / 256;
    if (a.n > 0) cell_flag_kernel<<<blocks, 256, 0, st>>>(a, lat->rank);
    hipError_t e = scan_exclusive<uint32_t>(lat->rank, a.n, lat->scan_tmp, st);
    if (e != hipSuccess) return e;
    cell_list_kernel<<<blocks ? blocks : 1u, 256, 0, st>>>(a, lat->rank, (uint32_t*)lat->cell_list,
                                                          (uint2*)(lat->cell_list + 16));
    return hipGetLastError();
}

hipError_t launch_build(const sphidx_lattice* lat, const uint32_t* x, const uint32_t* y, const uint32_t* z,
                        uint32_t n, hipStream_t st) {
    const BuildArgs a = build_args(lat, x, y, z, n);
    size_t ncount = (size_t)lat->ncells + 2;
    hipError_t e = launch_fill_u32(lat->cell_start, 0u, ncount + 1, st);
    if (e != hipSuccess) return e;
    const bool xo = lat->cell_order == SPHIDX_ORDER_X;
    // the x-order word: set here, cleared by a cell too large to order
    if ((e = launch_fill_u32(lat->status + 1, xo ? 1u : 0u, 1, st)) != hipSuccess) return e;
    uint32_t blocks = (n + 255) / 256;
    if (n > 0) hist_kernel<<<blocks, 256, 0, st>>>(a);
    e = scan_exclusive<uint32_t>(lat->cell_start, ncount, lat->scan_tmp, st);
    if (e != hipSuccess) return e;
    if (xo && lat->xbuf) {
        // the counting sort into the second array, then ranked into place
        BuildArgs ax = a;
        ax.pts = lat->xbuf;
        ax.out = lat->pts;
        if (n > 0) {
            scatter_kernel<<<blocks, 256, 0, st>>>(ax);
            xrank_kernel<<<blocks, 256, 0, st>>>(ax);
        }
    } else if (n > 0) {
        scatter_kernel<<<blocks, 256, 0, st>>>(a);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_cell_list(lat, st);
}

size_t scan_i64_tmp_bytes(uint32_t n) {
    size_t nb = ((size_t)n + kScanBlock - 1) / kScanBlock + 2;
    return nb * sizeof(int64_t);
}

hipError_t launch_scan_i64(int64_t* data, uint32_t n, void* tmp, hipStream_t st) {
    return scan_exclusive<int64_t>(data, n, (int64_t*)tmp, st);
}

size_t scan_u32_tmp_words(size_t n) { return (n + kScanBlock - 1) / kScanBlock + 2; }

hipError_t launch_scan_u32(uint32_t* data, size_t n, uint32_t* tmp, hipStream_t st) {
    return scan_exclusive<uint32_t>(data, n, tmp, st);
}

hipError_t launch_scan_u32_to(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp, hipStream_t st) {
    return scan_exclusive_to<uint32_t>(in, out, n, tmp, st);
}

// Rebuild from records (incremental maintenance): the same counting sort over
// `recs` (n records, not the lattice's own array) into the lattice's records.
hipError_t launch_build_records(const sphidx_lattice* lat, const uint4* recs, uint32_t n, hipStream_t st) {
    BuildArgs a = build_args(lat, nullptr, nullptr, nullptr, n);
    a.recs = recs;
    size_t ncount = (size_t)lat->ncells + 2;
    hipError_t e = launch_fill_u32(lat->cell_start, 0u, ncount + 1, st);
    if (e != hipSuccess) return e;
    // cells in the counting sort's order
    if ((e = launch_fill_u32(lat->status + 1, 0u, 1, st)) != hipSuccess) return e;
    uint32_t blocks = (n + 255) / 256;
    if (n > 0) hist_records_kernel<<<blocks, 256, 0, st>>>(a);
    e = scan_exclusive<uint32_t>(lat->cell_start, ncount, lat->scan_tmp, st);
    if (e != hipSuccess) return e;
    if (n > 0) scatter_records_kernel<<<blocks, 256, 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_cell_list(lat, st);
}
