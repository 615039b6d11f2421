// Moving agents (dynamic objects whose positions change every step,
// Section I) and the order-independent checksum of per-row neighbour counts.
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
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < Q; i += gridDim.x * blockDim.x) {
        uint64_t c = (uint64_t)(row_ptr[i + 1] - row_ptr[i]);
        s += c;
        h += mix64(((uint64_t)i << 32) | (c & 0xffffffffull));
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
