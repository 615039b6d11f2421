// Serving loop: batches of queries against one device-resident lattice, with
// continuous batching.  Each slot owns a stream (default priority), its
// inputs (device and pinned staging), its row_ptr and its query workspace;
// the server owns one output pool.  A batch starts when a slot is free (its
// inputs staged and its count pass launched), is admitted to the write pass
// in arrival order once its exact output fits the pool (first fit), and
// releases its slot and pool range when its write is seen complete.  The
// loop polls events; it never waits on a stream, so the batches' kernels
// overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <thread>
#include <utility>
#include <vector>

#include "sphidx_internal.h"

namespace {

constexpr size_t kPoolAlign = 256;

// First-fit allocator over [0, size) with a coalescing free list.
struct Pool {
    size_t size = 0;
    std::vector<std::pair<size_t, size_t>> free;  // (offset, length), sorted by offset

    void reset(size_t n) {
        size = n;
        free.assign(1, {0, n});
    }
    bool alloc(size_t n, size_t* off) {
        for (size_t i = 0; i < free.size(); ++i) {
            if (free[i].second >= n) {
                *off = free[i].first;
                if (free[i].second == n)
                    free.erase(free.begin() + (long)i);
                else
                    free[i] = {free[i].first + n, free[i].second - n};
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto it = std::lower_bound(free.begin(), free.end(), std::make_pair(off, (size_t)0));
        it = free.insert(it, {off, n});
        // merge with the next range, then with the previous one
        auto nx = it + 1;
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = it - 1;
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
};

enum SlotState { kIdle = 0, kCounting = 1, kWaiting = 2, kWriting = 3 };

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t counted = nullptr, written = nullptr;
    uint32_t* d_in = nullptr;      // one batch's x | y | z | radius | k, packed
    uint32_t* h_in = nullptr;      // pinned staging of the same
    int64_t* d_row_ptr = nullptr;  // max_batch + 1
    int64_t* h_total = nullptr;    // pinned: row_ptr[count] of the count pass
    void* d_ws = nullptr;
    size_t ws_bytes = 0;
    sphidx_queries q{};
    int state = kIdle;
    uint32_t batch = 0;
    size_t off = 0, nbytes = 0;
};

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct sphidx_server {
    const sphidx_lattice* lat = nullptr;
    const sphidx_tables* tab = nullptr;
    sphidx_launch launch{};
    bool has_launch = false;
    uint32_t max_batch = 0;
    char* d_pool = nullptr;
    Pool pool;
    std::vector<Slot> slots;
};

namespace {

void free_server(sphidx_server* s) {
    if (!s) return;
    for (Slot& sl : s->slots) {
        if (sl.st) (void)hipStreamSynchronize(sl.st);
        if (sl.counted) (void)hipEventDestroy(sl.counted);
        if (sl.written) (void)hipEventDestroy(sl.written);
        if (sl.d_in) (void)hipFree(sl.d_in);
        if (sl.h_in) (void)hipHostFree(sl.h_in);
        if (sl.d_row_ptr) (void)hipFree(sl.d_row_ptr);
        if (sl.h_total) (void)hipHostFree(sl.h_total);
        if (sl.d_ws) (void)hipFree(sl.d_ws);
        if (sl.st) {
            forget_stream((void*)sl.st);
            (void)hipStreamDestroy(sl.st);
        }
    }
    if (s->d_pool) (void)hipFree(s->d_pool);
    delete s;
}

sphidx_status launch_count(sphidx_server* s, Slot& sl, const sphidx_batch& b) {
    const uint32_t n = b.count;
    uint32_t* h = sl.h_in;
    std::memcpy(h, b.x, (size_t)n * 4);
    std::memcpy(h + n, b.y, (size_t)n * 4);
    std::memcpy(h + 2 * (size_t)n, b.z, (size_t)n * 4);
    std::memcpy(h + 3 * (size_t)n, b.radius_fx, (size_t)n * 4);
    if (b.k) std::memcpy(h + 4 * (size_t)n, b.k, (size_t)n * 4);
    const size_t bytes = (size_t)n * 4 * (b.k ? 5 : 4);
    if (hipMemcpyAsync(sl.d_in, h, bytes, hipMemcpyHostToDevice, sl.st) != hipSuccess) return SPHIDX_ERR_DEVICE;
    sphidx_queries& q = sl.q;
    std::memset(&q, 0, sizeof(q));
    q.count = n;
    q.x_dev = sl.d_in;
    q.y_dev = sl.d_in + n;
    q.z_dev = sl.d_in + 2 * (size_t)n;
    q.radius_fx_dev = sl.d_in + 3 * (size_t)n;
    q.k_dev = b.k ? sl.d_in + 4 * (size_t)n : nullptr;
    q.mode = b.k ? SPHIDX_MODE_MIXED : SPHIDX_MODE_RADIUS;
    sphidx_csr c{};
    c.row_ptr_dev = sl.d_row_ptr;
    c.capacity = 0;
    c.workspace_dev = sl.d_ws;
    c.workspace_bytes = sl.ws_bytes;
    const sphidx_status st = sphidx_count(s->lat, s->tab, &q, &c, s->has_launch ? &s->launch : nullptr, sl.st);
    if (st != SPHIDX_OK) return st;
    if (hipMemcpyAsync(sl.h_total, sl.d_row_ptr + n, 8, hipMemcpyDeviceToHost, sl.st) != hipSuccess)
        return SPHIDX_ERR_DEVICE;
    if (hipEventRecord(sl.counted, sl.st) != hipSuccess) return SPHIDX_ERR_DEVICE;
    return SPHIDX_OK;
}

sphidx_status launch_write(sphidx_server* s, Slot& sl, const sphidx_batch& b, int64_t pairs) {
    sphidx_csr c{};
    c.row_ptr_dev = sl.d_row_ptr;
    c.ids_dev = (uint32_t*)(s->d_pool + sl.off);
    c.capacity = (int64_t)(sl.nbytes / 4);
    c.workspace_dev = sl.d_ws;
    c.workspace_bytes = sl.ws_bytes;
    const sphidx_status st = sphidx_write(s->lat, s->tab, &sl.q, &c, s->has_launch ? &s->launch : nullptr, sl.st);
    if (st != SPHIDX_OK) return st;
    if (b.row_ptr_out &&
        hipMemcpyAsync(b.row_ptr_out, sl.d_row_ptr, ((size_t)b.count + 1) * 8, hipMemcpyDeviceToHost, sl.st) !=
            hipSuccess)
        return SPHIDX_ERR_DEVICE;
    if (b.ids_out && pairs > 0 && (uint64_t)pairs <= b.ids_capacity &&
        hipMemcpyAsync(b.ids_out, c.ids_dev, (size_t)pairs * 4, hipMemcpyDeviceToHost, sl.st) != hipSuccess)
        return SPHIDX_ERR_DEVICE;
    if (hipEventRecord(sl.written, sl.st) != hipSuccess) return SPHIDX_ERR_DEVICE;
    return SPHIDX_OK;
}

}  // namespace

extern "C" {

sphidx_status sphidx_server_create(const sphidx_lattice* lat, const sphidx_tables* tab, uint32_t slots,
                                   uint32_t max_batch, size_t pool_bytes, uint64_t stash_pairs,
                                   const sphidx_launch* launch, sphidx_server** out) {
    if (!out) return SPHIDX_ERR_INVALID_ARG;
    *out = nullptr;
    if (!lat || slots == 0 || max_batch == 0 || pool_bytes < kPoolAlign) return SPHIDX_ERR_INVALID_ARG;
    const sphidx_status lc = check_launch(launch, tab);
    if (lc != SPHIDX_OK) return lc;
    sphidx_server* s = new sphidx_server();
    s->lat = lat;
    s->tab = tab;
    if (launch) {
        s->launch = *launch;
        // per-call outputs have no meaning across overlapping batches
        s->launch.stats_dev = nullptr;
        s->launch.method_dev = nullptr;
        s->launch.event_begin = nullptr;
        s->launch.event_end = nullptr;
        s->has_launch = true;
    }
    s->max_batch = max_batch;
    const size_t pool = pool_bytes / kPoolAlign * kPoolAlign;
    if (hipMalloc((void**)&s->d_pool, pool) != hipSuccess) {
        free_server(s);
        return SPHIDX_ERR_OUT_OF_MEMORY;
    }
    s->pool.reset(pool);
    const size_t ws = sphidx_query_workspace_bytes(max_batch) + (stash_pairs ? sphidx_query_stash_bytes(stash_pairs, 0) : 0);
    s->slots.resize(slots);
    for (Slot& sl : s->slots) {
        sl.ws_bytes = ws;
        bool ok = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&sl.counted, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&sl.written, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            free_server(s);
            return SPHIDX_ERR_DEVICE;
        }
        ok = hipMalloc((void**)&sl.d_in, (size_t)max_batch * 20) == hipSuccess &&
             hipHostMalloc((void**)&sl.h_in, (size_t)max_batch * 20, hipHostMallocDefault) == hipSuccess &&
             hipMalloc((void**)&sl.d_row_ptr, ((size_t)max_batch + 1) * 8) == hipSuccess &&
             hipHostMalloc((void**)&sl.h_total, 8, hipHostMallocDefault) == hipSuccess &&
             hipMalloc(&sl.d_ws, ws) == hipSuccess;
        if (!ok || hipMemset(sl.d_ws, 0, ws) != hipSuccess) {
            free_server(s);
            return SPHIDX_ERR_OUT_OF_MEMORY;
        }
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        free_server(s);
        return SPHIDX_ERR_DEVICE;
    }
    *out = s;
    return SPHIDX_OK;
}

void sphidx_server_destroy(sphidx_server* s) { free_server(s); }

sphidx_status sphidx_server_run(sphidx_server* s, uint32_t nbatch, const sphidx_batch* batches,
                                sphidx_batch_result* results) {
    if (!s || (nbatch && (!batches || !results))) return SPHIDX_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < nbatch; ++i) {
        const sphidx_batch& b = batches[i];
        if (b.count > s->max_batch) return SPHIDX_ERR_INVALID_ARG;
        if (b.count && (!b.x || !b.y || !b.z || !b.radius_fx)) return SPHIDX_ERR_INVALID_ARG;
        if (i && b.arrival_s < batches[i - 1].arrival_s) return SPHIDX_ERR_INVALID_ARG;
        std::memset(&results[i], 0, sizeof(results[i]));
    }
    for (Slot& sl : s->slots) sl.state = kIdle;
    const auto t0 = std::chrono::steady_clock::now();
    auto clock = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    std::vector<uint32_t> free_slots;
    for (uint32_t i = 0; i < (uint32_t)s->slots.size(); ++i) free_slots.push_back((uint32_t)s->slots.size() - 1 - i);
    std::deque<uint32_t> waiting;  // slots whose count is done, in arrival order
    uint32_t next = 0, busy = 0;
    uint64_t in_use = 0;
    sphidx_status first = SPHIDX_OK;
    auto finish = [&](uint32_t si, double t, sphidx_status st) {
        Slot& sl = s->slots[si];
        results[sl.batch].done_s = t;
        if (st != SPHIDX_OK && results[sl.batch].status == SPHIDX_OK) results[sl.batch].status = st;
        if (sl.nbytes) {
            s->pool.release(sl.off, sl.nbytes);
            in_use -= sl.nbytes;
        }
        sl.nbytes = 0;
        sl.state = kIdle;
        free_slots.push_back(si);
        --busy;
    };
    while (next < nbatch || busy) {
        bool progressed = false;
        double now = clock();
        // arrivals, while a slot is free (an error stops further starts)
        while (first == SPHIDX_OK && next < nbatch && batches[next].arrival_s <= now && !free_slots.empty()) {
            const sphidx_batch& b = batches[next];
            results[next].start_s = now;
            if (b.count == 0) {
                // nothing to run: an empty row_ptr
                if (b.row_ptr_out) b.row_ptr_out[0] = 0;
                results[next].done_s = now;
                ++next;
                progressed = true;
                continue;
            }
            const uint32_t si = free_slots.back();
            free_slots.pop_back();
            Slot& sl = s->slots[si];
            sl.batch = next;
            sl.nbytes = 0;
            sl.state = kCounting;
            ++busy;
            const sphidx_status st = launch_count(s, sl, b);
            ++next;
            progressed = true;
            if (st != SPHIDX_OK) {
                first = st;
                (void)hipStreamSynchronize(sl.st);
                finish(si, clock(), st);
            }
        }
        // counts done
        for (uint32_t si = 0; si < (uint32_t)s->slots.size(); ++si) {
            Slot& sl = s->slots[si];
            if (sl.state != kCounting) continue;
            const hipError_t e = hipEventQuery(sl.counted);
            if (e == hipErrorNotReady) continue;
            progressed = true;
            if (e != hipSuccess) {
                first = first == SPHIDX_OK ? SPHIDX_ERR_DEVICE : first;
                finish(si, clock(), SPHIDX_ERR_DEVICE);
                continue;
            }
            results[sl.batch].pairs = *sl.h_total;
            sl.state = kWaiting;
            waiting.push_back(si);
        }
        // admission by memory, in arrival order
        while (!waiting.empty()) {
            const uint32_t si = waiting.front();
            Slot& sl = s->slots[si];
            const int64_t pairs = results[sl.batch].pairs;
            const size_t need = round_up((size_t)std::max<int64_t>(pairs, 1) * 4, kPoolAlign);
            if (need > s->pool.size) {
                results[sl.batch].rejected = 1;
                waiting.pop_front();
                finish(si, clock(), SPHIDX_OK);
                progressed = true;
                continue;
            }
            size_t off = 0;
            if (!s->pool.alloc(need, &off)) break;
            waiting.pop_front();
            sl.off = off;
            sl.nbytes = need;
            sl.state = kWriting;
            in_use += need;
            results[sl.batch].admit_s = clock();
            results[sl.batch].pool_in_use = in_use;
            progressed = true;
            const sphidx_status st = launch_write(s, sl, batches[sl.batch], pairs);
            if (st != SPHIDX_OK) {
                first = first == SPHIDX_OK ? st : first;
                (void)hipStreamSynchronize(sl.st);
                finish(si, clock(), st);
            }
        }
        // writes done
        for (uint32_t si = 0; si < (uint32_t)s->slots.size(); ++si) {
            Slot& sl = s->slots[si];
            if (sl.state != kWriting) continue;
            const hipError_t e = hipEventQuery(sl.written);
            if (e == hipErrorNotReady) continue;
            progressed = true;
            finish(si, clock(), e == hipSuccess ? SPHIDX_OK : SPHIDX_ERR_DEVICE);
            if (e != hipSuccess && first == SPHIDX_OK) first = SPHIDX_ERR_DEVICE;
        }
        if (first != SPHIDX_OK && busy == 0) break;
        if (!progressed) std::this_thread::yield();
    }
    for (uint32_t i = next; i < nbatch; ++i) results[i].status = first;
    return first;
}

}  // extern "C"
