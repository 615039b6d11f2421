// Query entry point that allocates nothing: for callers that cannot call
// hipMalloc (code under HIP graph capture, tight serving loops, harnesses that
// forbid allocation).  The query workspace -- work-queue counters, per-query
// descriptors, query lists, scan partials and the stash of sorted rows -- is a
// fixed array in device memory that the code object brings with it, one copy
// per GPU, held until the process ends.  Everything else is sphidx_query.
#include <mutex>

#include "sphidx_internal.h"

// The workspace of every sphidx_query_noalloc call on a GPU.  In host code
// this name is only a stand-in for the symbol: its device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[SPHIDX_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up on the
// first call made with that device current.
sphidx_status scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPHIDX_ERR_DEVICE;
    if (dev < 0 || dev >= kMaxDevices) return SPHIDX_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SPHIDX_ERR_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SPHIDX_OK;
}

}  // namespace

extern "C" sphidx_status sphidx_query_noalloc(const sphidx_lattice* lat, const sphidx_tables* tab,
                                              const sphidx_queries* q, sphidx_csr* csr,
                                              const sphidx_launch* launch, void* stream) {
    if (!lat || !q || !csr) return SPHIDX_ERR_INVALID_ARG;
    // the workspace is the library's: a caller's would be ignored, so it is
    // refused rather than silently unused
    if (csr->workspace_dev || csr->workspace_bytes) return SPHIDX_ERR_INVALID_ARG;
    if (q->count > SPHIDX_NOALLOC_MAX_QUERIES) return SPHIDX_ERR_CAPACITY;
    // tables are uploaded when they are built or loaded on a host with a
    // device; a query must not upload them here
    const uint32_t method = launch ? launch->method : SPHIDX_METHOD_SPHERE;
    const bool tables = method == SPHIDX_METHOD_SPHERE || method == SPHIDX_METHOD_AUTO ||
                        method == SPHIDX_METHOD_PAPER64;
    if (tables && tab && !tab->d_rows) return SPHIDX_ERR_INVALID_ARG;
    void* ws = nullptr;
    const sphidx_status s = scratch_address(&ws);
    if (s != SPHIDX_OK) return s;
    sphidx_csr c = *csr;
    c.workspace_dev = ws;
    c.workspace_bytes = SPHIDX_NOALLOC_SCRATCH_BYTES;
    return sphidx_query(lat, tab, q, &c, launch, stream);
}
