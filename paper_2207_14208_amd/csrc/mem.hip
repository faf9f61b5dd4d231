// Device memory of the library.  Every device allocation goes through one
// source: the caller's callbacks (bcmg_set_allocator) or, without them, a
// private stream-ordered pool per device that keeps freed memory for the
// next problem (the process's default pool and its release threshold are
// left alone).  Allocations are stream-ordered: a free names the stream that
// last used the memory, and the memory may be handed out again only in that
// stream's order.
#include <cstdint>
#include <mutex>
#include <unordered_map>

#include "mem.h"

namespace bcmg {

namespace {

std::mutex g_mu;
MemSource g_source;                               // set by bcmg_set_allocator
std::unordered_map<void *, size_t> g_sizes;       // live allocations and their sizes
hipMemPool_t g_pools[64] = {};
thread_local const MemSource *t_scope = nullptr;  // source of setup temporaries on this thread

hipMemPool_t private_pool(int dev) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (dev < 0 || dev >= 64) return nullptr;
    if (!g_pools[dev]) {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        if (hipMemPoolCreate(&pool, &props) != hipSuccess) return nullptr;
        uint64_t keep = UINT64_MAX;
        hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        g_pools[dev] = pool;
    }
    return g_pools[dev];
}

}  // namespace

void mem_set_source(bcmg_alloc_fn alloc, bcmg_free_fn free, void *ctx) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_source.alloc = alloc;
    g_source.free = free;
    g_source.ctx = ctx;
}

MemSource mem_current() {
    MemSource m;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        m = g_source;
    }
    if (hipGetDevice(&m.device) != hipSuccess) m.device = 0;
    return m;
}

hipError_t mem_alloc(const MemSource &m, void **p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipSuccess;
    if (m.alloc) {
        *p = m.alloc(bytes, (void *)s, m.ctx);
        if (!*p) e = hipErrorOutOfMemory;
    } else {
        hipMemPool_t pool = private_pool(m.device);
        e = pool ? hipMallocFromPoolAsync(p, bytes, pool, s) : hipMallocAsync(p, bytes, s);
        if (e != hipSuccess) *p = nullptr;
    }
    if (*p) {
        std::lock_guard<std::mutex> lock(g_mu);
        g_sizes[*p] = bytes;
    }
    return e;
}

void mem_free(const MemSource &m, void *p, hipStream_t s) {
    if (!p) return;
    size_t bytes = 0;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_sizes.find(p);
        if (it != g_sizes.end()) {
            bytes = it->second;
            g_sizes.erase(it);
        }
    }
    if (m.free)
        m.free(p, bytes, (void *)s, m.ctx);
    else
        hipFreeAsync(p, s);
}

MemScope::MemScope(const MemSource &m) : prev(t_scope) { t_scope = &m; }
MemScope::~MemScope() { t_scope = prev; }

hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t s) {
    static const MemSource none{};
    return mem_alloc(t_scope ? *t_scope : none, p, bytes, s);
}

void scratch_free(void *p, hipStream_t s) {
    static const MemSource none{};
    mem_free(t_scope ? *t_scope : none, p, s);
}

}  // namespace bcmg
