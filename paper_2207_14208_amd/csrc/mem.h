// Device memory of the library (see mem.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "bcmg.h"

namespace bcmg {

// Where a problem's or a batch's device memory comes from: the caller's
// callbacks, or (both null) the library's private pool on `device`.
struct MemSource {
    bcmg_alloc_fn alloc = nullptr;
    bcmg_free_fn free = nullptr;
    void *ctx = nullptr;
    int device = 0;
};

void mem_set_source(bcmg_alloc_fn alloc, bcmg_free_fn free, void *ctx);
// the source in effect now, on the current device (problems and batches keep
// the one they were created with)
MemSource mem_current();
hipError_t mem_alloc(const MemSource &m, void **p, size_t bytes, hipStream_t s);
void mem_free(const MemSource &m, void *p, hipStream_t s);

// Temporaries of setup kernels come from the source bound to the calling
// thread by a MemScope (the private pool when none is bound).
struct MemScope {
    explicit MemScope(const MemSource &m);
    ~MemScope();
    const MemSource *prev;
};
hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t s);
void scratch_free(void *p, hipStream_t s);

}  // namespace bcmg
