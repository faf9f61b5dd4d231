// Row segments: decoding of a segment work item and the per-wavefront
// prologue shared by the segment kernels.
#pragma once

#include "bcmg_internal.h"

namespace bcmg {

struct Seg {
    long long p0;  // first node
    int len, x0, yj, zk;
};

__device__ __forceinline__ Seg seg_of(const Item &it) {
    Seg s;
    s.p0 = it.y;
    s.len = it.z >> 16;
    s.x0 = it.z & 0xffff;
    s.yj = it.w & 0xffff;
    s.zk = it.w >> 16;
    return s;
}

__device__ __forceinline__ long long clampi(long long q, long long nn) { return q < 0 ? 0 : (q >= nn ? nn - 1 : q); }

// One wavefront per segment item; returns early for padding waves and for
// problems whose slot is no longer active.
#define SEG_ITEM                                                  \
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;   \
    const int sidx = blockIdx.x * kWavesPerBlock + wave;          \
    if (sidx >= nseg) return;                                     \
    const Item it = items[sidx];                                  \
    const Desc &L = descs[it.x];                                  \
    if (!st[L.slot].active) return;

}  // namespace bcmg
