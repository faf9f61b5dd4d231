// Row segments: decoding of a segment work item and the per-wavefront
// prologue shared by the segment kernels.
#pragma once

#include "bcmg_internal.h"

namespace bcmg {

// Pointers into global memory.  Pointers kept in descriptors are generic;
// casting them to the global address space makes the compiler emit global
// (not flat) loads, which a wavefront can wait for without also waiting for
// its outstanding scalar loads.
template <typename T>
using gp = __attribute__((address_space(1))) T *;
template <typename T>
using gcp = const __attribute__((address_space(1))) T *;

// A level's node array, indexed by the x-fastest node index p.  A split
// array stores the nodes of even p first, then those of odd p: with n = N + 1
// odd, the parity of p is the colour (i + j + k) mod 2 of red-black ordering,
// and every axis neighbour has the other parity, so a colour pass reads one
// half contiguously and writes the other.  half = the number of even indices
// ((nn + 1) / 2) for a split array, 0 for the natural order.
template <typename T>
struct NodeArr {
    gp<T> a;
    long long half;
    __device__ __forceinline__ long long at(long long p) const {
        return half ? (p >> 1) + ((p & 1) ? half : 0LL) : p;
    }
    __device__ __forceinline__ __attribute__((address_space(1))) T &operator[](long long p) const { return a[at(p)]; }
};

// the descriptor's u and rhs (one layout) and r (its own layout)
template <typename T>
__device__ __forceinline__ NodeArr<T> node_u(const Desc &L) { return NodeArr<T>{(gp<T>)L.u, L.half_u}; }
template <typename T>
__device__ __forceinline__ NodeArr<T> node_rhs(const Desc &L) { return NodeArr<T>{(gp<T>)L.rhs, L.half_u}; }
template <typename T>
__device__ __forceinline__ NodeArr<T> node_r(const Desc &L) { return NodeArr<T>{(gp<T>)L.r, L.half_r}; }

// Node q of a row segment that lane takes as its h-th node (two per lane):
// lane + 64 h keeps each load of a natural-order array contiguous across the
// wavefront; 2 lane + h does so for a split array (each h is one parity).
__device__ __forceinline__ int seg_lane_node(int lane, int h, long long half) {
    return half ? 2 * lane + h : lane + 64 * h;
}

struct Seg {
    long long p0;  // first node
    int len, x0, yj, zk;
    bool all_inside;  // every node of the segment is INSIDE
};

__device__ __forceinline__ Seg seg_of(const Item &it) {
    Seg s;
    s.p0 = it.y;
    s.len = (it.z >> 16) & 0xff;
    s.x0 = it.z & 0xffff;
    s.all_inside = (it.z & kSegAllInside) != 0;
    s.yj = it.w & 0xffff;
    s.zk = it.w >> 16;
    return s;
}

__device__ __forceinline__ long long clampi(long long q, long long nn) { return q < 0 ? 0 : (q >= nn ? nn - 1 : q); }

// Workgroups are handed to the chip's 8 XCDs round-robin (workgroup b to
// XCD b mod 8), and each XCD has its own L2.  The logical workgroup index
// gives every XCD one contiguous range of the work list, so that the rows a
// stencil shares (y and z neighbours) are fetched into the same L2.
// A grid may hold two lists, nfirst blocks of one (row segments) followed
// by blocks of another (chunks); each XCD then gets one contiguous range of
// each list, in even shares.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int nfirst) {
    const int b = blockIdx.x, nb = gridDim.x;
    const int x = b % kXcds, i = b / kXcds;
    const int qa = nfirst / kXcds, ra = nfirst % kXcds;       // first list: blocks per XCD
    const int qt = nb / kXcds, rt = nb % kXcds;               // whole grid: blocks per XCD
    const int na = qa + (x < ra ? 1 : 0);
    const int abeg = x * qa + min(x, ra);
    if (i < na) return abeg + i;
    const int tbeg = x * qt + min(x, rt);
    return nfirst + (tbeg - abeg) + (i - na);
}
__device__ __forceinline__ int xcd_block() { return xcd_block(gridDim.x); }

// Keeps the computation of v, and the loads it needs, ahead of the branches
// that follow: a wavefront then issues all of its loads before it first
// waits, instead of waiting once per test (the compiler would otherwise sink
// loads whose results are only used under a condition).
template <typename V>
__device__ __forceinline__ void pin(const V &v) {
    asm volatile("" ::"v"(v));
}

// One wavefront per segment item; returns early for padding waves.  live
// tells whether the item's problem still iterates; node updates test it
// just before their stores, so its load overlaps the data loads.
#define SEG_ITEM SEG_ITEM_AT(xcd_block())
#define SEG_ITEM_AT(lblock)                                                              \
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;                          \
    const int sidx = __builtin_amdgcn_readfirstlane((lblock) * kWavesPerBlock + wave);   \
    if (sidx >= nseg) return;                                                            \
    const Item it = items[sidx];                                                         \
    const Desc L = descs[it.x];                                                          \
    const bool live = st[L.slot].active != 0;

}  // namespace bcmg
