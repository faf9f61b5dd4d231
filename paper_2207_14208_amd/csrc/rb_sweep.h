// Red-black Gauss-Seidel sweep of the interior (INSIDE) rows: one colour of
// one row segment per wavefront.
#pragma once

#include "seg.h"

namespace bcmg {

// ------------------------------------------------------------ node updates
// Interior Gauss-Seidel on the nodes of one colour of a segment (red:
// i+j+k even), one node per lane.  eq. GSLEX_2D in red-black order:
// u_P = (h^2 f_P + sum of the 2d neighbours) / (2d + c h^2), c the reaction
// coefficient of c u - Laplace u (0 for Poisson).
template <int D, typename T>
__device__ __forceinline__ void seg_rb(const Desc &L, const Item &it, int lane, int colour, bool live) {
    const Seg s = seg_of(it);
    const int q = (((s.x0 + s.yj + s.zk) & 1) == colour ? 0 : 1) + 2 * lane;
    const long long p = s.p0 + (q < s.len ? q : 0);
    const NodeArr<T> u = node_u<T>(L);
    const NodeArr<const T> f = node_rhs<const T>(L);
    const long long nn = L.nn;
    int c = C_INSIDE;  // segments of INSIDE nodes only skip the class load
    if (!s.all_inside) c = ((gcp<uint8_t>)L.cls)[p];
    const T fp = f[p];
    const T xm = u[clampi(p - 1, nn)], xp = u[clampi(p + 1, nn)];
    T ym = 0, yp = 0, zm = 0, zp = 0;
    if (D >= 2) {
        ym = u[clampi(p - L.sy, nn)];
        yp = u[clampi(p + L.sy, nn)];
    }
    if (D >= 3) {
        zm = u[clampi(p - L.sz, nn)];
        zp = u[clampi(p + L.sz, nn)];
    }
    T sum = xp + xm;
    if (D >= 2) sum += yp + ym;
    if (D >= 3) sum += zp + zm;
    const T v = ((T)L.h2 * fp + sum) / (T)(2.0 * D + L.reaction * L.h2);
    pin(v);
    pin(c);
    if (q >= s.len || c != C_INSIDE || !live) return;
    u[p] = v;
}

template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_rb_sweep(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                     int nseg, int colour, const SlotState *__restrict__ st) {
    SEG_ITEM
    seg_rb<D, T>(L, it, lane, colour, live);
}

// The same sweep with S consecutive segments per wavefront: every load of
// the S segments is issued before the first wait, so a wavefront keeps S
// times the bytes in flight and the launch needs S times fewer wavefronts
// (each carries a chain of dependent loads: item, descriptor, data).
template <int D, typename T, int S>
__global__ __launch_bounds__(kBlock) void k_rb_sweep_multi(const Desc *__restrict__ descs,
                                                           const Item *__restrict__ items, int nseg, int colour,
                                                           const SlotState *__restrict__ st) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int first = __builtin_amdgcn_readfirstlane((xcd_block() * kWavesPerBlock + wave) * S);
    if (first >= nseg) return;
    T v[S];
    long long pw[S];
    int cw[S];
    bool ok[S];
    NodeArr<T> uw[S];
#pragma unroll
    for (int j = 0; j < S; j++) {
        const int sidx = first + j < nseg ? first + j : nseg - 1;
        const Item it = items[sidx];
        const Desc &L = descs[it.x];
        const Seg sg = seg_of(it);
        const int q = (((sg.x0 + sg.yj + sg.zk) & 1) == colour ? 0 : 1) + 2 * lane;
        const long long p = sg.p0 + (q < sg.len ? q : 0);
        const NodeArr<T> u = node_u<T>(L);
        const NodeArr<const T> f = node_rhs<const T>(L);
        const long long nn = L.nn;
        cw[j] = C_INSIDE;
        if (!sg.all_inside) cw[j] = ((gcp<uint8_t>)L.cls)[p];
        const T fp = f[p];
        const T xm = u[clampi(p - 1, nn)], xp = u[clampi(p + 1, nn)];
        T ym = 0, yp = 0, zm = 0, zp = 0;
        if (D >= 2) {
            ym = u[clampi(p - L.sy, nn)];
            yp = u[clampi(p + L.sy, nn)];
        }
        if (D >= 3) {
            zm = u[clampi(p - L.sz, nn)];
            zp = u[clampi(p + L.sz, nn)];
        }
        T sum = xp + xm;
        if (D >= 2) sum += yp + ym;
        if (D >= 3) sum += zp + zm;
        v[j] = ((T)L.h2 * fp + sum) / (T)(2.0 * D + L.reaction * L.h2);
        pw[j] = p;
        uw[j] = u;
        ok[j] = first + j < nseg && q < sg.len && st[L.slot].active != 0;
    }
#pragma unroll
    for (int j = 0; j < S; j++) {
        pin(v[j]);
        pin(cw[j]);
    }
#pragma unroll
    for (int j = 0; j < S; j++)
        if (ok[j] && cw[j] == C_INSIDE) uw[j][pw[j]] = v[j];
}

}  // namespace bcmg
