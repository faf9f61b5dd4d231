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
    gp<T> __restrict__ u = (gp<T>)L.u;
    gcp<T> __restrict__ f = (gcp<T>)L.rhs;
    const long long nn = L.nn;
    const int c = ((gcp<uint8_t>)L.cls)[p];
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

}  // namespace bcmg
