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

// The sweep of a level stored split by node parity (FP32; see NodeArr), four
// row segments per wavefront, sixteen lanes per segment and four consecutive
// nodes of the colour per lane.  In split storage the nodes of one colour of a
// segment are consecutive in that colour's half, and so are, in the other
// half, their x, y and z neighbours: a lane reads them with 16-byte loads
// (five values for the x neighbours, four for f and for each other axis),
// four times fewer load instructions for the same bytes.  The update is
// seg_rb's, node by node (the same result).  Split arrays carry kSplitPad
// spare entries, so a lane's loads past the last node stay in the array.
using f32x4u = float __attribute__((ext_vector_type(4), aligned(4)));

template <int D>
__device__ __forceinline__ void split4_lane(const Desc &L, const Item &it, int t, int colour, bool live) {
    const Seg s = seg_of(it);
    const int q0 = ((s.x0 + s.yj + s.zk) & 1) == colour ? 0 : 1;  // first node of the colour
    const int ncol = s.len > q0 ? (s.len - q0 + 1) >> 1 : 0;     // nodes of the colour
    const int i0 = 4 * t;
    const int nv = min(max(ncol - i0, 0), 4);
    if (nv <= 0) return;
    const long long pc = s.p0 + q0 + 2 * i0;  // the lane's first node
    const long long half = L.half_u;
    const long long chalf = (pc & 1) ? half : 0, ohalf = (pc & 1) ? 0 : half;
    // start of a 5-wide read at most here (only lanes without INSIDE nodes,
    // on the box faces, reach past the array or below 0; their values are not used)
    const long long lim = L.nn + kSplitPad - 5;
    auto base = [&](long long b) { return b < 0 ? 0LL : (b > lim ? lim : b); };
    gcp<float> U = (gcp<float>)L.u;
    gcp<float> F = (gcp<float>)L.rhs;
    const long long bc = chalf + (pc >> 1);
    const long long bx = base(ohalf + ((pc - 1) >> 1));
    const f32x4u f4 = *(gcp<f32x4u>)(F + base(bc));
    const f32x4u x4 = *(gcp<f32x4u>)(U + bx);
    const float x5 = U[bx + 4];
    f32x4u ym4 = {0, 0, 0, 0}, yp4 = {0, 0, 0, 0}, zm4 = {0, 0, 0, 0}, zp4 = {0, 0, 0, 0};
    if (D >= 2) {
        ym4 = *(gcp<f32x4u>)(U + base(ohalf + ((pc - L.sy) >> 1)));
        yp4 = *(gcp<f32x4u>)(U + base(ohalf + ((pc + L.sy) >> 1)));
    }
    if (D >= 3) {
        zm4 = *(gcp<f32x4u>)(U + base(ohalf + ((pc - L.sz) >> 1)));
        zp4 = *(gcp<f32x4u>)(U + base(ohalf + ((pc + L.sz) >> 1)));
    }
    int c[4] = {C_INSIDE, C_INSIDE, C_INSIDE, C_INSIDE};
    if (!s.all_inside) {
        gcp<uint8_t> cls = (gcp<uint8_t>)L.cls;
#pragma unroll
        for (int k = 0; k < 4; k++) c[k] = cls[pc + 2 * (k < nv ? k : 0)];
    }
    const float xs[5] = {x4.x, x4.y, x4.z, x4.w, x5};
    const float fs[4] = {f4.x, f4.y, f4.z, f4.w};
    const float yms[4] = {ym4.x, ym4.y, ym4.z, ym4.w}, yps[4] = {yp4.x, yp4.y, yp4.z, yp4.w};
    const float zms[4] = {zm4.x, zm4.y, zm4.z, zm4.w}, zps[4] = {zp4.x, zp4.y, zp4.z, zp4.w};
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        float sum = xs[k + 1] + xs[k];
        if (D >= 2) sum += yps[k] + yms[k];
        if (D >= 3) sum += zps[k] + zms[k];
        v[k] = ((float)L.h2 * fs[k] + sum) / (float)(2.0 * D + L.reaction * L.h2);
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        pin(v[k]);
        pin(c[k]);
    }
    if (!live) return;
    gp<float> Uw = (gp<float>)L.u;
    if (nv == 4 && c[0] == C_INSIDE && c[1] == C_INSIDE && c[2] == C_INSIDE && c[3] == C_INSIDE) {
        const f32x4u w4 = {v[0], v[1], v[2], v[3]};
        *(gp<f32x4u>)(Uw + bc) = w4;
        return;
    }
#pragma unroll
    for (int k = 0; k < 4; k++)
        if (k < nv && c[k] == C_INSIDE) Uw[bc + k] = v[k];
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_rb_sweep_split4(const Desc *__restrict__ descs,
                                                            const Item *__restrict__ items, int nseg, int colour,
                                                            const SlotState *__restrict__ st) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int first = __builtin_amdgcn_readfirstlane((xcd_block() * kWavesPerBlock + wave) * 4);
    if (first >= nseg) return;
    const int g = lane >> 4, t = lane & 15;
    Item its[4];
#pragma unroll
    for (int k = 0; k < 4; k++) its[k] = items[min(first + k, nseg - 1)];
    const int nk = min(nseg - first, 4);  // segments of this wavefront
    bool uniform = true;
#pragma unroll
    for (int k = 1; k < 4; k++) uniform = uniform && (k >= nk || its[k].x == its[0].x);
    if (uniform) {
        const Desc L = descs[its[0].x];
        const bool live = st[L.slot].active != 0;
        Item mine = its[0];
#pragma unroll
        for (int k = 1; k < 4; k++)
            if (g == k) mine = its[k];
        if (g < nk) split4_lane<D>(L, mine, t, colour, live);
        return;
    }
    // segments of several problems: one descriptor at a time
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if (k >= nk) break;
        const Desc L = descs[its[k].x];
        const bool live = st[L.slot].active != 0;
        if (g == k) split4_lane<D>(L, its[k], t, colour, live);
    }
}

}  // namespace bcmg
