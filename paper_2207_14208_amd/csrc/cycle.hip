// Kernels of one multigrid cycle (smoothing, ghost relaxation, residual and
// norm, normal extension, restriction, prolongation, coarse solve, iterative
// refinement update).  Each launch walks a work list (see bcmg_internal.h)
// and reads its level descriptor from a table, so the same kernels serve a
// single problem and a batch of problems of different sizes.
//
// Row segments hold up to 128 consecutive nodes of a grid row and are
// processed by one wavefront (two nodes per lane, or for a red-black sweep the
// 64 nodes of one colour, one per lane); ghost and band chunks hold up to 256
// entries, one per thread.  Every gather issues all of its loads before it
// tests classes (neighbour indices are clamped into the array), so a
// wavefront waits for memory once per node instead of once per load.
//
// The small coarse levels of a problem are cycled by one workgroup of 512
// threads per problem (k_coarse_cycle) with workgroup barriers between the
// steps, which replaces a dozen dependent launches per level.
#include "bcmg_internal.h"
#include "launch.h"
#include "rb_sweep.h"
#include "seg.h"

namespace bcmg {

__device__ __forceinline__ double lagrange(int w, int m, double t) {
    if (w == 1) return 1.0;
    if (w == 2) return m == 0 ? 1.0 - t : t;
    if (m == 0) return (1.0 - t) * (2.0 - t) / 2.0;
    if (m == 1) return t * (2.0 - t);
    return t * (t - 1.0) / 2.0;
}

__device__ __forceinline__ double lagrange_dt(int w, int m, double t) {  // d/dt of lagrange
    if (w == 1) return 0.0;
    if (w == 2) return m == 0 ? -1.0 : 1.0;
    if (m == 0) return t - 1.5;
    if (m == 1) return 2.0 - 2.0 * t;
    return t - 0.5;
}

// Left side of ghost row g, sum_m w_m u(G - m o s) (eq. BCh), from the
// ghost's code (widths, signs) and local coordinates tau; PI/PD/PU are
// pointers into global memory or LDS.  Dirichlet rows: the tensor-product
// Lagrange weights prod_k L_{m_k}(tau_k) of widths w_k.  Neumann rows (only
// compiled with NEU, taken where neu): the normal derivative of that
// interpolant, sum_k nd_k L'_{m_k}(tau_k) prod_{j != k} L_{m_j}(tau_j), with
// the ghost's derivative coefficients nd = gnd[3g..3g+2].  The 3^d candidate
// nodes are loaded first (nodes outside the stencil read G itself), then
// accumulated in lexicographic order of m.  Kernels without NEU keep the
// register footprint of the Dirichlet row.  PLANES (Dirichlet rows): load and
// accumulate one plane of m2 at a time (the same terms in the same order, so
// the same result) - three memory round trips instead of one, but a third
// of the registers, for kernels whose other work needs the occupancy.
template <int D, bool NEU, bool PLANES = false, typename PI, typename PD, typename PU>
__device__ __forceinline__ double ghost_row_at(PI gidx, PI gcode, PD gtau, PD gnd, bool neu, long long sy, long long sz,
                                               int g, PU u) {
    const long long p = gidx[g];
    const int code = gcode[g];
    int w[3];
    long long step[3];
    double la[3][3];
    const long long str[3] = {1, sy, sz};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        w[k] = k < D ? code_w(code, k) : 1;
        step[k] = k < D ? (long long)code_s(code, k) * str[k] : 0;
        const double t = k < D ? gtau[3 * g + k] : 0.0;
#pragma unroll
        for (int m = 0; m < 3; m++) la[k][m] = lagrange(w[k], m, t);
    }
    constexpr int M1 = D >= 2 ? 3 : 1, M2 = D >= 3 ? 3 : 1;
    if constexpr (PLANES && !NEU) {
        double acc = 0.0;
#pragma unroll
        for (int m2 = 0; m2 < M2; m2++) {
            double pv[M1][3];
#pragma unroll
            for (int m1 = 0; m1 < M1; m1++)
#pragma unroll
                for (int m0 = 0; m0 < 3; m0++) {
                    const bool in = m0 < w[0] && m1 < w[1] && m2 < w[2];
                    const long long q = in ? p - m0 * step[0] - m1 * step[1] - m2 * step[2] : p;
                    pv[m1][m0] = (double)u[q];
                }
#pragma unroll
            for (int m1 = 0; m1 < M1; m1++)
#pragma unroll
                for (int m0 = 0; m0 < 3; m0++) {
                    if (!(m0 < w[0] && m1 < w[1] && m2 < w[2])) continue;
                    double wgt = 1.0;
                    wgt *= la[0][m0];
                    wgt *= la[1][m1];
                    wgt *= la[2][m2];
                    acc += wgt * pv[m1][m0];
                }
            // the next plane's loads stay below this point
            asm volatile("" ::"v"(acc) : "memory");
        }
        return acc;
    }
    double val[M2][M1][3];
#pragma unroll
    for (int m2 = 0; m2 < M2; m2++)
#pragma unroll
        for (int m1 = 0; m1 < M1; m1++)
#pragma unroll
            for (int m0 = 0; m0 < 3; m0++) {
                const bool in = m0 < w[0] && m1 < w[1] && m2 < w[2];
                const long long q = in ? p - m0 * step[0] - m1 * step[1] - m2 * step[2] : p;
                val[m2][m1][m0] = (double)u[q];
            }
    double acc = 0.0;
    if constexpr (NEU) {
        if (neu) {
            double da[3][3];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double t = k < D ? gtau[3 * g + k] : 0.0;
                const double nd = k < D ? gnd[3 * g + k] : 0.0;
#pragma unroll
                for (int m = 0; m < 3; m++) da[k][m] = nd * lagrange_dt(w[k], m, t);
            }
#pragma unroll
            for (int m2 = 0; m2 < M2; m2++)
#pragma unroll
                for (int m1 = 0; m1 < M1; m1++)
#pragma unroll
                    for (int m0 = 0; m0 < 3; m0++) {
                        if (!(m0 < w[0] && m1 < w[1] && m2 < w[2])) continue;
                        double wgt = 0.0;
                        wgt += da[0][m0] * la[1][m1] * la[2][m2];
                        wgt += da[1][m1] * la[0][m0] * la[2][m2];
                        wgt += da[2][m2] * la[0][m0] * la[1][m1];
                        acc += wgt * val[m2][m1][m0];
                    }
            return acc;
        }
    }
#pragma unroll
    for (int m2 = 0; m2 < M2; m2++)
#pragma unroll
        for (int m1 = 0; m1 < M1; m1++)
#pragma unroll
            for (int m0 = 0; m0 < 3; m0++) {
                if (!(m0 < w[0] && m1 < w[1] && m2 < w[2])) continue;
                double wgt = 1.0;
                wgt *= la[0][m0];
                wgt *= la[1][m1];
                wgt *= la[2][m2];
                acc += wgt * val[m2][m1][m0];
            }
    return acc;
}

template <int D, typename T, bool NEU, bool PLANES = false>
__device__ __forceinline__ double ghost_row(const Desc &L, int g, const NodeArr<const T> &u) {
    return ghost_row_at<D, NEU, PLANES>((gcp<int>)L.gidx, (gcp<int>)L.gcode, (gcp<double>)L.gtau, (gcp<double>)L.gnd,
                                        L.gnd != nullptr, L.sy, L.sz, g, u);
}

// ------------------------------------------------------------ node updates
// Residual of the INSIDE rows of a segment (two nodes per lane); returns the
// lane's sum of r^2.
// store false: only the lane's sum of r^2 is wanted (the FP64 convergence
// check, whose residual the next cycle recomputes before it is read).
template <int D, typename Tu, typename Tr>
__device__ __forceinline__ double seg_residual(const Desc &L, const Item &it, int lane, bool live, bool store = true) {
    const Seg s = seg_of(it);
    double r2 = 0.0;
    const NodeArr<const Tu> u = node_u<const Tu>(L);
    const NodeArr<const Tu> f = node_rhs<const Tu>(L);
    gcp<uint8_t> cls = (gcp<uint8_t>)L.cls;
    const NodeArr<Tr> r = node_r<Tr>(L);
    const long long nn = L.nn;
    // both nodes of the lane are loaded and computed before either store,
    // so that their loads are in flight together
    double rv[2];
    int cc[2];
    long long pp[2];
    int qs[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int q = seg_lane_node(lane, h, L.half_u);
        qs[h] = q;
        const long long p = s.p0 + (q < s.len ? q : 0);
        cc[h] = cls[p];
        pp[h] = p;
        const double up = (double)u[p], fp = (double)f[p];
        const double xm = (double)u[clampi(p - 1, nn)], xp = (double)u[clampi(p + 1, nn)];
        double ym = 0, yp = 0, zm = 0, zp = 0;
        if (D >= 2) {
            ym = (double)u[clampi(p - L.sy, nn)];
            yp = (double)u[clampi(p + L.sy, nn)];
        }
        if (D >= 3) {
            zm = (double)u[clampi(p - L.sz, nn)];
            zp = (double)u[clampi(p + L.sz, nn)];
        }
        double sum = xp + xm;
        if (D >= 2) sum += yp + ym;
        if (D >= 3) sum += zp + zm;
        double lap = (2.0 * D * up - sum) / L.h2;
        if (L.reaction != 0.0) lap += L.reaction * up;  // c u - Laplace u
        rv[h] = fp - lap;
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        pin(rv[h]);
        pin(cc[h]);
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        if (qs[h] < s.len && cc[h] == C_INSIDE && live) {
            if (store) r[pp[h]] = (Tr)rv[h];
            r2 += rv[h] * rv[h];
        }
    }
    return r2;
}

// Two adjacent FP64 values by one 16-byte load or store (8-byte aligned).
using f64x2u = double __attribute__((ext_vector_type(2), aligned(8)));

// Every pair load of seg_residual_pair over segment s (one node before the
// segment to one after it, in its row and the y and z neighbour rows) stays
// in the level's arrays.
template <int D>
__device__ __forceinline__ bool pair_loads_fit(const Desc &L, const Seg &s) {
    const long long reach = 1 + (D >= 3 ? L.sz : (D >= 2 ? L.sy : 0));
    return s.p0 - reach >= 0 && s.p0 + s.len + reach < L.nn;
}

// Residual of the INSIDE rows of a segment of an FP64 natural-order field:
// lane t takes the adjacent nodes q0 = 2t and q0 + 1 and reads them with
// 16-byte loads (u at x - 1 .. x + 2, the four y and z neighbour pairs, f);
// the arithmetic is seg_residual's, node by node (the same r).  The caller
// has checked pair_loads_fit.
template <int D, typename Tr>
__device__ __forceinline__ double seg_residual_pair(const Desc &L, const Seg &s, int lane, bool live, bool store) {
    const int q0 = 2 * lane;
    const int nv = min(max(s.len - q0, 0), 2);
    const long long p = s.p0 + (nv > 0 ? q0 : 0);
    gcp<double> U = (gcp<double>)L.u;
    gcp<double> F = (gcp<double>)L.rhs;
    const f64x2u xl = *(gcp<f64x2u>)(U + p - 1);  // x - 1, x
    const f64x2u xr = *(gcp<f64x2u>)(U + p + 1);  // x + 1, x + 2
    const f64x2u f2 = *(gcp<f64x2u>)(F + p);
    f64x2u ym = {0.0, 0.0}, yp = {0.0, 0.0}, zm = {0.0, 0.0}, zp = {0.0, 0.0};
    if (D >= 2) {
        ym = *(gcp<f64x2u>)(U + p - L.sy);
        yp = *(gcp<f64x2u>)(U + p + L.sy);
    }
    if (D >= 3) {
        zm = *(gcp<f64x2u>)(U + p - L.sz);
        zp = *(gcp<f64x2u>)(U + p + L.sz);
    }
    int cc[2] = {C_INSIDE, C_INSIDE};
    if (!s.all_inside) {
        gcp<uint8_t> cls = (gcp<uint8_t>)L.cls;
        cc[0] = cls[p];
        cc[1] = cls[p + (nv > 1 ? 1 : 0)];
    }
    const double X[4] = {xl.x, xl.y, xr.x, xr.y};
    const double FP[2] = {f2.x, f2.y}, YM[2] = {ym.x, ym.y}, YP[2] = {yp.x, yp.y};
    const double ZM[2] = {zm.x, zm.y}, ZP[2] = {zp.x, zp.y};
    double rv[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const double up = X[h + 1];
        double sum = X[h + 2] + X[h];
        if (D >= 2) sum += YP[h] + YM[h];
        if (D >= 3) sum += ZP[h] + ZM[h];
        double lap = (2.0 * D * up - sum) / L.h2;
        if (L.reaction != 0.0) lap += L.reaction * up;  // c u - Laplace u
        rv[h] = FP[h] - lap;
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        pin(rv[h]);
        pin(cc[h]);
    }
    double r2 = 0.0;
    if (!live) return r2;
    const NodeArr<Tr> r = node_r<Tr>(L);
    if (store && sizeof(Tr) == 8 && !r.half && nv == 2 && cc[0] == C_INSIDE && cc[1] == C_INSIDE) {
        *(gp<f64x2u>)((gp<double>)L.r + p) = f64x2u{rv[0], rv[1]};
        return rv[0] * rv[0] + rv[1] * rv[1];
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        if (h < nv && cc[h] == C_INSIDE) {
            if (store) r[p + h] = (Tr)rv[h];
            r2 += rv[h] * rv[h];
        }
    }
    return r2;
}

// Restriction (fine level F, coarse level C; eq. coarseFW, Sec. 3.2 FW,
// Sec. 3.3).  Coarse INSIDE node: FW over the 3^d fine box around X = 2J if
// all of it is INSIDE, else the FW weights of its INSIDE nodes renormalised
// (or their plain mean).  Also zeroes the coarse unknown (initial guess of
// the coarse correction).  Coarse GHOST nodes are done by restrict_ghost.
// FW of the fine residual r over the 3^d box around fine node X for a
// coarse INSIDE row: all of the box INSIDE and in the grid, else the FW
// weights of its INSIDE nodes renormalised (or their plain mean).
// PLANES: load and accumulate one plane of m2 at a time (the same terms in
// the same order), a third of the registers for three memory round trips.
// PAIRS (r an FP64 natural-order NodeArr): each fine row's three residuals
// come from one 16-byte and one 8-byte load; the caller has checked that
// x - 1 and x + 1 of every row stay in the array.
template <int D, bool PLANES = false, bool PAIRS = false, typename PR, typename PC>
__device__ __forceinline__ double restrict_inside_at(PR r, PC fcls, int FN, long long fsy, long long fsz, int X0,
                                                     int X1, int X2, int mode) {
    constexpr int R1 = D >= 2 ? 1 : 0, R2 = D >= 3 ? 1 : 0;
    constexpr int NP = PLANES ? 2 * R2 + 1 : 1;  // planes loaded together
    constexpr int NL = PLANES ? 1 : 2 * R2 + 1;  // planes per load group
    const long long pf = X0 + X1 * fsy + X2 * fsz;
    double full = 0.0, sel = 0.0, selw = 0.0, msum = 0.0, mcnt = 0.0;
    bool all_ok = true;
#pragma unroll
    for (int g = 0; g < NP; g++) {
        uint8_t fc[NL][2 * R1 + 1][3];
        double rv[NL][2 * R1 + 1][3];
        bool inb[NL][2 * R1 + 1][3];
        if constexpr (PAIRS) {
#pragma unroll
            for (int i2 = 0; i2 < NL; i2++)
#pragma unroll
                for (int m1 = -R1; m1 <= R1; m1++) {
                    const int m2 = g + i2 - R2;
                    const int J1 = X1 + m1, J2 = X2 + m2;
                    const bool rin = (D < 2 || (J1 >= 0 && J1 <= FN)) && (D < 3 || (J2 >= 0 && J2 <= FN));
                    const long long qc = rin ? pf + m1 * fsy + m2 * fsz : pf;
                    const f64x2u lo = *(gcp<f64x2u>)(r.a + qc - 1);  // x - 1, x
                    const double hi = r.a[qc + 1];
                    const double v3[3] = {lo.x, lo.y, hi};
#pragma unroll
                    for (int m0 = -1; m0 <= 1; m0++) {
                        const int J0 = X0 + m0;
                        const bool in = rin && J0 >= 0 && J0 <= FN;
                        inb[i2][m1 + R1][m0 + 1] = in;
                        fc[i2][m1 + R1][m0 + 1] = fcls[in ? qc + m0 : pf];
                        rv[i2][m1 + R1][m0 + 1] = v3[m0 + 1];  // read only where in
                    }
                }
        } else {
#pragma unroll
            for (int i2 = 0; i2 < NL; i2++)
#pragma unroll
                for (int m1 = -R1; m1 <= R1; m1++)
#pragma unroll
                    for (int m0 = -1; m0 <= 1; m0++) {
                        const int m2 = g + i2 - R2;
                        const int J0 = X0 + m0, J1 = X1 + m1, J2 = X2 + m2;
                        const bool in = J0 >= 0 && J0 <= FN && (D < 2 || (J1 >= 0 && J1 <= FN)) &&
                                        (D < 3 || (J2 >= 0 && J2 <= FN));
                        const long long q = in ? pf + m0 + m1 * fsy + m2 * fsz : pf;
                        inb[i2][m1 + R1][m0 + 1] = in;
                        fc[i2][m1 + R1][m0 + 1] = fcls[q];
                        rv[i2][m1 + R1][m0 + 1] = (double)r[q];
                    }
        }
#pragma unroll
        for (int i2 = 0; i2 < NL; i2++)
#pragma unroll
            for (int m1 = -R1; m1 <= R1; m1++)
#pragma unroll
                for (int m0 = -1; m0 <= 1; m0++) {
                    const int m2 = g + i2 - R2;
                    double wgt = 1.0;
                    wgt *= (m0 == 0 ? 0.5 : 0.25);
                    if (D >= 2) wgt *= (m1 == 0 ? 0.5 : 0.25);
                    if (D >= 3) wgt *= (m2 == 0 ? 0.5 : 0.25);
                    if (!inb[i2][m1 + R1][m0 + 1]) {
                        all_ok = false;
                        continue;
                    }
                    const bool take = fc[i2][m1 + R1][m0 + 1] == C_INSIDE;
                    if (!take) all_ok = false;
                    const double v = rv[i2][m1 + R1][m0 + 1];
                    full += wgt * v;
                    if (take) {
                        sel += wgt * v;
                        selw += wgt;
                        msum += v;
                        mcnt += 1.0;
                    }
                }
        // the next plane's loads stay below this point
        if (PLANES) asm volatile("" ::"v"(full), "v"(sel), "v"(selw), "v"(msum) : "memory");
    }
    if (all_ok) return full;
    if (mode == BCMG_RESTRICT_PLAIN_MEAN) return mcnt > 0.0 ? msum / mcnt : 0.0;
    return selw > 0.0 ? sel / selw : 0.0;
}

// Restriction (fine level F, coarse level C; eq. coarseFW, Sec. 3.2 FW,
// Sec. 3.3) to coarse node pc: its right-hand side fv, its class cc, and the
// initial guess uv of the coarse correction, zero (seg_restrict stores them
// at INSIDE nodes).  Coarse GHOST nodes are done by restrict_ghost.
// With red, the node also takes the first red half-sweep of the coarse
// pre-smoothing: from the zero initial guess every neighbour of an INSIDE
// node is zero, so the update of a red node (i+j+k even) is h^2 f / (2d),
// computed as the sweep computes it (a zero neighbour sum added).
// pairs: FP64 fields, whose rows the segment's pair loads keep inside the
// fine array (restrict_pairs_fit).
template <int D, typename T>
__device__ __forceinline__ void restrict_node(const Desc &C, const Desc &F, long long pc, int X0, int X1, int X2,
                                              bool red, T &fv, T &uv, int &cc, bool pairs = false) {
    double out;
    if (sizeof(T) == 8 && pairs)
        out = restrict_inside_at<D, true, sizeof(T) == 8>(node_r<const T>(F), (gcp<uint8_t>)F.cls, F.N, F.sy, F.sz,
                                                          X0, X1, X2, C.restrict_mode);
    else
        out = restrict_inside_at<D, true>(node_r<const T>(F), (gcp<uint8_t>)F.cls, F.N, F.sy, F.sz, X0, X1, X2,
                                          C.restrict_mode);
    cc = ((gcp<uint8_t>)C.cls)[pc];
    fv = (T)out;
    uv = (T)0;
    if (red && (((X0 + X1 + X2) >> 1) & 1) == 0) {
        const T sum = (T)0;
        uv = ((T)C.h2 * fv + sum) / (T)(2.0 * D + C.reaction * C.h2);
    }
}

// Sparse row sums.  The sum over j in [beg, end) of coef[j] * value(idx[j])
// is defined as eight strided partial sums, partial k over j = beg + k,
// beg + k + 8, ... in increasing j, added as ((p0 + p1) + (p2 + p3)) +
// ((p4 + p5) + (p6 + p7)).  row_dot computes it in one thread, row_dot_group
// with eight lanes (one partial each, a shuffle tree), so that every path
// gives the same bits.
constexpr int kRowLanes = 8;

__device__ __forceinline__ double row_tree(const double (&a)[kRowLanes]) {
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

template <typename F>
__device__ __forceinline__ double row_dot(gcp<int> idx, gcp<double> coef, int beg, int end, F value) {
    double a[kRowLanes] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int j = beg; j < end; j += kRowLanes) {  // eight entries' loads in flight per step
        int ix[kRowLanes];
        double cf[kRowLanes], x[kRowLanes];
#pragma unroll
        for (int k = 0; k < kRowLanes; k++) {
            const int jj = min(j + k, end - 1);
            ix[k] = idx[jj];
            cf[k] = coef[jj];
        }
#pragma unroll
        for (int k = 0; k < kRowLanes; k++) x[k] = value(ix[k]);
#pragma unroll
        for (int k = 0; k < kRowLanes; k++)
            if (j + k < end) a[k] += cf[k] * x[k];
    }
    return row_tree(a);
}

// The same sum by the eight lanes sub = 0..7 of an aligned lane group (all
// eight call it together; each gets the sum).  A lane keeps four of its
// entries' loads in flight per step.
template <typename F>
__device__ __forceinline__ double row_dot_group(gcp<int> idx, gcp<double> coef, int beg, int end, int sub, F value) {
    constexpr int M = 4;
    double a = 0.0;
    for (int j = beg + sub; j < end; j += M * kRowLanes) {
        int ix[M];
        double cf[M], x[M];
#pragma unroll
        for (int m = 0; m < M; m++) {
            const int jj = max(min(j + m * kRowLanes, end - 1), beg);
            ix[m] = idx[jj];
            cf[m] = coef[jj];
        }
#pragma unroll
        for (int m = 0; m < M; m++) x[m] = value(ix[m]);
#pragma unroll
        for (int m = 0; m < M; m++)
            if (j + m * kRowLanes < end) a += cf[m] * x[m];
    }
    a += __shfl_xor(a, 1);
    a += __shfl_xor(a, 2);
    a += __shfl_xor(a, 4);
    return a;
}

// Restriction to coarse ghost g: its precomputed row over the fine ghost
// residuals (FW or renormalised FW of the extended fine residual, with the
// extension folded in); zeroes the coarse unknown.
template <typename T>
__device__ __forceinline__ void restrict_ghost(const Desc &C, const Desc &F, int g, bool live) {
    const NodeArr<const T> r = node_r<const T>(F);
    gcp<int> rptr = (gcp<int>)C.rptr, ridx = (gcp<int>)C.ridx;
    gcp<double> rcoef = (gcp<double>)C.rcoef;
    const int beg = rptr[g], end = rptr[g + 1];
    const long long pc = ((gcp<int>)C.gidx)[g];
    const double acc = row_dot(ridx, rcoef, beg, end, [&](int q) { return (double)r[q]; });
    if (!live) return;
    node_rhs<T>(C)[pc] = (T)acc;
    node_u<T>(C)[pc] = (T)0;
}

// The restriction of coarse node q of a segment (one node per lane: its 3^d
// box of fine residuals and classes is 54 loads, all in flight at once).
// The fine rows of a coarse segment's restriction boxes stay inside the
// fine array with one node to spare at either end (their pair loads).
template <int D>
__device__ __forceinline__ bool restrict_pairs_fit(const Desc &F, const Seg &s) {
    const long long rows = (D >= 2 ? F.sy : 0) + (D >= 3 ? F.sz : 0);
    const long long pf0 = 2LL * s.x0 + 2LL * s.yj * F.sy + 2LL * s.zk * F.sz;
    return pf0 - 1 - rows >= 0 && pf0 + 2LL * (s.len - 1) + 1 + rows < F.nn;
}

template <int D, typename T>
__device__ __forceinline__ void seg_restrict_one(const Desc &C, const Desc &F, const Item &it, int q, bool live,
                                                 bool red) {
    const Seg s = seg_of(it);
    const int qq = q < s.len ? q : 0;
    T fv, uv;
    int cc;
    const bool pairs = sizeof(T) == 8 && restrict_pairs_fit<D>(F, s);
    restrict_node<D, T>(C, F, s.p0 + qq, 2 * (s.x0 + qq), 2 * s.yj, 2 * s.zk, red, fv, uv, cc, pairs);
    pin(fv);
    pin(uv);
    pin(cc);
    if (!live || q >= s.len || cc != C_INSIDE) return;
    node_u<T>(C)[s.p0 + q] = uv;
    node_rhs<T>(C)[s.p0 + q] = fv;
}

// restrict_ghost by the eight lanes sub of a group (one coarse ghost each group)
template <typename T>
__device__ __forceinline__ void restrict_ghost_group(const Desc &C, const Desc &F, int g, int sub, bool live) {
    const NodeArr<const T> r = node_r<const T>(F);
    const int beg = ((gcp<int>)C.rptr)[g], end = ((gcp<int>)C.rptr)[g + 1];
    const long long pc = ((gcp<int>)C.gidx)[g];
    const double acc =
        row_dot_group((gcp<int>)C.ridx, (gcp<double>)C.rcoef, beg, end, sub, [&](int q) { return (double)r[q]; });
    if (!live || sub != 0) return;
    node_rhs<T>(C)[pc] = (T)acc;
    node_u<T>(C)[pc] = (T)0;
}

template <int D, typename T>
__device__ __forceinline__ void seg_restrict(const Desc &C, const Desc &F, const Item &it, int lane, bool live,
                                             bool red) {
    const Seg s = seg_of(it);
    T fv[2], uv[2];
    int cc[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {  // both nodes computed before either store
        const int q = lane + 64 * h;
        const int qq = q < s.len ? q : 0;
        restrict_node<D, T>(C, F, s.p0 + qq, 2 * (s.x0 + qq), 2 * s.yj, 2 * s.zk, red, fv[h], uv[h], cc[h]);
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        pin(fv[h]);
        pin(uv[h]);
        pin(cc[h]);
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int q = lane + 64 * h;
        if (!live || q >= s.len || cc[h] != C_INSIDE) continue;
        const long long pc = s.p0 + q;
        node_u<T>(C)[pc] = uv[h];
        node_rhs<T>(C)[pc] = fv[h];
    }
}

// Prolongation and correction: multilinear interpolation of the (extended)
// coarse error to INSIDE and GHOST nodes, u += e (Sec. 2.1 interpolation,
// Sec. 3.2 bilinear interpolation, Sec. 3.3).
// Multilinear interpolation at fine node I of the coarse error ec (its
// coarse cell corners; Sec. 2.1 interpolation, Sec. 3.2).
template <int D, typename PE>
__device__ __forceinline__ double prolong_at(PE ec, long long csy, long long csz, int I0, int I1, int I2) {
    const int h0 = I0 & 1, h1 = D >= 2 ? (I1 & 1) : 0, h2 = D >= 3 ? (I2 & 1) : 0;
    const int B0 = (I0 - h0) / 2, B1 = (I1 - h1) / 2, B2 = (I2 - h2) / 2;
    constexpr int M1 = D >= 2 ? 2 : 1, M2 = D >= 3 ? 2 : 1;
    double ev[M2][M1][2];
    const long long b = B0 + B1 * csy + B2 * csz;
#pragma unroll
    for (int m2 = 0; m2 < M2; m2++)
#pragma unroll
        for (int m1 = 0; m1 < M1; m1++)
#pragma unroll
            for (int m0 = 0; m0 < 2; m0++) {
                const bool in = m0 <= h0 && m1 <= h1 && m2 <= h2;
                ev[m2][m1][m0] = (double)ec[in ? b + m0 + m1 * csy + m2 * csz : b];
            }
    double e = 0.0;
#pragma unroll
    for (int m2 = 0; m2 < M2; m2++)
#pragma unroll
        for (int m1 = 0; m1 < M1; m1++)
#pragma unroll
            for (int m0 = 0; m0 < 2; m0++) {
                if (!(m0 <= h0 && m1 <= h1 && m2 <= h2)) continue;
                double wgt = 1.0;
                if (h0) wgt *= 0.5;
                if (h1) wgt *= 0.5;
                if (h2) wgt *= 0.5;
                e += wgt * ev[m2][m1][m0];
            }
    return e;
}

// Prolongation and correction at fine node p: v = u + P e and the class fc
// (seg_prolong stores v at INSIDE and GHOST nodes; Sec. 3.3: the coarse
// error was extended into its band first).
template <int D, typename T>
__device__ __forceinline__ void prolong_node(const Desc &F, const Desc &C, long long p, int I0, int I1, int I2, T &v,
                                             int &fc) {
    const double e = prolong_at<D>(node_u<const T>(C), C.sy, C.sz, I0, I1, I2);
    fc = ((gcp<uint8_t>)F.cls)[p];
    v = (T)((double)node_u<const T>(F)[p] + e);
}

// Prolongation at two x-adjacent fine nodes I0 and I0 + 1 of one row: both
// read coarse x-positions B and B + 1 only (B = floor(I0 / 2)), so the coarse
// values are loaded once for the pair; each node then sums its corners as
// prolong_at does (the same terms in the same order).  bvalid: node I0 + 1 is
// wanted (else x = B + 1 is read only if node I0 needs it: with I0 even on
// the box face, B + 1 lies beyond the row).  PAIRS (an FP64 natural-order
// coarse array ec, gcp<double>): each coarse row's two values come from one
// 16-byte load; the caller has checked that x = B + 1 stays in the array.
template <int D, bool PAIRS = false, typename PE>
__device__ __forceinline__ void prolong_pair(PE ec, long long csy, long long csz, int I0, int I1, int I2,
                                             bool bvalid, double &ea, double &eb) {
    const int h0 = I0 & 1, h1 = D >= 2 ? (I1 & 1) : 0, h2 = D >= 3 ? (I2 & 1) : 0;
    const int B0 = (I0 - h0) / 2, B1 = (I1 - h1) / 2, B2 = (I2 - h2) / 2;
    constexpr int M1 = D >= 2 ? 2 : 1, M2 = D >= 3 ? 2 : 1;
    double ev[M2][M1][2];  // coarse values at x = B0, B0 + 1
    const long long b = B0 + B1 * csy + B2 * csz;
    if constexpr (PAIRS) {
#pragma unroll
        for (int m2 = 0; m2 < M2; m2++)
#pragma unroll
            for (int m1 = 0; m1 < M1; m1++) {
                const bool in = m1 <= h1 && m2 <= h2;
                const f64x2u pr = *(gcp<f64x2u>)(ec + (in ? b + m1 * csy + m2 * csz : b));
                ev[m2][m1][0] = pr.x;
                ev[m2][m1][1] = pr.y;
            }
    } else {
#pragma unroll
        for (int m2 = 0; m2 < M2; m2++)
#pragma unroll
            for (int m1 = 0; m1 < M1; m1++)
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    const bool in = m1 <= h1 && m2 <= h2 && (c == 0 || h0 == 1 || bvalid);
                    ev[m2][m1][c] = (double)ec[in ? b + c + m1 * csy + m2 * csz : b];
                }
    }
    // node a = I0 (corners x = B0 .. B0 + h0); node b = I0 + 1: with I0 even
    // it is odd over B0, B0 + 1, with I0 odd it is even at B0 + 1 alone
    double a = 0.0, e2 = 0.0;
#pragma unroll
    for (int m2 = 0; m2 < M2; m2++)
#pragma unroll
        for (int m1 = 0; m1 < M1; m1++) {
            if (!(m1 <= h1 && m2 <= h2)) continue;
#pragma unroll
            for (int m0 = 0; m0 < 2; m0++) {
                if (m0 <= h0) {  // node a, corner x = B0 + m0
                    double wgt = 1.0;
                    if (h0) wgt *= 0.5;
                    if (h1) wgt *= 0.5;
                    if (h2) wgt *= 0.5;
                    a += wgt * ev[m2][m1][m0];
                }
                if (m0 <= 1 - h0) {  // node b, corner x = (B0 + h0) + m0
                    double wgt = 1.0;
                    if (!h0) wgt *= 0.5;
                    if (h1) wgt *= 0.5;
                    if (h2) wgt *= 0.5;
                    e2 += wgt * ev[m2][m1][h0 + m0];
                }
            }
        }
    ea = a;
    eb = e2;
}

// FP64 fields (natural order): the pair's fine values, and each coarse
// row's two values, by 16-byte loads, where every such load of the segment
// stays in its array.
template <int D>
__device__ __forceinline__ void seg_prolong_pairs(const Desc &F, const Desc &C, const Seg &s, int lane, bool live) {
    const int q0 = 2 * lane;
    const int qa = q0 < s.len ? q0 : 0;
    double e[2];
    prolong_pair<D, true>((gcp<double>)C.u, C.sy, C.sz, s.x0 + qa, s.yj, s.zk, q0 + 1 < s.len, e[0], e[1]);
    const long long p = s.p0 + qa;
    gp<double> U = (gp<double>)F.u;
    const f64x2u u2 = *(gcp<f64x2u>)(U + p);
    int fc[2] = {C_INSIDE, C_INSIDE};
    if (!s.all_inside) {
        fc[0] = ((gcp<uint8_t>)F.cls)[p];
        fc[1] = ((gcp<uint8_t>)F.cls)[p + (q0 + 1 < s.len ? 1 : 0)];
    }
    double v[2] = {u2.x + e[0], u2.y + e[1]};
#pragma unroll
    for (int h = 0; h < 2; h++) {
        pin(v[h]);
        pin(fc[h]);
    }
    if (!live || q0 >= s.len) return;
    const bool w0 = fc[0] == C_INSIDE || fc[0] == C_GHOST;
    const bool w1 = q0 + 1 < s.len && (fc[1] == C_INSIDE || fc[1] == C_GHOST);
    if (w0 && w1) {
        *(gp<f64x2u>)(U + p) = f64x2u{v[0], v[1]};
    } else {
        if (w0) U[p] = v[0];
        if (w1) U[p + 1] = v[1];
    }
}

template <int D, typename T>
__device__ __forceinline__ void seg_prolong(const Desc &F, const Desc &C, const Item &it, int lane, bool live) {
    const Seg s = seg_of(it);
    if constexpr (sizeof(T) == 8) {
        // the last coarse value a pair load may touch, and the fine pair
        // after the segment's last node
        const long long cmax = ((s.x0 + s.len) >> 1) + 1 + ((s.yj + 1) >> 1) * C.sy + ((s.zk + 1) >> 1) * C.sz;
        if (cmax < C.nn && s.p0 + s.len < F.nn) {
            seg_prolong_pairs<D>(F, C, s, lane, live);
            return;
        }
    }
    // lane takes the adjacent nodes q0 = 2 lane and q0 + 1 (for a split
    // array, one of each parity: both loads stay contiguous per half)
    const int q0 = 2 * lane;
    const int qa = q0 < s.len ? q0 : 0;
    double e[2];
    prolong_pair<D>(node_u<const T>(C), C.sy, C.sz, s.x0 + qa, s.yj, s.zk, q0 + 1 < s.len, e[0], e[1]);
    T v[2];
    int fc[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {  // both nodes computed before either store
        const int q = q0 + h;
        const long long p = s.p0 + (q < s.len ? q : qa);
        fc[h] = ((gcp<uint8_t>)F.cls)[p];
        v[h] = (T)((double)node_u<const T>(F)[p] + e[h]);
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        pin(v[h]);
        pin(fc[h]);
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int q = q0 + h;
        if (!live || q >= s.len || (fc[h] != C_INSIDE && fc[h] != C_GHOST)) continue;
        node_u<T>(F)[s.p0 + q] = v[h];
    }
}

// Ghost relaxation (eq. rel with P_GG = I/dtau: new interior values, old ghost
// values): increment, then u_G += increment in a second pass.
template <int D, typename T, bool NEU>
__device__ __forceinline__ void ghost_delta(const Desc &L, int g, bool live) {
    const NodeArr<const T> u = node_u<const T>(L);
    const NodeArr<const T> rhs = node_rhs<const T>(L);
    const long long p = ((gcp<int>)L.gidx)[g];
    const double rg = (double)rhs[p];
    const double up = (double)u[p];
    const double row = ghost_row<D, T, NEU>(L, g, u);
    const double v = (double)(T)(up + ((gcp<double>)L.gdtau)[g] * (rg - row));
    pin(v);
    if (!live) return;
    ((gp<double>)L.gnew)[g] = v;
}

template <typename T>
__device__ __forceinline__ void ghost_apply(const Desc &L, int g, bool live) {
    const long long p = ((gcp<int>)L.gidx)[g];
    const T v = (T)((gcp<double>)L.gnew)[g];
    pin(v);
    if (!live) return;
    node_u<T>(L)[p] = v;
}

template <int D, typename Tu, typename Tr, bool NEU>
__device__ __forceinline__ double ghost_residual(const Desc &L, int g, bool live, bool store = true) {
    const long long pg = ((gcp<int>)L.gidx)[g];
    const double rg = (double)node_rhs<const Tu>(L)[pg];
    const double r = rg - ghost_row<D, Tu, NEU, true>(L, g, node_u<const Tu>(L));
    pin(r);
    if (!live) return 0.0;
    if (store) node_r<Tr>(L)[pg] = (Tr)r;
    return r * r;
}

// Normal extension at band node b (Sec. 3.3 transfer operators): the K
// upwind Jacobi sweeps from zero, folded at setup into a row over the ghost
// values; gsrc gives the ghost values in list order (the new values of a
// ghost step), or null to read them from the field.
template <typename T>
__device__ __forceinline__ void ext_gather(const Desc &L, int b, const double *gsrc, bool live) {
    const NodeArr<T> field = node_u<T>(L);
    gcp<int> gidx = (gcp<int>)L.gidx;
    gcp<double> src = (gcp<double>)gsrc;
    const int beg = ((gcp<int>)L.eptr)[b], end = ((gcp<int>)L.eptr)[b + 1];
    const long long p = ((gcp<int>)L.bidx)[b];
    const double v =
        src ? row_dot((gcp<int>)L.eidx, (gcp<double>)L.ecoef, beg, end, [&](int g) { return src[g]; })
            : row_dot((gcp<int>)L.eidx, (gcp<double>)L.ecoef, beg, end, [&](int g) { return (double)field[gidx[g]]; });
    if (!live) return;
    field[p] = (T)v;
}

// ext_gather by the eight lanes sub of a group (one band entry each group)
template <typename T>
__device__ __forceinline__ void ext_gather_group(const Desc &L, int b, const double *gsrc, int sub, bool live) {
    const NodeArr<T> field = node_u<T>(L);
    gcp<int> gidx = (gcp<int>)L.gidx;
    gcp<double> src = (gcp<double>)gsrc;
    const int beg = ((gcp<int>)L.eptr)[b], end = ((gcp<int>)L.eptr)[b + 1];
    const long long p = ((gcp<int>)L.bidx)[b];
    gcp<int> eidx = (gcp<int>)L.eidx;
    gcp<double> ecoef = (gcp<double>)L.ecoef;
    const double v = src ? row_dot_group(eidx, ecoef, beg, end, sub, [&](int g) { return src[g]; })
                         : row_dot_group(eidx, ecoef, beg, end, sub, [&](int g) { return (double)field[gidx[g]]; });
    if (!live || sub != 0) return;
    field[p] = (T)v;
}

// Row blocks: a chunk item of up to kChunk rows is served by kRowLanes
// workgroups of kBlock / kRowLanes row groups of kRowLanes lanes.
constexpr int kRowsPerBlock = kBlock / kRowLanes;
static_assert(kRowsPerBlock * kRowLanes == kChunk, "a chunk spans kRowLanes row blocks");

// Coarsest level: x = A^{-1} b over INSIDE then GHOST unknowns, in FP64, by
// the threads of one workgroup (b staged in LDS).
template <typename T>
__device__ void coarse_solve_block(const Desc &L, double *b) {
    const int nc = L.nc;
    const T *rhs = (const T *)L.rhs;
    for (int t = threadIdx.x; t < nc; t += blockDim.x) b[t] = (double)rhs[L.cmap[t]];
    __syncthreads();
    for (int t = threadIdx.x; t < nc; t += blockDim.x) {
        double x = 0.0;
        const double *row = L.ainv + (long long)t * nc;
        for (int j = 0; j < nc; j++) x += row[j] * b[j];
        ((T *)L.u)[L.cmap[t]] = (T)x;
    }
    __syncthreads();
}

// ----------------------------------------------------------------- kernels
// The two-list mapping of xcd_block with each XCD's blocks of the second
// list dispatched before its blocks of the first: the second list holds the
// blocks with the longer dependent-load chains (ghost rows, sparse rows),
// which should not start last.
__device__ __forceinline__ int xcd_block_second_first(int nfirst) {
    const int b = blockIdx.x, nb = gridDim.x;
    const int x = b % kXcds, i = b / kXcds;
    const int qa = nfirst / kXcds, ra = nfirst % kXcds;
    const int qt = nb / kXcds, rt = nb % kXcds;
    const int na = qa + (x < ra ? 1 : 0);
    const int abeg = x * qa + min(x, ra);
    const int tbeg = x * qt + min(x, rt);
    const int nsec = qt + (x < rt ? 1 : 0) - na;
    if (i < nsec) return nfirst + (tbeg - abeg) + i;
    return abeg + (i - nsec);
}

#define CHUNK_ITEM CHUNK_ITEM_AT(xcd_block())
#define CHUNK_ITEM_AT(lblock)                                     \
    const Item it = items[lblock];                                \
    const Desc &L = descs[it.x];                                  \
    const bool live = st[L.slot].active != 0;                     \
    if ((int)threadIdx.x >= it.z) return;                         \
    const int e = it.y + threadIdx.x;

// Ghost step, first half: one wavefront-sized workgroup per quarter chunk, so
// that the finest level's chunks spread their dependent gathers over every CU
// (a whole chunk per workgroup leaves the 257^3 flower's 52,873 ghosts on 207
// workgroups).  Each thread computes the same entry as with whole chunks.
constexpr int kGhostSplit = 4;
constexpr int kGhostBlock = kChunk / kGhostSplit;
static_assert(kGhostBlock * kGhostSplit == kChunk, "a chunk splits into whole workgroups");

template <int D, typename T, bool NEU>
__global__ __launch_bounds__(kGhostBlock) void k_ghost_delta(const Desc *__restrict__ descs,
                                                             const Item *__restrict__ items,
                                                             const SlotState *__restrict__ st) {
    const int lb = xcd_block();
    const Item it = items[lb / kGhostSplit];
    const Desc &L = descs[it.x];
    const bool live = st[L.slot].active != 0;
    const int t = (lb % kGhostSplit) * kGhostBlock + (int)threadIdx.x;
    if (t >= it.z) return;
    ghost_delta<D, T, NEU>(L, it.y + t, live);
}

// Ghost step, second half: the new ghost values into u (chunk blocks), and,
// in the same launch, the extension of the new field into the band chunks
// bch (their ghost values come from gnew, which this launch does not write).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ghost_apply(const Desc *__restrict__ descs,
                                                        const Item *__restrict__ items, int ngch,
                                                        const Item *__restrict__ bch,
                                                        const SlotState *__restrict__ st) {
    const int lb = xcd_block_second_first(ngch);
    if (lb < ngch) {
        CHUNK_ITEM_AT(lb)
        ghost_apply<T>(L, e, live);
        return;
    }
    const int rb = lb - ngch;
    const Item it = bch[rb / kRowLanes];
    const Desc &L = descs[it.x];
    const bool live = st[L.slot].active != 0;
    const int row = (rb % kRowLanes) * kRowsPerBlock + (int)threadIdx.x / kRowLanes;
    if (row >= it.z) return;  // whole lane groups leave together
    ext_gather_group<T>(L, ((gcp<int>)L.bneed)[it.y + row], L.gnew, threadIdx.x % kRowLanes, live);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Residual on INSIDE rows (segment blocks) and GHOST rows (chunk blocks);
// with NORM, one partial sum of r^2 per segment, then one per ghost chunk,
// each reduced in a fixed order.
template <int D, typename Tu, typename Tr, bool NORM, bool NEU>
__global__ __launch_bounds__(kBlock) void k_residual(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                     int nseg, const Item *__restrict__ gch, int nseg_blocks,
                                                     const SlotState *__restrict__ st, double *__restrict__ partials,
                                                     int store) {
    const int lb = xcd_block_second_first(nseg_blocks);
    if (lb < nseg_blocks) {
        SEG_ITEM_AT(lb)
        double r2;
        if constexpr (sizeof(Tu) == 8 && D >= 2) {  // FP64 fields are in the natural order
            const Seg s = seg_of(it);
            if (pair_loads_fit<D>(L, s))
                r2 = seg_residual_pair<D, Tr>(L, s, lane, live, store != 0);
            else
                r2 = seg_residual<D, Tu, Tr>(L, it, lane, live, store != 0);
        } else {
            r2 = seg_residual<D, Tu, Tr>(L, it, lane, live, store != 0);
        }
        if (NORM) {
            r2 = wave_sum(r2);
            if (lane == 0) partials[sidx] = r2;
        }
        return;
    }
    const int cb = lb - nseg_blocks;
    const Item it = gch[cb];
    const Desc &L = descs[it.x];
    const bool live = st[L.slot].active != 0;
    double r2 = 0.0;
    if ((int)threadIdx.x < it.z) r2 = ghost_residual<D, Tu, Tr, NEU>(L, it.y + threadIdx.x, live, store != 0);
    if (NORM) {
        __shared__ double ws[kWavesPerBlock];
        r2 = wave_sum(r2);
        if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = r2;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kWavesPerBlock; w++) s += ws[w];
            partials[nseg + cb] = s;
        }
    }
}

// Residual of the INSIDE rows of a level stored split by node parity (FP32),
// four row segments per wavefront, sixteen lanes per segment and eight
// consecutive nodes per lane: four of each parity, a and b, whose values,
// x neighbours and f are consecutive in their halves (a: entries ia ..
// ia + 3, b: ib .. ib + 3), x neighbours included: node a_k sits between b
// entries k - 1 and k, node b_k between a entries k and k + 1.  16-byte loads
// and stores; the arithmetic is seg_residual's, node by node (the same
// result).  The rows of the ghost chunks follow as in k_residual.
template <int D>
__device__ __forceinline__ void split_residual_lane(const Desc &L, const Item &it, int t, bool live) {
    const Seg s = seg_of(it);
    const int q0 = 8 * t;
    const int nv = min(max(s.len - q0, 0), 8);
    const long long pa = s.p0 + (nv > 0 ? q0 : 0), pb = pa + 1;
    const long long half = L.half_u;
    auto at = [&](long long p, long long h) { return (p >> 1) + ((p & 1) ? h : 0LL); };
    const long long lim = L.nn + kSplitPad - 5;
    auto base = [&](long long b) { return b < 0 ? 0LL : (b > lim ? lim : b); };
    gcp<float> U = (gcp<float>)L.u;
    gcp<float> F = (gcp<float>)L.rhs;
    const long long ia = at(pa, half), ib = at(pb, half);
    const f32x4u a4 = *(gcp<f32x4u>)(U + base(ia));
    const float a5 = U[base(ia) + 4];
    const float b0 = U[base(ib - 1)];
    const f32x4u b4 = *(gcp<f32x4u>)(U + base(ib));
    const f32x4u fa = *(gcp<f32x4u>)(F + base(ia));
    const f32x4u fb = *(gcp<f32x4u>)(F + base(ib));
    f32x4u yam = {0, 0, 0, 0}, yap = {0, 0, 0, 0}, ybm = {0, 0, 0, 0}, ybp = {0, 0, 0, 0};
    f32x4u zam = {0, 0, 0, 0}, zap = {0, 0, 0, 0}, zbm = {0, 0, 0, 0}, zbp = {0, 0, 0, 0};
    if (D >= 2) {
        yam = *(gcp<f32x4u>)(U + base(at(pa - L.sy, half)));
        yap = *(gcp<f32x4u>)(U + base(at(pa + L.sy, half)));
        ybm = *(gcp<f32x4u>)(U + base(at(pb - L.sy, half)));
        ybp = *(gcp<f32x4u>)(U + base(at(pb + L.sy, half)));
    }
    if (D >= 3) {
        zam = *(gcp<f32x4u>)(U + base(at(pa - L.sz, half)));
        zap = *(gcp<f32x4u>)(U + base(at(pa + L.sz, half)));
        zbm = *(gcp<f32x4u>)(U + base(at(pb - L.sz, half)));
        zbp = *(gcp<f32x4u>)(U + base(at(pb + L.sz, half)));
    }
    int c[8];
#pragma unroll
    for (int j = 0; j < 8; j++) c[j] = C_INSIDE;
    if (!s.all_inside) {
        gcp<uint8_t> cls = (gcp<uint8_t>)L.cls;
#pragma unroll
        for (int j = 0; j < 8; j++) c[j] = cls[pa + (j < nv ? j : 0)];
    }
    const float A[5] = {a4.x, a4.y, a4.z, a4.w, a5};
    const float B[5] = {b0, b4.x, b4.y, b4.z, b4.w};  // b entries ib - 1 .. ib + 3
    const float FA[4] = {fa.x, fa.y, fa.z, fa.w}, FB[4] = {fb.x, fb.y, fb.z, fb.w};
    const float YAM[4] = {yam.x, yam.y, yam.z, yam.w}, YAP[4] = {yap.x, yap.y, yap.z, yap.w};
    const float YBM[4] = {ybm.x, ybm.y, ybm.z, ybm.w}, YBP[4] = {ybp.x, ybp.y, ybp.z, ybp.w};
    const float ZAM[4] = {zam.x, zam.y, zam.z, zam.w}, ZAP[4] = {zap.x, zap.y, zap.z, zap.w};
    const float ZBM[4] = {zbm.x, zbm.y, zbm.z, zbm.w}, ZBP[4] = {zbp.x, zbp.y, zbp.z, zbp.w};
    float ra[4], rb[4];
    auto row = [&](double up, double fp, double xm, double xp, double ym, double yp, double zm, double zp) {
        double sum = xp + xm;
        if (D >= 2) sum += yp + ym;
        if (D >= 3) sum += zp + zm;
        double lap = (2.0 * D * up - sum) / L.h2;
        if (L.reaction != 0.0) lap += L.reaction * up;  // c u - Laplace u
        return fp - lap;
    };
#pragma unroll
    for (int k = 0; k < 4; k++) {
        ra[k] = (float)row((double)A[k], (double)FA[k], (double)B[k], (double)B[k + 1], (double)YAM[k],
                           (double)YAP[k], (double)ZAM[k], (double)ZAP[k]);
        rb[k] = (float)row((double)B[k + 1], (double)FB[k], (double)A[k], (double)A[k + 1], (double)YBM[k],
                           (double)YBP[k], (double)ZBM[k], (double)ZBP[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        pin(ra[k]);
        pin(rb[k]);
    }
    if (!live || nv <= 0) return;
    gp<float> R = (gp<float>)L.r;
    const long long ra0 = at(pa, L.half_r), rb0 = at(pb, L.half_r);
    // node a_k is segment node q0 + 2k, b_k is q0 + 2k + 1
    bool fa_all = nv == 8, fb_all = nv == 8;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        fa_all = fa_all && c[2 * k] == C_INSIDE;
        fb_all = fb_all && c[2 * k + 1] == C_INSIDE;
    }
    if (fa_all) {
        *(gp<f32x4u>)(R + ra0) = f32x4u{ra[0], ra[1], ra[2], ra[3]};
    } else {
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (2 * k < nv && c[2 * k] == C_INSIDE) R[ra0 + k] = ra[k];
    }
    if (fb_all) {
        *(gp<f32x4u>)(R + rb0) = f32x4u{rb[0], rb[1], rb[2], rb[3]};
    } else {
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (2 * k + 1 < nv && c[2 * k + 1] == C_INSIDE) R[rb0 + k] = rb[k];
    }
}

template <int D, bool NEU>
__global__ __launch_bounds__(kBlock) void k_residual_split(const Desc *__restrict__ descs,
                                                           const Item *__restrict__ items, int nseg,
                                                           const Item *__restrict__ gch, int nseg_blocks,
                                                           const SlotState *__restrict__ st) {
    const int lb = xcd_block_second_first(nseg_blocks);
    if (lb < nseg_blocks) {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int first = __builtin_amdgcn_readfirstlane((lb * kWavesPerBlock + wave) * 4);
        if (first >= nseg) return;
        const int g = lane >> 4, t = lane & 15;
        Item its[4];
#pragma unroll
        for (int k = 0; k < 4; k++) its[k] = items[min(first + k, nseg - 1)];
        const int nk = min(nseg - first, 4);
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
            if (g < nk) split_residual_lane<D>(L, mine, t, live);
            return;
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (k >= nk) break;
            const Desc L = descs[its[k].x];
            const bool live = st[L.slot].active != 0;
            if (g == k) split_residual_lane<D>(L, its[k], t, live);
        }
        return;
    }
    const int cb = lb - nseg_blocks;
    const Item it = gch[cb];
    const Desc &L = descs[it.x];
    const bool live = st[L.slot].active != 0;
    if ((int)threadIdx.x < it.z) ghost_residual<D, float, float, NEU>(L, it.y + threadIdx.x, live, true);
}

// Weighted Jacobi on the INSIDE rows (Sec. 2.1: the smoother omega D + (1 -
// omega) I, with omega = 2d / (2d + 1) in d dimensions, 2/3 in 1D).  Pass 0
// computes u + omega ((h^2 f + sum of the 2d neighbours) / (2d + c h^2) - u)
// from the old field into r; pass 1 copies r back into u.  Two nodes per
// lane, both loaded before either store.
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                   int nseg, int pass, const SlotState *__restrict__ st) {
    SEG_ITEM
    const Seg s = seg_of(it);
    const NodeArr<T> u = node_u<T>(L);
    const NodeArr<const T> f = node_rhs<const T>(L);
    const NodeArr<T> r = node_r<T>(L);
    const long long nn = L.nn;
    T v[2];
    int cc[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int q = seg_lane_node(lane, h, L.half_u);
        const long long p = s.p0 + (q < s.len ? q : 0);
        cc[h] = ((gcp<uint8_t>)L.cls)[p];
        if (pass == 1) {
            v[h] = r[p];
            continue;
        }
        const T up = u[p], fp = f[p];
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
        const T omega = (T)(2.0 * D / (2.0 * D + 1.0));
        v[h] = up + omega * (((T)L.h2 * fp + sum) / (T)(2.0 * D + L.reaction * L.h2) - up);
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        pin(v[h]);
        pin(cc[h]);
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int q = seg_lane_node(lane, h, L.half_u);
        if (!live || q >= s.len || cc[h] != C_INSIDE) continue;
        if (pass == 0)
            r[s.p0 + q] = v[h];
        else
            u[s.p0 + q] = v[h];
    }
}

// Per-slot sum of the partials in a fixed order (thread t adds entries t,
// t + 1024, ..., then a tree), then the convergence test.  mode 0: ||r^0|| of slots
// waiting for it; mode 1: after ncyc cycles (the first ncyc - 1 of them were
// not followed by a check; their history entries are NaN); mode 2: only store
// the norm.
constexpr int kNormThreads = 1024;

// the workgroup's fixed-order sum of entries [lo, hi) of a slot's partials
// (segment partials first, then its ghost-chunk partials); every thread
// takes part, thread 0 gets the sum
__device__ __forceinline__ double norm_range_sum(const NormRange &R, const double *__restrict__ partials,
                                                 int nseg_total, int lo, int hi) {
    const int nA = R.seg_end - R.seg_beg;
    // a thread's entries are loaded eight at a time and added in order; the
    // tree pairs t with t + w, through LDS while w spans wavefronts and by
    // shuffles within the first wavefront after that (the same pairs)
    double acc = 0.0;
    for (int i0 = lo + (int)threadIdx.x; i0 < hi; i0 += 8 * kNormThreads) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int i = min(i0 + k * kNormThreads, hi - 1);
            v[k] = i < nA ? partials[R.seg_beg + i] : partials[nseg_total + R.gch_beg + (i - nA)];
        }
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (i0 + k * kNormThreads < hi) acc += v[k];
    }
    __shared__ double red[kNormThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kNormThreads / 2; w >= 64; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    double t = 0.0;
    if (threadIdx.x < 64) {
        t = red[threadIdx.x];
        for (int w = 32; w > 0; w >>= 1) t += __shfl_down(t, w);
    }
    return t;
}

// the slot's bookkeeping once its squared norm tot is known (one thread)
__device__ void norm_update(SlotState &S, int s, double tot, const double *__restrict__ rtol2,
                            double *__restrict__ hist, int hist_stride, int mode, int ncyc, double *__restrict__ out) {
    if (out) out[s] = tot;
    if (mode == 0) {
        // a non-finite initial residual (a NaN or Inf in f, g(Q) or u0) ends
        // the solve before any cycle, as a divergence
        const bool finite = isfinite(tot);
        S.r0sq = tot;
        S.tolsq = rtol2[s] * tot;
        S.refsq = tot;
        S.lastsq = tot;
        S.cycles = 0;
        S.status = finite ? BCMG_OK : BCMG_ERR_DIVERGED;
        S.active = finite && tot > 0.0 ? 1 : 0;
        if (hist) hist[(long long)s * hist_stride] = sqrt(tot);
    } else if (mode == 1) {
        const int c0 = S.cycles, c = c0 + ncyc;
        S.cycles = c;
        S.lastsq = tot;
        if (hist) {
            for (int k = c0 + 1; k < c && k < hist_stride; k++) hist[(long long)s * hist_stride + k] = __builtin_nan("");
            if (c < hist_stride) hist[(long long)s * hist_stride + c] = sqrt(tot);
        }
        if (c0 == 0) S.refsq = fmax(S.r0sq, tot);
        if (!isfinite(tot)) {
            S.active = 0;
            S.status = BCMG_ERR_DIVERGED;
        } else if (tot <= S.tolsq) {
            S.active = 0;
            S.status = BCMG_OK;
        } else if (c >= 2 && tot > 1e6 * S.refsq) {
            S.active = 0;
            S.status = BCMG_ERR_DIVERGED;
        } else if (c >= S.max_cycles) {
            S.active = 0;
            S.status = BCMG_ERR_NOT_CONVERGED;
        }
    } else {
        S.lastsq = tot;
    }
}

__global__ __launch_bounds__(kNormThreads) void k_norm_finish(const NormRange *__restrict__ ranges, int nslots,
                                                              const double *__restrict__ partials, int nseg_total,
                                                              SlotState *__restrict__ st,
                                                              const double *__restrict__ rtol2,
                                                              double *__restrict__ hist, int hist_stride, int mode,
                                                              int ncyc, double *__restrict__ out) {
    const int s = blockIdx.x;
    if (s >= nslots) return;
    if (mode == 1 && st[s].active != 1) return;
    if (mode == 0 && st[s].active != 2) return;
    const NormRange R = ranges[s];
    const int n = (R.seg_end - R.seg_beg) + (R.gch_end - R.gch_beg);
    const double tot = norm_range_sum(R, partials, nseg_total, 0, n);
    if (threadIdx.x != 0) return;
    norm_update(st[s], s, tot, rtol2, hist, hist_stride, mode, ncyc, out);
}

// The same for slots with many partials, by nblk workgroups per slot: block
// b sums its fixed share of the entries, in the order above, into
// blk[s nblk + b]; the last block of the slot to finish (counted in cnt[s],
// which it resets) adds the nblk sums in index order and does the
// bookkeeping.  The result depends on nblk only, not on the blocks' timing.
__global__ __launch_bounds__(kNormThreads) void k_norm_finish_split(
    const NormRange *__restrict__ ranges, int nslots, int nblk, const double *__restrict__ partials, int nseg_total,
    double *__restrict__ blk, int *__restrict__ cnt, SlotState *__restrict__ st, const double *__restrict__ rtol2,
    double *__restrict__ hist, int hist_stride, int mode, int ncyc, double *__restrict__ out) {
    const int s = blockIdx.x / nblk, b = blockIdx.x % nblk;
    if (s >= nslots) return;
    if (mode == 1 && st[s].active != 1) return;
    if (mode == 0 && st[s].active != 2) return;
    const NormRange R = ranges[s];
    const int n = (R.seg_end - R.seg_beg) + (R.gch_end - R.gch_beg);
    const int lo = (int)((long long)n * b / nblk), hi = (int)((long long)n * (b + 1) / nblk);
    const double part = norm_range_sum(R, partials, nseg_total, lo, hi);
    if (threadIdx.x != 0) return;
    blk[(long long)s * nblk + b] = part;
    __threadfence();
    if (atomicAdd(&cnt[s], 1) != nblk - 1) return;
    __threadfence();
    double tot = 0.0;
    for (int k = 0; k < nblk; k++) tot += blk[(long long)s * nblk + k];
    cnt[s] = 0;
    norm_update(st[s], s, tot, rtol2, hist, hist_stride, mode, ncyc, out);
}

// Extension of u into the band chunks (ghost values read from u).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ext_gather(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                       int via_need, const SlotState *__restrict__ st) {
    const int rb = xcd_block();
    const Item it = items[rb / kRowLanes];
    const Desc &L = descs[it.x];
    const bool live = st[L.slot].active != 0;
    const int row = (rb % kRowLanes) * kRowsPerBlock + (int)threadIdx.x / kRowLanes;
    if (row >= it.z) return;
    const int e = it.y + row;
    ext_gather_group<T>(L, via_need ? ((gcp<int>)L.bneed)[e] : e, nullptr, threadIdx.x % kRowLanes, live);
}

// Restriction: coarse INSIDE rows by segment blocks, then coarse GHOST rows by
// chunk blocks.
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                     int nseg, const Item *__restrict__ gch, int nseg_blocks,
                                                     const SlotState *__restrict__ st, int red) {
    const int lb = xcd_block_second_first(nseg_blocks);
    if (lb < nseg_blocks) {
        // two wavefronts per segment, one coarse node per lane
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int hidx = __builtin_amdgcn_readfirstlane(lb * kWavesPerBlock + wave);
        if (hidx >= 2 * nseg) return;
        const Item it = items[hidx >> 1];
        const Desc L = descs[it.x];
        const bool live = st[L.slot].active != 0;
        seg_restrict_one<D, T>(L, descs[it.x - 1], it, (hidx & 1) * 64 + lane, live, red != 0);
        return;
    }
    const int rb = lb - nseg_blocks;
    const Item it = gch[rb / kRowLanes];
    const Desc &C = descs[it.x];
    const bool live = st[C.slot].active != 0;
    const int row = (rb % kRowLanes) * kRowsPerBlock + (int)threadIdx.x / kRowLanes;
    if (row >= it.z) return;
    restrict_ghost_group<T>(C, descs[it.x - 1], it.y + row, threadIdx.x % kRowLanes, live);
}

template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                    int nseg, const SlotState *__restrict__ st) {
    SEG_ITEM
    seg_prolong<D, T>(L, descs[it.x + 1], it, lane, live);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse(const Desc *__restrict__ descs, const int *__restrict__ list,
                                                   const SlotState *__restrict__ st) {
    const Desc &L = descs[list[blockIdx.x]];
    if (!st[L.slot].active) return;
    if (L.nc == 0 || L.singular) return;
    __shared__ double b[kCoarseMax];
    coarse_solve_block<T>(L, b);
}

// Iterative refinement: u64 += e32 on INSIDE and GHOST nodes, e32 = 0.
__global__ __launch_bounds__(kBlock) void k_ir_update(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                      int nseg, const SlotState *__restrict__ st,
                                                      float *const *__restrict__ eptr) {
    SEG_ITEM
    const Seg s = seg_of(it);
    // the correction has the layout of the finest FP32 arrays, which the
    // outer descriptor's r (the correction's right-hand side) shares
    const NodeArr<float> ev{(gp<float>)eptr[it.x], L.half_r};
    const NodeArr<double> u = node_u<double>(L);
    double v[2];
    int c[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {  // both nodes loaded before either store
        const int q = lane + 64 * h;
        const long long p = s.p0 + (q < s.len ? q : 0);
        c[h] = ((gcp<uint8_t>)L.cls)[p];
        v[h] = u[p] + (double)ev[p];
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        pin(v[h]);
        pin(c[h]);
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int q = lane + 64 * h;
        if (q >= s.len || !live || (c[h] != C_INSIDE && c[h] != C_GHOST)) continue;
        u[s.p0 + q] = v[h];
        ev[s.p0 + q] = 0.0f;
    }
}

// ------------------------------------------------- coarse levels, one block
// One workgroup per problem runs the part of the V-cycle on its aligned
// levels 0..top (top = min(its finest level, the batch's coarse threshold)):
// pre-smoothing, residual, extension and restriction down to the coarsest
// grid, the exact coarse solve (or 50 smoothing steps when the coarsest
// matrix is singular), then extension, prolongation and post-smoothing back
// up.  Steps are separated by workgroup barriers only.
constexpr int kCoarseThreads = 512;
constexpr int kCoarseWaves = kCoarseThreads / 64;

template <int D, typename T, bool NEU>
__device__ void blk_smooth(const Desc *descs, const Item *items, const CoarseLevel &lv) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int colour = 0; colour < 2; colour++) {
        for (int s = wave; s < lv.nseg; s += kCoarseWaves) {
            const Item it = items[lv.seg + s];
            seg_rb<D, T>(descs[it.x], it, lane, colour, true);
        }
        __syncthreads();
    }
    const int grp = threadIdx.x / kChunk, t = threadIdx.x % kChunk, ngrp = kCoarseThreads / kChunk;
    for (int c = grp; c < lv.ngch; c += ngrp) {
        const Item it = items[lv.gch + c];
        if (t < it.z) ghost_delta<D, T, NEU>(descs[it.x], it.y + t, true);
    }
    __syncthreads();
    for (int c = grp; c < lv.ngch; c += ngrp) {
        const Item it = items[lv.gch + c];
        if (t < it.z) ghost_apply<T>(descs[it.x], it.y + t, true);
    }
    __syncthreads();
}

// Extension of u into the band of one level (after a workgroup barrier).
template <typename T>
__device__ void blk_extend(const Desc *descs, const Item *items, const CoarseLevel &lv) {
    const int grp = threadIdx.x / kChunk, t = threadIdx.x % kChunk, ngrp = kCoarseThreads / kChunk;
    for (int c = grp; c < lv.nbch; c += ngrp) {
        const Item it = items[lv.bch + c];
        if (t < it.z) ext_gather<T>(descs[it.x], it.y + t, nullptr, true);
    }
    __syncthreads();
}

template <int D, typename T, bool NEU>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_cycle(const Desc *__restrict__ descs,
                                                                 const Item *__restrict__ items,
                                                                 const CoarseProg *__restrict__ progs,
                                                                 const SlotState *__restrict__ st, int nu1,
                                                                 int nu2) {
    const CoarseProg &P = progs[blockIdx.x];
    if (!st[P.slot].active) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = threadIdx.x / kChunk, t = threadIdx.x % kChunk, ngrp = kCoarseThreads / kChunk;
    __shared__ double b[kCoarseMax];
    for (int a = P.top; a >= 1; a--) {
        const CoarseLevel &lv = P.lev[a];
        for (int i = 0; i < nu1; i++) blk_smooth<D, T, NEU>(descs, items, lv);
        for (int s = wave; s < lv.nseg; s += kCoarseWaves) {
            const Item it = items[lv.seg + s];
            seg_residual<D, T, T>(descs[it.x], it, lane, true);
        }
        for (int c = grp; c < lv.ngch; c += ngrp) {
            const Item it = items[lv.gch + c];
            if (t < it.z) ghost_residual<D, T, T, NEU>(descs[it.x], it.y + t, true);
        }
        __syncthreads();
        const CoarseLevel &cv = P.lev[a - 1];
        for (int s = wave; s < cv.nseg; s += kCoarseWaves) {
            const Item it = items[cv.seg + s];
            seg_restrict<D, T>(descs[it.x], descs[it.x - 1], it, lane, true, false);
        }
        for (int c = grp; c < cv.ngch; c += ngrp) {
            const Item it = items[cv.gch + c];
            if (t < it.z) restrict_ghost<T>(descs[it.x], descs[it.x - 1], it.y + t, true);
        }
        __syncthreads();
    }
    {
        const CoarseLevel &lv = P.lev[0];
        const Desc &L = descs[lv.desc];
        if (L.nc > 0 && !L.singular) {
            coarse_solve_block<T>(L, b);
        } else if (L.nc > 0) {
            for (int i = 0; i < 50; i++) blk_smooth<D, T, NEU>(descs, items, lv);
        }
    }
    for (int a = 1; a <= P.top; a++) {
        const CoarseLevel &lv = P.lev[a];
        blk_extend<T>(descs, items, P.lev[a - 1]);
        for (int s = wave; s < lv.nseg; s += kCoarseWaves) {
            const Item it = items[lv.seg + s];
            seg_prolong<D, T>(descs[it.x], descs[it.x + 1], it, lane, true);
        }
        __syncthreads();
        for (int i = 0; i < nu2; i++) blk_smooth<D, T, NEU>(descs, items, lv);
    }
    // the error of the top level, extended for the prolongation that follows
    if (P.ext_top) blk_extend<T>(descs, items, P.lev[P.top]);
}

// ------------------------------------------- coarse levels, one block, in LDS
// The same sub-V-cycle as k_coarse_cycle, with every array of the levels
// 0..top (node arrays, ghost records, extension and restriction rows) copied
// into the workgroup's LDS first: each step then loops densely over the
// level's nodes and waits on LDS only.  The top level's u is written back at
// the end (only its unknowns when it is the caller's array).
template <typename V>
using lp = __attribute__((address_space(3))) V *;

template <typename T>
struct LdsView {
    int n, nn, ng, nb, ni, nred;
    long long sy, sz;
    double h2;
    int N;
    lp<uint8_t> cls;
    lp<T> u, rhs, r;
    gp<T> rg;  // the residual in HBM instead of r (null when r is in LDS)
    lp<int> gidx, gcode, ilist, bneed;
    int nbn;
    lp<double> gtau, gdtau, gnew, gnd;
    bool neu;         // Neumann ghost rows (gnd valid)
    double reaction;  // c of c u - Laplace u
    gcp<int> eptr, eidx, bidx, rptr, ridx;  // rows in HBM
    gcp<double> ecoef, rcoef;
};

template <typename V>
__device__ __forceinline__ lp<V> lds_ptr(unsigned char *base, int off) {
    return (lp<V>)(base + off);
}

template <typename V>
__device__ __forceinline__ void lds_zero(lp<V> dst, int n) {
    for (int i = threadIdx.x; i < n; i += kCoarseThreads) dst[i] = V(0);
}

template <int D>
__device__ __forceinline__ void node_coords(int p, int n, int &i, int &j, int &k) {
    i = p % n;
    j = D >= 2 ? (p / n) % n : 0;
    k = D >= 3 ? p / (n * n) : 0;
}

template <int D, typename T, bool NEU>
__device__ __forceinline__ void lds_smooth(const LdsView<T> &L) {
    for (int colour = 0; colour < 2; colour++) {
        const int beg = colour ? L.nred : 0, end = colour ? L.ni : L.nred;
        for (int t = beg + (int)threadIdx.x; t < end; t += kCoarseThreads) {
            const int p = L.ilist[t];
            T sum = L.u[p + 1] + L.u[p - 1];
            if (D >= 2) sum += L.u[p + L.sy] + L.u[p - L.sy];
            if (D >= 3) sum += L.u[p + L.sz] + L.u[p - L.sz];
            L.u[p] = ((T)L.h2 * L.rhs[p] + sum) / (T)(2.0 * D + L.reaction * L.h2);
        }
        __syncthreads();
    }
    for (int g = threadIdx.x; g < L.ng; g += kCoarseThreads) {
        const int p = L.gidx[g];
        const double row = ghost_row_at<D, NEU>(L.gidx, L.gcode, L.gtau, L.gnd, L.neu, L.sy, L.sz, g, L.u);
        L.gnew[g] = (double)(T)((double)L.u[p] + L.gdtau[g] * ((double)L.rhs[p] - row));
    }
    __syncthreads();
    for (int g = threadIdx.x; g < L.ng; g += kCoarseThreads) L.u[L.gidx[g]] = (T)L.gnew[g];
    __syncthreads();
}

template <int D, typename T, bool NEU>
__device__ __forceinline__ void lds_residual(const LdsView<T> &L) {
    for (int t = threadIdx.x; t < L.ni; t += kCoarseThreads) {
        const int p = L.ilist[t];
        double sum = (double)L.u[p + 1] + (double)L.u[p - 1];
        if (D >= 2) sum += (double)L.u[p + L.sy] + (double)L.u[p - L.sy];
        if (D >= 3) sum += (double)L.u[p + L.sz] + (double)L.u[p - L.sz];
        double lap = (2.0 * D * (double)L.u[p] - sum) / L.h2;
        if (L.reaction != 0.0) lap += L.reaction * (double)L.u[p];
        const T v = (T)((double)L.rhs[p] - lap);
        if (L.rg)
            L.rg[p] = v;
        else
            L.r[p] = v;
    }
    for (int g = threadIdx.x; g < L.ng; g += kCoarseThreads) {
        const int p = L.gidx[g];
        const T v = (T)((double)L.rhs[p] - ghost_row_at<D, NEU>(L.gidx, L.gcode, L.gtau, L.gnd, L.neu, L.sy, L.sz, g, L.u));
        if (L.rg)
            L.rg[p] = v;
        else
            L.r[p] = v;
    }
    __threadfence_block();
    __syncthreads();
}

// coarse level C from the residual of the finer level F
template <int D, typename T>
__device__ __forceinline__ void lds_restrict(const LdsView<T> &C, const LdsView<T> &F, int mode) {
    for (int t = threadIdx.x; t < C.ni; t += kCoarseThreads) {
        const int p = C.ilist[t];
        int i, j, k;
        node_coords<D>(p, C.n, i, j, k);
        C.rhs[p] = (T)(F.rg ? restrict_inside_at<D>((gcp<T>)F.rg, F.cls, F.N, F.sy, F.sz, 2 * i, 2 * j, 2 * k, mode)
                            : restrict_inside_at<D>(F.r, F.cls, F.N, F.sy, F.sz, 2 * i, 2 * j, 2 * k, mode));
        C.u[p] = (T)0;
    }
    // coarse ghost rows by lane groups (the bound is a multiple of the group size)
    for (int t = threadIdx.x; t < C.ng * kRowLanes; t += kCoarseThreads) {
        const int g = t / kRowLanes, sub = t % kRowLanes;
        const int beg = C.rptr[g], end = C.rptr[g + 1];
        const double acc =
            F.rg ? row_dot_group(C.ridx, C.rcoef, beg, end, sub, [&](int q) { return (double)((gcp<T>)F.rg)[q]; })
                 : row_dot_group(C.ridx, C.rcoef, beg, end, sub, [&](int q) { return (double)F.r[q]; });
        if (sub != 0) continue;
        const int p = C.gidx[g];
        C.rhs[p] = (T)acc;
        C.u[p] = (T)0;
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void lds_extend(const LdsView<T> &L) {
    for (int t = threadIdx.x; t < L.nbn * kRowLanes; t += kCoarseThreads) {  // by lane groups
        const int b = L.bneed[t / kRowLanes];
        const double v = row_dot_group(L.eidx, L.ecoef, L.eptr[b], L.eptr[b + 1], t % kRowLanes,
                                       [&](int g) { return (double)L.u[L.gidx[g]]; });
        if (t % kRowLanes == 0) L.u[L.bidx[b]] = (T)v;
    }
    __syncthreads();
}

template <int D, typename T>
__device__ __forceinline__ void lds_prolong(const LdsView<T> &F, const LdsView<T> &C) {
    for (int t = threadIdx.x; t < F.ni + F.ng; t += kCoarseThreads) {
        const int p = t < F.ni ? F.ilist[t] : F.gidx[t - F.ni];
        int i, j, k;
        node_coords<D>(p, F.n, i, j, k);
        F.u[p] = (T)((double)F.u[p] + prolong_at<D>(C.u, C.sy, C.sz, i, j, k));
    }
    __syncthreads();
}

// Copy n 4-byte words from HBM into LDS with every thread of the workgroup,
// sixteen loads in flight per thread and round.
__device__ __forceinline__ void lds_copy_words(lp<uint32_t> dst, gcp<uint32_t> src, int n) {
    constexpr int U = 16;
    for (int w0 = threadIdx.x; w0 < n; w0 += U * kCoarseThreads) {
        uint32_t v[U];
#pragma unroll
        for (int k = 0; k < U; k++) v[k] = src[min(w0 + k * kCoarseThreads, n - 1)];
#pragma unroll
        for (int k = 0; k < U; k++)
            if (w0 + k * kCoarseThreads < n) dst[w0 + k * kCoarseThreads] = v[k];
    }
}

// A program's image: the arrays of its levels fixed during a solve, at their
// LDS offsets (one workgroup per program; run when the programs are built).
__global__ __launch_bounds__(kBlock) void k_lds_images(const Desc *__restrict__ descs,
                                                        const LdsProg *__restrict__ progs) {
    const LdsProg &P = progs[blockIdx.x];
    gp<uint32_t> img = (gp<uint32_t>)P.image;
    for (int a = 0; a <= P.top; a++) {
        const LdsLevel &Q = P.lev[a];
        const Desc &G = descs[Q.desc];
        // class arrays are padded allocations, the others whole words
        auto put = [&](const void *src, int off, long long bytes) {
            const int n = (int)((bytes + 3) / 4);
            gcp<uint32_t> sw = (gcp<uint32_t>)src;
            for (int w = threadIdx.x; w < n; w += kBlock) img[off / 4 + w] = sw[w];
        };
        put(G.cls, Q.cls, Q.nn);
        put(G.gidx, Q.gidx, 4LL * Q.ng);
        put(G.gcode, Q.gcode, 4LL * Q.ng);
        put(G.gtau, Q.gtau, 24LL * Q.ng);
        put(G.gdtau, Q.gdtau, 8LL * Q.ng);
        if (Q.gnd >= 0) put(G.gnd, Q.gnd, 24LL * Q.ng);
        put(G.ilist, Q.ilist, 4LL * Q.ni);
        put(G.bneed, Q.bneed, 4LL * Q.nbn);
    }
}

template <int D, typename T, bool NEU>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_lds(const Desc *__restrict__ descs,
                                                               const LdsProg *__restrict__ progs,
                                                               const SlotState *__restrict__ st, int nu1, int nu2) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ double bsh[kCoarseMax];
    const LdsProg &P = progs[blockIdx.x];
    if (!st[P.slot].active) return;
    __shared__ LdsView<T> V[kMaxLevels];
    // Thread a sets up the view of level a.  The LDS block starts with the
    // arrays fixed during a solve, copied from the program's image; the top
    // level's u and rhs follow from HBM: whole when it is the caller's finest
    // level (its box values are read), else rhs at its unknowns only (the
    // other entries are never read) and u zero-filled (after the restriction
    // its unknowns are zero, and its other nodes are written by the
    // extension before they are read).
    const int top = P.top;
    const bool finest = P.finest != 0;
    if ((int)threadIdx.x <= top) {
        const int a = threadIdx.x;
        const LdsLevel &Q = P.lev[a];
        const Desc &G = descs[Q.desc];
        LdsView<T> &W = V[a];
        W.n = G.n;
        W.N = G.N;
        W.nn = Q.nn;
        W.ng = Q.ng;
        W.nb = Q.nb;
        W.ni = Q.ni;
        W.nred = Q.nred;
        W.ilist = lds_ptr<int>(lds, Q.ilist);
        W.nbn = Q.nbn;
        W.bneed = lds_ptr<int>(lds, Q.bneed);
        W.sy = G.sy;
        W.sz = G.sz;
        W.h2 = G.h2;
        W.cls = lds_ptr<uint8_t>(lds, Q.cls);
        W.u = lds_ptr<T>(lds, Q.u);
        W.rhs = lds_ptr<T>(lds, Q.rhs);
        W.r = lds_ptr<T>(lds, Q.r < 0 ? 0 : Q.r);
        W.rg = Q.r < 0 ? (gp<T>)G.r : nullptr;
        W.gidx = lds_ptr<int>(lds, Q.gidx);
        W.gcode = lds_ptr<int>(lds, Q.gcode);
        W.gtau = lds_ptr<double>(lds, Q.gtau);
        W.gdtau = lds_ptr<double>(lds, Q.gdtau);
        W.gnew = lds_ptr<double>(lds, Q.gnew);
        W.neu = Q.gnd >= 0;
        W.gnd = lds_ptr<double>(lds, Q.gnd < 0 ? 0 : Q.gnd);
        W.reaction = G.reaction;
        W.eptr = (gcp<int>)G.eptr;
        W.eidx = (gcp<int>)G.eidx;
        W.ecoef = (gcp<double>)G.ecoef;
        W.bidx = (gcp<int>)G.bidx;
        W.rptr = (gcp<int>)G.rptr;
        W.ridx = (gcp<int>)G.ridx;
        W.rcoef = (gcp<double>)G.rcoef;
    }
    lds_copy_words((lp<uint32_t>)lds, (gcp<uint32_t>)P.image, P.static_words);
    const Desc &GT = descs[P.lev[top].desc];
    if (finest) {
        const LdsLevel &Q = P.lev[top];
        lds_copy_words((lp<uint32_t>)(lds + Q.u), (gcp<uint32_t>)GT.u, (int)((sizeof(T) * Q.nn) / 4));
        lds_copy_words((lp<uint32_t>)(lds + Q.rhs), (gcp<uint32_t>)GT.rhs, (int)((sizeof(T) * Q.nn) / 4));
    }
    __syncthreads();
    if (!finest) {
        const LdsView<T> &W = V[top];
        gcp<T> rhs = (gcp<T>)GT.rhs;
        for (int t0 = threadIdx.x; t0 < W.ni + W.ng; t0 += 4 * kCoarseThreads) {
            int pk[4];
            T v[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int t = min(t0 + k * kCoarseThreads, W.ni + W.ng - 1);
                pk[k] = t < W.ni ? W.ilist[t] : W.gidx[t - W.ni];
            }
#pragma unroll
            for (int k = 0; k < 4; k++) v[k] = rhs[pk[k]];
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (t0 + k * kCoarseThreads < W.ni + W.ng) W.rhs[pk[k]] = v[k];
        }
    }
    for (int a = 0; a <= top; a++) {
        const LdsView<T> &W = V[a];
        if (a != top || !finest) lds_zero(W.u, W.nn);
        if (a != top) lds_zero(W.rhs, W.nn);
        if (!W.rg) lds_zero(W.r, W.nn);
    }
    __syncthreads();
    const int mode = descs[P.lev[0].desc].restrict_mode;
    for (int a = top; a >= 1; a--) {
        for (int i = 0; i < nu1; i++) lds_smooth<D, T, NEU>(V[a]);
        lds_residual<D, T, NEU>(V[a]);
        lds_restrict<D, T>(V[a - 1], V[a], mode);
    }
    {
        const Desc &G = descs[P.lev[0].desc];
        if (G.nc > 0 && !G.singular) {
            gcp<int> cmap = (gcp<int>)G.cmap;
            gcp<double> ainv = (gcp<double>)G.ainv;
            for (int t = threadIdx.x; t < G.nc; t += kCoarseThreads) bsh[t] = (double)V[0].rhs[cmap[t]];
            __syncthreads();
            for (int t = threadIdx.x; t < G.nc; t += kCoarseThreads) {
                gcp<double> row = ainv + (long long)t * G.nc;
                double x = 0.0;
                for (int j = 0; j < G.nc; j += 8) {  // eight loads in flight, sum in row order
                    double a[8];
#pragma unroll
                    for (int k = 0; k < 8; k++) a[k] = row[min(j + k, G.nc - 1)];
#pragma unroll
                    for (int k = 0; k < 8; k++)
                        if (j + k < G.nc) x += a[k] * bsh[j + k];
                }
                V[0].u[cmap[t]] = (T)x;
            }
            __syncthreads();
        } else if (G.nc > 0) {
            for (int i = 0; i < 50; i++) lds_smooth<D, T, NEU>(V[0]);
        }
    }
    for (int a = 1; a <= top; a++) {
        lds_extend<T>(V[a - 1]);
        lds_prolong<D, T>(V[a], V[a - 1]);
        for (int i = 0; i < nu2; i++) lds_smooth<D, T, NEU>(V[a]);
    }
    if (P.ext_top) lds_extend<T>(V[top]);
    const LdsView<T> &W = V[top];
    gp<T> ug = (gp<T>)descs[P.lev[top].desc].u;
    for (int p = threadIdx.x; p < W.nn; p += kCoarseThreads) {
        const int c = W.cls[p];
        if (finest && c != C_INSIDE && c != C_GHOST) continue;
        ug[p] = W.u[p];
    }
}

// ---------------------------------------------------------------- launchers
static inline int blocks_for_segs(int nseg) { return (nseg + kWavesPerBlock - 1) / kWavesPerBlock; }

#define DISPATCH_D(d, KERNEL, T, ...)                                          \
    do {                                                                       \
        if ((d) == 1) hipLaunchKernelGGL((KERNEL<1, T>), __VA_ARGS__);         \
        if ((d) == 2) hipLaunchKernelGGL((KERNEL<2, T>), __VA_ARGS__);         \
        if ((d) == 3) hipLaunchKernelGGL((KERNEL<3, T>), __VA_ARGS__);         \
    } while (0)

#define DISPATCH_DB(d, KERNEL, T, B, ...)                                      \
    do {                                                                       \
        if ((d) == 1) hipLaunchKernelGGL((KERNEL<1, T, B>), __VA_ARGS__);      \
        if ((d) == 2) hipLaunchKernelGGL((KERNEL<2, T, B>), __VA_ARGS__);      \
        if ((d) == 3) hipLaunchKernelGGL((KERNEL<3, T, B>), __VA_ARGS__);      \
    } while (0)

// kernels with the Neumann ghost rows compiled in (neu: some problem of the
// launch has them) or not
#define DISPATCH_DN(d, neu, KERNEL, T, ...)                                    \
    do {                                                                       \
        if (neu)                                                               \
            DISPATCH_DB(d, KERNEL, T, true, __VA_ARGS__);                      \
        else                                                                   \
            DISPATCH_DB(d, KERNEL, T, false, __VA_ARGS__);                     \
    } while (0)

void launch_rb_sweep(int d, int fp32, const Desc *descs, const Item *items, int nseg, int colour,
                     const SlotState *st, hipStream_t s, int pair_min) {
    if (nseg <= 0) return;
    dim3 b(kBlock);
    if (fp32 && nseg >= pair_min && d >= 2) {  // split levels: four segments per wavefront
        dim3 g(blocks_for_segs((nseg + 3) / 4));
        if (d == 2) hipLaunchKernelGGL((k_rb_sweep_split4<2>), g, b, 0, s, descs, items, nseg, colour, st);
        if (d == 3) hipLaunchKernelGGL((k_rb_sweep_split4<3>), g, b, 0, s, descs, items, nseg, colour, st);
        return;
    }
    dim3 g(blocks_for_segs(nseg));
    if (fp32)
        DISPATCH_D(d, k_rb_sweep, float, g, b, 0, s, descs, items, nseg, colour, st);
    else
        DISPATCH_D(d, k_rb_sweep, double, g, b, 0, s, descs, items, nseg, colour, st);
}

void launch_jacobi(int d, int fp32, const Desc *descs, const Item *items, int nseg, const SlotState *st,
                   hipStream_t s) {
    if (nseg <= 0) return;
    dim3 g(blocks_for_segs(nseg)), b(kBlock);
    for (int pass = 0; pass < 2; pass++) {
        if (fp32)
            DISPATCH_D(d, k_jacobi, float, g, b, 0, s, descs, items, nseg, pass, st);
        else
            DISPATCH_D(d, k_jacobi, double, g, b, 0, s, descs, items, nseg, pass, st);
    }
}

void launch_ghost_relax(int d, int fp32, const Desc *descs, const Item *gch, int ngch, const SlotState *st,
                        hipStream_t s, const Item *bch, int nbch, int neu) {
    if (ngch <= 0 && nbch <= 0) return;
    dim3 g(ngch * kGhostSplit), gb(kGhostBlock), ga(ngch + nbch * kRowLanes), b(kBlock);
    if (fp32) {
        if (ngch > 0) DISPATCH_DN(d, neu, k_ghost_delta, float, g, gb, 0, s, descs, gch, st);
        hipLaunchKernelGGL((k_ghost_apply<float>), ga, b, 0, s, descs, gch, ngch, bch, st);
    } else {
        if (ngch > 0) DISPATCH_DN(d, neu, k_ghost_delta, double, g, gb, 0, s, descs, gch, st);
        hipLaunchKernelGGL((k_ghost_apply<double>), ga, b, 0, s, descs, gch, ngch, bch, st);
    }
}

template <typename Tu, typename Tr, bool NORM, bool NEU>
static void residual_t(int d, const Desc *descs, const Item *segs, int nseg, const Item *gch, int ngch,
                       const SlotState *st, double *partials, hipStream_t s, int store) {
    const int sb = blocks_for_segs(nseg);
    if (sb + ngch <= 0) return;
    dim3 g(sb + ngch), b(kBlock);
    if (d == 1)
        hipLaunchKernelGGL((k_residual<1, Tu, Tr, NORM, NEU>), g, b, 0, s, descs, segs, nseg, gch, sb, st, partials,
                           store);
    if (d == 2)
        hipLaunchKernelGGL((k_residual<2, Tu, Tr, NORM, NEU>), g, b, 0, s, descs, segs, nseg, gch, sb, st, partials,
                           store);
    if (d == 3)
        hipLaunchKernelGGL((k_residual<3, Tu, Tr, NORM, NEU>), g, b, 0, s, descs, segs, nseg, gch, sb, st, partials,
                           store);
}

template <bool NEU>
static void residual_n(int d, int tu32, int tr32, int norm, const Desc *descs, const Item *segs, int nseg,
                       const Item *gch, int ngch, const SlotState *st, double *partials, hipStream_t s, int store,
                       int split) {
    if (split && tu32 && tr32 && !norm && store && d >= 2) {  // split FP32 level: vector loads and stores
        const int sb = blocks_for_segs((nseg + 3) / 4);
        if (sb + ngch <= 0) return;
        dim3 g(sb + ngch), b(kBlock);
        if (d == 2) hipLaunchKernelGGL((k_residual_split<2, NEU>), g, b, 0, s, descs, segs, nseg, gch, sb, st);
        if (d == 3) hipLaunchKernelGGL((k_residual_split<3, NEU>), g, b, 0, s, descs, segs, nseg, gch, sb, st);
        return;
    }
    if (!tu32 && !tr32) {
        if (norm)
            residual_t<double, double, true, NEU>(d, descs, segs, nseg, gch, ngch, st, partials, s, store);
        else
            residual_t<double, double, false, NEU>(d, descs, segs, nseg, gch, ngch, st, partials, s, store);
    } else if (!tu32 && tr32) {
        if (norm)
            residual_t<double, float, true, NEU>(d, descs, segs, nseg, gch, ngch, st, partials, s, store);
        else
            residual_t<double, float, false, NEU>(d, descs, segs, nseg, gch, ngch, st, partials, s, store);
    } else {
        residual_t<float, float, false, NEU>(d, descs, segs, nseg, gch, ngch, st, partials, s, store);
    }
}

void launch_residual(int d, int tu32, int tr32, int norm, const Desc *descs, const Item *segs, int nseg,
                     const Item *gch, int ngch, const SlotState *st, double *partials, hipStream_t s, int neu,
                     int store, int split) {
    if (neu)
        residual_n<true>(d, tu32, tr32, norm, descs, segs, nseg, gch, ngch, st, partials, s, store, split);
    else
        residual_n<false>(d, tu32, tr32, norm, descs, segs, nseg, gch, ngch, st, partials, s, store, split);
}

void launch_norm_finish(const NormRange *ranges, int nslots, const double *partials, int nseg_total, SlotState *st,
                        const double *rtol2, double *hist, int hist_stride, int mode, double *out, hipStream_t s,
                        int ncyc, int nblk, double *blk, int *cnt) {
    if (nslots <= 0) return;
    if (nblk > 1 && blk && cnt) {
        hipLaunchKernelGGL(k_norm_finish_split, dim3(nslots * nblk), dim3(kNormThreads), 0, s, ranges, nslots, nblk,
                           partials, nseg_total, blk, cnt, st, rtol2, hist, hist_stride, mode, ncyc, out);
        return;
    }
    hipLaunchKernelGGL(k_norm_finish, dim3(nslots), dim3(kNormThreads), 0, s, ranges, nslots, partials, nseg_total,
                       st, rtol2, hist, hist_stride, mode, ncyc, out);
}

void launch_ext_gather(int fp32, const Desc *descs, const Item *bch, int nbch, int via_need, const SlotState *st,
                       hipStream_t s) {
    if (nbch <= 0) return;
    if (fp32)
        hipLaunchKernelGGL((k_ext_gather<float>), dim3(nbch * kRowLanes), dim3(kBlock), 0, s, descs, bch, via_need, st);
    else
        hipLaunchKernelGGL((k_ext_gather<double>), dim3(nbch * kRowLanes), dim3(kBlock), 0, s, descs, bch, via_need,
                           st);
}

void launch_restrict(int d, int fp32, const Desc *descs, const Item *csegs, int nseg, const Item *cgch, int ncgch,
                     const SlotState *st, hipStream_t s, int red) {
    const int sb = blocks_for_segs(2 * nseg);  // two wavefronts per coarse segment
    if (sb + ncgch <= 0) return;
    dim3 g(sb + ncgch * kRowLanes), b(kBlock);
    if (fp32)
        DISPATCH_D(d, k_restrict, float, g, b, 0, s, descs, csegs, nseg, cgch, sb, st, red);
    else
        DISPATCH_D(d, k_restrict, double, g, b, 0, s, descs, csegs, nseg, cgch, sb, st, red);
}

void launch_prolong(int d, int fp32, const Desc *descs, const Item *fsegs, int nseg, const SlotState *st,
                    hipStream_t s) {
    if (nseg <= 0) return;
    dim3 g(blocks_for_segs(nseg)), b(kBlock);
    if (fp32)
        DISPATCH_D(d, k_prolong, float, g, b, 0, s, descs, fsegs, nseg, st);
    else
        DISPATCH_D(d, k_prolong, double, g, b, 0, s, descs, fsegs, nseg, st);
}

void launch_coarse(int fp32, const Desc *descs, const int *list, int n, const SlotState *st, hipStream_t s) {
    if (n <= 0) return;
    if (fp32)
        hipLaunchKernelGGL((k_coarse<float>), dim3(n), dim3(kBlock), 0, s, descs, list, st);
    else
        hipLaunchKernelGGL((k_coarse<double>), dim3(n), dim3(kBlock), 0, s, descs, list, st);
}

void launch_coarse_cycle(int d, int fp32, const Desc *descs, const Item *items, const CoarseProg *progs, int nprog,
                         const SlotState *st, int nu1, int nu2, hipStream_t s, int neu) {
    if (nprog <= 0) return;
    dim3 g(nprog), b(kCoarseThreads);
    if (fp32)
        DISPATCH_DN(d, neu, k_coarse_cycle, float, g, b, 0, s, descs, items, progs, st, nu1, nu2);
    else
        DISPATCH_DN(d, neu, k_coarse_cycle, double, g, b, 0, s, descs, items, progs, st, nu1, nu2);
}

void launch_lds_images(const Desc *descs, const LdsProg *progs, int nprog, hipStream_t s) {
    if (nprog <= 0) return;
    hipLaunchKernelGGL(k_lds_images, dim3(nprog), dim3(kBlock), 0, s, descs, progs);
}

void launch_coarse_lds(int d, int fp32, const Desc *descs, const LdsProg *progs, int nprog, size_t lds_bytes,
                       const SlotState *st, int nu1, int nu2, hipStream_t s, int neu) {
    if (nprog <= 0) return;
    dim3 g(nprog), b(kCoarseThreads);
    if (fp32)
        DISPATCH_DN(d, neu, k_coarse_lds, float, g, b, lds_bytes, s, descs, progs, st, nu1, nu2);
    else
        DISPATCH_DN(d, neu, k_coarse_lds, double, g, b, lds_bytes, s, descs, progs, st, nu1, nu2);
}

void launch_ir_update(const Desc *descs, const Item *segs, int nseg, const SlotState *st, float *const *eptr,
                      hipStream_t s) {
    if (nseg <= 0) return;
    hipLaunchKernelGGL(k_ir_update, dim3(blocks_for_segs(nseg)), dim3(kBlock), 0, s, descs, segs, nseg, st, eptr);
}

}  // namespace bcmg
