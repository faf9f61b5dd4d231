// Kernels of one multigrid cycle (smoothing, ghost relaxation, residual and
// norm, normal extension, restriction, prolongation, coarse solve, iterative
// refinement update).  Each launch walks a work list (see bcmg_internal.h)
// and reads its level descriptor from a table, so the same kernels serve a
// single problem and a batch of problems of different sizes.
//
// Row-segment kernels: one wavefront per segment of <= 64 consecutive nodes
// of a grid row (coalesced 64 x 8 B accesses); chunk kernels: one workgroup
// per <= 256 ghost or band entries.
#include "bcmg_internal.h"
#include "launch.h"

namespace bcmg {

#define SEG_PROLOGUE                                                  \
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;       \
    const int sidx = blockIdx.x * kWavesPerBlock + wave;              \
    if (sidx >= nseg) return;                                         \
    const Item it = items[sidx];                                      \
    const Desc &L = descs[it.x];                                      \
    if (!st[L.slot].active) return;                                   \
    const int len = it.z >> 16, x0 = it.z & 0xffff;                   \
    const int yj = it.w & 0xffff, zk = it.w >> 16;                    \
    const long long p = (long long)it.y + lane;

__device__ __forceinline__ double lagrange(int w, int m, double t) {
    if (w == 1) return 1.0;
    if (w == 2) return m == 0 ? 1.0 - t : t;
    if (m == 0) return (1.0 - t) * (2.0 - t) / 2.0;
    if (m == 1) return t * (2.0 - t);
    return t * (t - 1.0) / 2.0;
}

// sum_m w_m u(G - m o s) of ghost g (eq. BCh, Dirichlet), tensor-product
// Lagrange weights of widths w_k at the local coordinates tau_k of Q.
template <int D, typename T>
__device__ __forceinline__ double ghost_row(const Desc &L, int g, const T *__restrict__ u) {
    const long long p = L.gidx[g];
    const int code = L.gcode[g];
    int w[3];
    long long step[3];
    double la[3][3];
    const long long str[3] = {1, L.sy, L.sz};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        w[k] = k < D ? code_w(code, k) : 1;
        step[k] = k < D ? (long long)code_s(code, k) * str[k] : 0;
        const double t = k < D ? L.gtau[3 * g + k] : 0.0;
#pragma unroll
        for (int m = 0; m < 3; m++) la[k][m] = lagrange(w[k], m, t);
    }
    double acc = 0.0;
    for (int m2 = 0; m2 < w[2]; m2++)
        for (int m1 = 0; m1 < w[1]; m1++)
            for (int m0 = 0; m0 < w[0]; m0++) {
                double wgt = 1.0;
                wgt *= la[0][m0];
                wgt *= la[1][m1];
                wgt *= la[2][m2];
                acc += wgt * (double)u[p - m0 * step[0] - m1 * step[1] - m2 * step[2]];
            }
    return acc;
}

// --------------------------------------------------------------------------
// Interior Gauss-Seidel, one colour (red: i+j+k even).  eq. GSLEX_2D in
// red-black order: u_P = (h^2 f_P + sum of the 2d neighbours) / (2d).
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_rb_sweep(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                     int nseg, int colour, const SlotState *__restrict__ st) {
    SEG_PROLOGUE
    if (lane >= len) return;
    if (((x0 + lane + yj + zk) & 1) != colour) return;
    if (L.cls[p] != C_INSIDE) return;
    T *__restrict__ u = (T *)L.u;
    const T *__restrict__ f = (const T *)L.rhs;
    T s = u[p + 1] + u[p - 1];
    if (D >= 2) s += u[p + L.sy] + u[p - L.sy];
    if (D >= 3) s += u[p + L.sz] + u[p - L.sz];
    u[p] = ((T)L.h2 * f[p] + s) / (T)(2 * D);
}

// Ghost relaxation, first half: increments from the current values (eq. rel
// with P_GG = I/dtau: new interior values, old ghost values).
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_ghost_delta(const Desc *__restrict__ descs,
                                                        const Item *__restrict__ items,
                                                        const SlotState *__restrict__ st) {
    const Item it = items[blockIdx.x];
    const Desc &L = descs[it.x];
    if (!st[L.slot].active) return;
    if ((int)threadIdx.x >= it.z) return;
    const int g = it.y + threadIdx.x;
    const T *u = (const T *)L.u;
    const T *rhs = (const T *)L.rhs;
    const double row = ghost_row<D, T>(L, g, u);
    L.gdelta[g] = L.gdtau[g] * ((double)rhs[L.gidx[g]] - row);
}

// Ghost relaxation, second half: u_G += increment.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ghost_apply(const Desc *__restrict__ descs,
                                                        const Item *__restrict__ items,
                                                        const SlotState *__restrict__ st) {
    const Item it = items[blockIdx.x];
    const Desc &L = descs[it.x];
    if (!st[L.slot].active) return;
    if ((int)threadIdx.x >= it.z) return;
    const int g = it.y + threadIdx.x;
    T *u = (T *)L.u;
    const long long p = L.gidx[g];
    u[p] = (T)((double)u[p] + L.gdelta[g]);
}

// --------------------------------------------------------------------------
// Residual r = rhs - A u on INSIDE rows (segment blocks) and GHOST rows (chunk
// blocks), optionally with partial sums of r^2 in a fixed order: one partial
// per segment wavefront, then one per ghost chunk.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int D, typename Tu, typename Tr, bool NORM>
__global__ __launch_bounds__(kBlock) void k_residual(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                     int nseg, const Item *__restrict__ gch, int nseg_blocks,
                                                     const SlotState *__restrict__ st, double *__restrict__ partials) {
    if ((int)blockIdx.x < nseg_blocks) {
        SEG_PROLOGUE
        double r2 = 0.0;
        if (lane < len && L.cls[p] == C_INSIDE) {
            const Tu *__restrict__ u = (const Tu *)L.u;
            const Tu *__restrict__ f = (const Tu *)L.rhs;
            double s = (double)u[p + 1] + (double)u[p - 1];
            if (D >= 2) s += (double)u[p + L.sy] + (double)u[p - L.sy];
            if (D >= 3) s += (double)u[p + L.sz] + (double)u[p - L.sz];
            const double lap = (2.0 * D * (double)u[p] - s) / L.h2;
            const double r = (double)f[p] - lap;
            ((Tr *)L.r)[p] = (Tr)r;
            r2 = r * r;
        }
        if (NORM) {
            r2 = wave_sum(r2);
            if (lane == 0) partials[sidx] = r2;
        }
        return;
    }
    const int cb = blockIdx.x - nseg_blocks;
    const Item it = gch[cb];
    const Desc &L = descs[it.x];
    if (!st[L.slot].active) return;
    double r2 = 0.0;
    if ((int)threadIdx.x < it.z) {
        const int g = it.y + threadIdx.x;
        const long long pg = L.gidx[g];
        const double r = (double)((const Tu *)L.rhs)[pg] - ghost_row<D, Tu>(L, g, (const Tu *)L.u);
        ((Tr *)L.r)[pg] = (Tr)r;
        r2 = r * r;
    }
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

// Per-slot sum of the partials in a fixed order, then the convergence test.
// mode 0: ||r^0|| (start of a solve); mode 1: after a cycle; mode 2: only
// store the norm (residual query).
__global__ __launch_bounds__(kBlock) void k_norm_finish(const NormRange *__restrict__ ranges, int nslots,
                                                        const double *__restrict__ partials, int nseg_total,
                                                        SlotState *__restrict__ st, const double *__restrict__ rtol2,
                                                        double *__restrict__ hist, int hist_stride, int mode,
                                                        double *__restrict__ out) {
    const int s = blockIdx.x;
    if (s >= nslots) return;
    if (mode == 1 && st[s].active != 1) return;
    if (mode == 0 && st[s].active != 2) return;  // only slots waiting for ||r^0||
    const NormRange R = ranges[s];
    const int nA = R.seg_end - R.seg_beg, nB = R.gch_end - R.gch_beg;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nA + nB; i += kBlock)
        acc += i < nA ? partials[R.seg_beg + i] : partials[nseg_total + R.gch_beg + (i - nA)];
    __shared__ double red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double tot = red[0];
    if (out) out[s] = tot;
    SlotState &S = st[s];
    if (mode == 0) {
        S.r0sq = tot;
        S.tolsq = rtol2[s] * tot;
        S.refsq = tot;
        S.lastsq = tot;
        S.cycles = 0;
        S.status = BCMG_OK;
        S.active = tot > 0.0 ? 1 : 0;
        if (hist) hist[(long long)s * hist_stride] = sqrt(tot);
    } else if (mode == 1) {
        const int c = S.cycles + 1;
        S.cycles = c;
        S.lastsq = tot;
        if (hist && c < hist_stride) hist[(long long)s * hist_stride + c] = sqrt(tot);
        if (c == 1) S.refsq = fmax(S.r0sq, tot);
        if (tot <= S.tolsq) {
            S.active = 0;
            S.status = BCMG_OK;
        } else if (!isfinite(tot) || (c >= 2 && tot > 1e6 * S.refsq)) {
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

// --------------------------------------------------------------------------
// Normal extension, one Jacobi sweep over the band: v(X) = sum_k |n_k|
// v(X - s_k e_k) / sum_k |n_k| (Sec. 2.3 transfer operators).  Sweep j of K
// reads the band values of sweep j-1 (0 for j = 1) and writes a ping-pong
// buffer, the last sweep writes the field itself.
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_ext_sweep(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                      int which, int j, int K, const SlotState *__restrict__ st) {
    const Item it = items[blockIdx.x];
    const Desc &L = descs[it.x];
    if (!st[L.slot].active) return;
    if ((int)threadIdx.x >= it.z) return;
    const int b = it.y + threadIdx.x;
    T *field = (T *)(which ? L.r : L.u);
    const T *prev = (const T *)((j & 1) ? L.bufB : L.bufA);  // written by sweep j-1
    T *next = (T *)((j & 1) ? L.bufA : L.bufB);
    const int r0 = L.bref[3 * b];
    double v;
    if (r0 == kRefFallback) {
        // zero weight sum: mean of the GHOST nodes of the 3^d box
        long long x = L.bidx[b];
        int I[3] = {0, 0, 0};
        for (int k = 0; k < D; k++) {
            I[k] = (int)(x % L.n);
            x /= L.n;
        }
        double sum = 0.0;
        int cnt = 0;
        const int lo2 = D >= 3 ? -1 : 0, hi2 = D >= 3 ? 1 : 0, lo1 = D >= 2 ? -1 : 0, hi1 = D >= 2 ? 1 : 0;
        for (int m2 = lo2; m2 <= hi2; m2++)
            for (int m1 = lo1; m1 <= hi1; m1++)
                for (int m0 = -1; m0 <= 1; m0++) {
                    const int J0 = I[0] + m0, J1 = I[1] + m1, J2 = I[2] + m2;
                    if (J0 < 0 || J0 > L.N || (D >= 2 && (J1 < 0 || J1 > L.N)) || (D >= 3 && (J2 < 0 || J2 > L.N)))
                        continue;
                    const long long q = J0 + J1 * L.sy + J2 * L.sz;
                    if (L.cls[q] == C_GHOST) {
                        sum += (double)field[q];
                        cnt++;
                    }
                }
        v = cnt > 0 ? sum / cnt : 0.0;
    } else {
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int k = 0; k < D; k++) {
            const int ref = L.bref[3 * b + k];
            const double wk = L.bw[3 * b + k];
            double val;
            if (ref >= 0)
                val = j >= 2 ? (double)prev[ref] : 0.0;
            else if (ref == kRefZero)
                val = 0.0;
            else
                val = (double)field[-(long long)ref - 1];
            num += wk * val;
            den += wk;
        }
        v = den > 0.0 ? num / den : 0.0;
    }
    if (j == K)
        field[L.bidx[b]] = (T)v;
    else
        next[b] = (T)v;
}

// --------------------------------------------------------------------------
// Restriction to the coarse level of the item (fine level = descriptor - 1):
// coarse INSIDE: FW over the 3^d fine box if all INSIDE, else FW weights of
// the INSIDE nodes renormalised; coarse GHOST: FW of the extended residual if
// the box holds no INSIDE node and lies in the grid, else renormalised over its
// non-INSIDE, non-BOXDIR nodes (eq. coarseFW, Sec. 2.2 FW, Sec. 2.3).  Also
// zeroes the coarse unknowns (initial guess of the coarse correction).
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                     int nseg, const SlotState *__restrict__ st) {
    SEG_PROLOGUE
    if (lane >= len) return;
    const Desc &C = L;
    const Desc &F = descs[it.x - 1];
    const uint8_t cc = C.cls[p];
    if (cc != C_INSIDE && cc != C_GHOST) return;
    ((T *)C.u)[p] = (T)0;
    const int X0 = 2 * (x0 + lane), X1 = 2 * yj, X2 = 2 * zk;
    const T *__restrict__ r = (const T *)F.r;
    double full = 0.0, sel = 0.0, selw = 0.0, msum = 0.0, mcnt = 0.0;
    bool all_ok = true;
    const int lo2 = D >= 3 ? -1 : 0, hi2 = D >= 3 ? 1 : 0, lo1 = D >= 2 ? -1 : 0, hi1 = D >= 2 ? 1 : 0;
    for (int m2 = lo2; m2 <= hi2; m2++)
        for (int m1 = lo1; m1 <= hi1; m1++)
            for (int m0 = -1; m0 <= 1; m0++) {
                double wgt = 1.0;
                wgt *= (m0 == 0 ? 0.5 : 0.25);
                if (D >= 2) wgt *= (m1 == 0 ? 0.5 : 0.25);
                if (D >= 3) wgt *= (m2 == 0 ? 0.5 : 0.25);
                const int J0 = X0 + m0, J1 = X1 + m1, J2 = X2 + m2;
                if (J0 < 0 || J0 > F.N || (D >= 2 && (J1 < 0 || J1 > F.N)) || (D >= 3 && (J2 < 0 || J2 > F.N))) {
                    all_ok = false;
                    continue;
                }
                const long long q = J0 + J1 * F.sy + J2 * F.sz;
                const uint8_t fc = F.cls[q];
                bool take;
                if (cc == C_INSIDE) {
                    take = fc == C_INSIDE;
                    if (!take) all_ok = false;
                } else {
                    take = fc != C_INSIDE && fc != C_BOXDIR;
                    if (fc == C_INSIDE) all_ok = false;
                }
                const double rv = (double)r[q];
                full += wgt * rv;
                if (take) {
                    sel += wgt * rv;
                    selw += wgt;
                    msum += rv;
                    mcnt += 1.0;
                }
            }
    double out;
    if (all_ok)
        out = full;
    else if (C.restrict_mode == BCMG_RESTRICT_PLAIN_MEAN)
        out = mcnt > 0.0 ? msum / mcnt : 0.0;
    else
        out = selw > 0.0 ? sel / selw : 0.0;
    ((T *)C.rhs)[p] = (T)out;
}

// Prolongation and correction on the fine level of the item (coarse level =
// descriptor + 1): multilinear interpolation of the (extended) coarse error
// to INSIDE and GHOST nodes, u += e (Sec. 1.1 interpolation, Sec. 2.2, Sec. 2.3).
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                    int nseg, const SlotState *__restrict__ st) {
    SEG_PROLOGUE
    if (lane >= len) return;
    const Desc &F = L;
    const Desc &C = descs[it.x + 1];
    const uint8_t fc = F.cls[p];
    if (fc != C_INSIDE && fc != C_GHOST) return;
    const int I0 = x0 + lane, I1 = yj, I2 = zk;
    const int h0 = I0 & 1, h1 = D >= 2 ? (I1 & 1) : 0, h2 = D >= 3 ? (I2 & 1) : 0;
    const int B0 = (I0 - h0) / 2, B1 = (I1 - h1) / 2, B2 = (I2 - h2) / 2;
    const T *__restrict__ ec = (const T *)C.u;
    double e = 0.0;
    for (int m2 = 0; m2 <= h2; m2++)
        for (int m1 = 0; m1 <= h1; m1++)
            for (int m0 = 0; m0 <= h0; m0++) {
                double wgt = 1.0;
                if (h0) wgt *= 0.5;
                if (h1) wgt *= 0.5;
                if (h2) wgt *= 0.5;
                e += wgt * (double)ec[(B0 + m0) + (B1 + m1) * C.sy + (B2 + m2) * C.sz];
            }
    T *u = (T *)F.u;
    u[p] = (T)((double)u[p] + e);
}

// --------------------------------------------------------------------------
// Coarsest level: x = A^{-1} b over INSIDE then GHOST unknowns, in FP64.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse(const Desc *__restrict__ descs, const int *__restrict__ list,
                                                   const SlotState *__restrict__ st) {
    const Desc &L = descs[list[blockIdx.x]];
    if (!st[L.slot].active) return;
    const int nc = L.nc;
    if (nc == 0 || L.singular) return;
    __shared__ double b[kCoarseMax];
    const T *rhs = (const T *)L.rhs;
    for (int t = threadIdx.x; t < nc; t += kBlock) b[t] = (double)rhs[L.cmap[t]];
    __syncthreads();
    for (int t = threadIdx.x; t < nc; t += kBlock) {
        double x = 0.0;
        const double *row = L.ainv + (long long)t * nc;
        for (int j = 0; j < nc; j++) x += row[j] * b[j];
        ((T *)L.u)[L.cmap[t]] = (T)x;
    }
}

// --------------------------------------------------------------------------
// Iterative refinement: u64 += e32 on INSIDE and GHOST nodes, e32 = 0.
__global__ __launch_bounds__(kBlock) void k_ir_update(const Desc *__restrict__ descs, const Item *__restrict__ items,
                                                      int nseg, const SlotState *__restrict__ st,
                                                      float *const *__restrict__ eptr) {
    SEG_PROLOGUE
    if (lane >= len) return;
    const uint8_t c = L.cls[p];
    if (c != C_INSIDE && c != C_GHOST) return;
    float *e = eptr[it.x];
    double *u = (double *)L.u;
    u[p] += (double)e[p];
    e[p] = 0.0f;
}

// --------------------------------------------------------------------------
// launchers
static inline int blocks_for_segs(int nseg) { return (nseg + kWavesPerBlock - 1) / kWavesPerBlock; }

template <typename T>
static void rb_sweep_t(int d, const Desc *descs, const Item *items, int nseg, int colour, const SlotState *st,
                       hipStream_t s) {
    if (nseg <= 0) return;
    dim3 g(blocks_for_segs(nseg)), b(kBlock);
    if (d == 1) hipLaunchKernelGGL((k_rb_sweep<1, T>), g, b, 0, s, descs, items, nseg, colour, st);
    if (d == 2) hipLaunchKernelGGL((k_rb_sweep<2, T>), g, b, 0, s, descs, items, nseg, colour, st);
    if (d == 3) hipLaunchKernelGGL((k_rb_sweep<3, T>), g, b, 0, s, descs, items, nseg, colour, st);
}

void launch_rb_sweep(int d, int fp32, const Desc *descs, const Item *items, int nseg, int colour,
                     const SlotState *st, hipStream_t s) {
    if (fp32)
        rb_sweep_t<float>(d, descs, items, nseg, colour, st, s);
    else
        rb_sweep_t<double>(d, descs, items, nseg, colour, st, s);
}

template <typename T>
static void ghost_relax_t(int d, const Desc *descs, const Item *gch, int ngch, const SlotState *st, hipStream_t s) {
    if (ngch <= 0) return;
    dim3 g(ngch), b(kBlock);
    if (d == 1) hipLaunchKernelGGL((k_ghost_delta<1, T>), g, b, 0, s, descs, gch, st);
    if (d == 2) hipLaunchKernelGGL((k_ghost_delta<2, T>), g, b, 0, s, descs, gch, st);
    if (d == 3) hipLaunchKernelGGL((k_ghost_delta<3, T>), g, b, 0, s, descs, gch, st);
    hipLaunchKernelGGL((k_ghost_apply<T>), g, b, 0, s, descs, gch, st);
}

void launch_ghost_relax(int d, int fp32, const Desc *descs, const Item *gch, int ngch, const SlotState *st,
                        hipStream_t s) {
    if (fp32)
        ghost_relax_t<float>(d, descs, gch, ngch, st, s);
    else
        ghost_relax_t<double>(d, descs, gch, ngch, st, s);
}

template <typename Tu, typename Tr, bool NORM>
static void residual_t(int d, const Desc *descs, const Item *segs, int nseg, const Item *gch, int ngch,
                       const SlotState *st, double *partials, hipStream_t s) {
    const int sb = blocks_for_segs(nseg);
    if (sb + ngch <= 0) return;
    dim3 g(sb + ngch), b(kBlock);
    if (d == 1) hipLaunchKernelGGL((k_residual<1, Tu, Tr, NORM>), g, b, 0, s, descs, segs, nseg, gch, sb, st, partials);
    if (d == 2) hipLaunchKernelGGL((k_residual<2, Tu, Tr, NORM>), g, b, 0, s, descs, segs, nseg, gch, sb, st, partials);
    if (d == 3) hipLaunchKernelGGL((k_residual<3, Tu, Tr, NORM>), g, b, 0, s, descs, segs, nseg, gch, sb, st, partials);
}

void launch_residual(int d, int tu32, int tr32, int norm, const Desc *descs, const Item *segs, int nseg,
                     const Item *gch, int ngch, const SlotState *st, double *partials, hipStream_t s) {
    if (!tu32 && !tr32) {
        if (norm)
            residual_t<double, double, true>(d, descs, segs, nseg, gch, ngch, st, partials, s);
        else
            residual_t<double, double, false>(d, descs, segs, nseg, gch, ngch, st, partials, s);
    } else if (!tu32 && tr32) {
        if (norm)
            residual_t<double, float, true>(d, descs, segs, nseg, gch, ngch, st, partials, s);
        else
            residual_t<double, float, false>(d, descs, segs, nseg, gch, ngch, st, partials, s);
    } else {
        residual_t<float, float, false>(d, descs, segs, nseg, gch, ngch, st, partials, s);
    }
}

void launch_norm_finish(const NormRange *ranges, int nslots, const double *partials, int nseg_total, SlotState *st,
                        const double *rtol2, double *hist, int hist_stride, int mode, double *out, hipStream_t s) {
    if (nslots <= 0) return;
    hipLaunchKernelGGL(k_norm_finish, dim3(nslots), dim3(kBlock), 0, s, ranges, nslots, partials, nseg_total, st, rtol2,
                       hist, hist_stride, mode, out);
}

template <typename T>
static void extend_t(int d, const Desc *descs, const Item *bch, int nbch, int which, int K, const SlotState *st,
                     hipStream_t s) {
    if (nbch <= 0) return;
    dim3 g(nbch), b(kBlock);
    for (int j = 1; j <= K; j++) {
        if (d == 1) hipLaunchKernelGGL((k_ext_sweep<1, T>), g, b, 0, s, descs, bch, which, j, K, st);
        if (d == 2) hipLaunchKernelGGL((k_ext_sweep<2, T>), g, b, 0, s, descs, bch, which, j, K, st);
        if (d == 3) hipLaunchKernelGGL((k_ext_sweep<3, T>), g, b, 0, s, descs, bch, which, j, K, st);
    }
}

void launch_extend(int d, int fp32, const Desc *descs, const Item *bch, int nbch, int which, int K,
                   const SlotState *st, hipStream_t s) {
    if (fp32)
        extend_t<float>(d, descs, bch, nbch, which, K, st, s);
    else
        extend_t<double>(d, descs, bch, nbch, which, K, st, s);
}

template <typename T>
static void restrict_t(int d, const Desc *descs, const Item *csegs, int nseg, const SlotState *st, hipStream_t s) {
    if (nseg <= 0) return;
    dim3 g(blocks_for_segs(nseg)), b(kBlock);
    if (d == 1) hipLaunchKernelGGL((k_restrict<1, T>), g, b, 0, s, descs, csegs, nseg, st);
    if (d == 2) hipLaunchKernelGGL((k_restrict<2, T>), g, b, 0, s, descs, csegs, nseg, st);
    if (d == 3) hipLaunchKernelGGL((k_restrict<3, T>), g, b, 0, s, descs, csegs, nseg, st);
}

void launch_restrict(int d, int fp32, const Desc *descs, const Item *csegs, int nseg, const SlotState *st,
                     hipStream_t s) {
    if (fp32)
        restrict_t<float>(d, descs, csegs, nseg, st, s);
    else
        restrict_t<double>(d, descs, csegs, nseg, st, s);
}

template <typename T>
static void prolong_t(int d, const Desc *descs, const Item *fsegs, int nseg, const SlotState *st, hipStream_t s) {
    if (nseg <= 0) return;
    dim3 g(blocks_for_segs(nseg)), b(kBlock);
    if (d == 1) hipLaunchKernelGGL((k_prolong<1, T>), g, b, 0, s, descs, fsegs, nseg, st);
    if (d == 2) hipLaunchKernelGGL((k_prolong<2, T>), g, b, 0, s, descs, fsegs, nseg, st);
    if (d == 3) hipLaunchKernelGGL((k_prolong<3, T>), g, b, 0, s, descs, fsegs, nseg, st);
}

void launch_prolong(int d, int fp32, const Desc *descs, const Item *fsegs, int nseg, const SlotState *st,
                    hipStream_t s) {
    if (fp32)
        prolong_t<float>(d, descs, fsegs, nseg, st, s);
    else
        prolong_t<double>(d, descs, fsegs, nseg, st, s);
}

void launch_coarse(int fp32, const Desc *descs, const int *list, int n, const SlotState *st, hipStream_t s) {
    if (n <= 0) return;
    if (fp32)
        hipLaunchKernelGGL((k_coarse<float>), dim3(n), dim3(kBlock), 0, s, descs, list, st);
    else
        hipLaunchKernelGGL((k_coarse<double>), dim3(n), dim3(kBlock), 0, s, descs, list, st);
}

void launch_ir_update(const Desc *descs, const Item *segs, int nseg, const SlotState *st, float *const *eptr,
                      hipStream_t s) {
    if (nseg <= 0) return;
    hipLaunchKernelGGL(k_ir_update, dim3(blocks_for_segs(nseg)), dim3(kBlock), 0, s, descs, segs, nseg, st, eptr);
}

}  // namespace bcmg
