// Setup kernels: level-set injection, node classification, ordered
// compaction (ghost list, extension band), ghost geometry (normal, upwind
// stencil widths, projection Q, theta~, dtau), band references, row extents
// and the coarsest-level inverse.
//
// This file is compiled with -ffp-contract=off: the geometry is evaluated
// with exactly the rounded operations written here (no fused multiply-add),
// so classes, ghost lists and stencil codes depend only on exact comparisons
// of the given FP64 node values of phi.
#include <math.h>

#include "bcmg_internal.h"
#include "launch.h"
#include "mem.h"

namespace bcmg {

__device__ __forceinline__ void coords(long long p, int n, int d, int I[3]) {
    I[0] = I[1] = I[2] = 0;
    for (int k = 0; k < d; k++) {
        I[k] = (int)(p % n);
        p /= n;
    }
}

__device__ __forceinline__ long long index_of(const int I[3], int n, int d) {
    long long p = 0;
    for (int k = d - 1; k >= 0; k--) p = p * n + I[k];
    return p;
}

__device__ __forceinline__ bool in_box(const int I[3], int N, int d) {
    for (int k = 0; k < d; k++)
        if (I[k] < 0 || I[k] > N) return false;
    return true;
}

__global__ void k_check_finite(const double *a, long long n, int *flag) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(a[i])) *flag = 1;
}

void launch_check_finite(const double *a, long long n, int *flag, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a, n, flag);
}

// phi on a coarse level is the fine value at the same point (every coarse
// node is the fine node 2J).
__global__ void k_inject(int d, const double *phi_f, int nf, double *phi_c, int nc, long long nnc) {
    long long pc = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pc >= nnc) return;
    int J[3];
    coords(pc, nc, d, J);
    int X[3] = {2 * J[0], 2 * J[1], 2 * J[2]};
    phi_c[pc] = phi_f[index_of(X, nf, d)];
}

void launch_inject(int d, const double *phi_f, int nf, double *phi_c, int nc, hipStream_t s) {
    long long nnc = 1;
    for (int k = 0; k < d; k++) nnc *= nc;
    hipLaunchKernelGGL(k_inject, dim3((unsigned)((nnc + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, d, phi_f, nf, phi_c,
                       nc, nnc);
}

// Partition of the nodes (Sec. 3.3): INSIDE / BOXDIR by the sign of phi and
// the box faces, then GHOST = not inside with an INSIDE axis neighbour.
__global__ void k_classify_a(int d, int n, const double *phi, uint8_t *cls, long long nn) {
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nn) return;
    int I[3];
    coords(p, n, d, I);
    bool face = false;
    for (int k = 0; k < d; k++) face |= (I[k] == 0 || I[k] == n - 1);
    cls[p] = phi[p] < 0.0 ? (face ? C_BOXDIR : C_INSIDE) : C_OUTSIDE;
}

__global__ void k_classify_b(int d, int n, uint8_t *cls, long long nn) {
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nn) return;
    if (cls[p] != C_OUTSIDE) return;  // only OUTSIDE nodes change, to GHOST; INSIDE never changes
    int I[3];
    coords(p, n, d, I);
    long long str = 1;
    bool ghost = false;
    for (int k = 0; k < d; k++) {
        if (I[k] > 0 && cls[p - str] == C_INSIDE) ghost = true;
        if (I[k] < n - 1 && cls[p + str] == C_INSIDE) ghost = true;
        str *= n;
    }
    if (ghost) cls[p] = C_GHOST;
}

void launch_classify(int d, int n, const double *phi, uint8_t *cls, hipStream_t s) {
    long long nn = 1;
    for (int k = 0; k < d; k++) nn *= n;
    dim3 g((unsigned)((nn + kBlock - 1) / kBlock)), b(kBlock);
    hipLaunchKernelGGL(k_classify_a, g, b, 0, s, d, n, phi, cls, nn);
    hipLaunchKernelGGL(k_classify_b, g, b, 0, s, d, n, cls, nn);
}

// ---------------------------------------------------------------- compaction
constexpr int kPer = 16;
constexpr int kTile = kBlock * kPer;

int compact_blocks(long long nn) { return (int)((nn + kTile - 1) / kTile); }

__device__ int block_exclusive_scan(int v, int *total) {
    __shared__ int buf[kBlock];
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        int add = t >= o ? buf[t - o] : 0;
        __syncthreads();
        buf[t] += add;
        __syncthreads();
    }
    const int incl = buf[t];
    if (total) *total = buf[kBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_compact_count(const uint8_t *cls, long long nn, uint8_t value, int *counts) {
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kPer;
    int c = 0;
    for (int i = 0; i < kPer; i++) {
        const long long p = base + i;
        if (p < nn && cls[p] == value) c++;
    }
    int tot;
    block_exclusive_scan(c, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

__global__ void k_scan_counts(const int *counts, int n, int *offsets, int *total_dev) {
    const int per = (n + kBlock - 1) / kBlock;
    const int beg = threadIdx.x * per;
    int s = 0;
    for (int i = beg; i < beg + per && i < n; i++) s += counts[i];
    int tot;
    int off = block_exclusive_scan(s, &tot);
    for (int i = beg; i < beg + per && i < n; i++) {
        offsets[i] = off;
        off += counts[i];
    }
    if (threadIdx.x == 0) *total_dev = tot;
}

__global__ void k_compact_scatter(const uint8_t *cls, long long nn, uint8_t value, const int *offsets, int *out) {
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kPer;
    int c = 0;
    for (int i = 0; i < kPer; i++) {
        const long long p = base + i;
        if (p < nn && cls[p] == value) c++;
    }
    int off = offsets[blockIdx.x] + block_exclusive_scan(c, nullptr);
    for (int i = 0; i < kPer; i++) {
        const long long p = base + i;
        if (p < nn && cls[p] == value) out[off++] = (int)p;
    }
}

// Exclusive prefix sum of n counts of any size: blocks of kTile counts are
// reduced to block sums, those are scanned (recursively), and every block
// rescans its counts from its offset.
__global__ void k_scan_reduce(const int *in, int n, int *bsum) {
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kPer;
    int c = 0;
    for (int i = 0; i < kPer; i++)
        if (base + i < n) c += in[base + i];
    int tot;
    block_exclusive_scan(c, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_apply(const int *in, int n, const int *boff, int *out) {
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kPer;
    int c = 0;
    for (int i = 0; i < kPer; i++)
        if (base + i < n) c += in[base + i];
    int off = boff[blockIdx.x] + block_exclusive_scan(c, nullptr);
    for (int i = 0; i < kPer; i++)
        if (base + i < n) {
            out[base + i] = off;
            off += in[base + i];
        }
}

hipError_t scan_exclusive(const int *in, int n, int *out, int *total, hipStream_t s) {
    const int nb = (n + kTile - 1) / kTile;
    if (nb <= 1) {
        hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kBlock), 0, s, in, n, out, total);
        return hipSuccess;
    }
    int *tmp = nullptr;
    hipError_t e = scratch_alloc((void **)&tmp, sizeof(int) * 2 * (size_t)nb, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, in, n, tmp);
    e = scan_exclusive(tmp, nb, tmp + nb, total, s);
    if (e == hipSuccess) hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kBlock), 0, s, in, n, tmp + nb, out);
    scratch_free(tmp, s);
    return e;
}

hipError_t launch_compact(const uint8_t *cls, long long nn, uint8_t value, int *counts, int *offsets, int *out,
                          int *total_dev, hipStream_t s) {
    const int nb = compact_blocks(nn);
    hipLaunchKernelGGL(k_compact_count, dim3(nb), dim3(kBlock), 0, s, cls, nn, value, counts);
    const hipError_t e = scan_exclusive(counts, nb, offsets, total_dev, s);
    if (e != hipSuccess) return e;
    if (out) hipLaunchKernelGGL(k_compact_scatter, dim3(nb), dim3(kBlock), 0, s, cls, nn, value, offsets, out);
    return hipSuccess;
}

// ---------------------------------------------------------- ghost geometry
__device__ void grad_at(const double *phi, int n, int d, double h, const int I[3], long long p, double g[3]) {
    g[0] = g[1] = g[2] = 0.0;
    long long str = 1;
    for (int k = 0; k < d; k++) {
        if (I[k] > 0 && I[k] < n - 1)
            g[k] = (phi[p + str] - phi[p - str]) / (2.0 * h);
        else if (I[k] == 0)
            g[k] = (phi[p + str] - phi[p]) / h;
        else
            g[k] = (phi[p] - phi[p - str]) / h;
        str *= n;
    }
}

__device__ __forceinline__ double lag(int w, int m, double t) {
    if (w == 1) return 1.0;
    if (w == 2) return m == 0 ? 1.0 - t : t;
    if (m == 0) return (1.0 - t) * (2.0 - t) / 2.0;
    if (m == 1) return t * (2.0 - t);
    return t * (t - 1.0) / 2.0;
}

__device__ __forceinline__ double lag_dt(int w, int m, double t) {  // d/dt of lag
    if (w == 1) return 0.0;
    if (w == 2) return m == 0 ? -1.0 : 1.0;
    if (m == 0) return t - 1.5;
    if (m == 1) return 2.0 - 2.0 * t;
    return t - 0.5;
}

// Weight of block node m in a ghost row (eq. BCh): Dirichlet prod_k L_{m_k}(tau_k);
// Neumann sum_k nd_k L'_{m_k}(tau_k) prod_{j != k} L_{m_j}(tau_j), the normal
// derivative of the tensor-product interpolant (nd_k = -s_k n_k / h).
__device__ double row_weight(int bc, const int w[3], const double tau[3], const double nd[3], const int m[3]) {
    if (bc == BCMG_BC_DIRICHLET) {
        double wgt = 1.0;
        for (int k = 0; k < 3; k++) wgt *= lag(w[k], m[k], tau[k]);
        return wgt;
    }
    double acc = 0.0;
    for (int k = 0; k < 3; k++) {
        double term = nd[k] * lag_dt(w[k], m[k], tau[k]);
        for (int j = 0; j < 3; j++)
            if (j != k) term *= lag(w[j], m[j], tau[j]);
        acc += term;
    }
    return acc;
}

// tensor-product quadratic interpolant of phi on {I - m o s : m_k < 3}, from
// the node values pv[m2][m1][m0] = phi(I - m o s), loaded once
__device__ double phi_tilde_vals(const double pv[3][3][3], int d, const double t[3]) {
    double val = 0.0;
    const int mmax0 = 3, mmax1 = d >= 2 ? 3 : 1, mmax2 = d >= 3 ? 3 : 1;
    for (int m2 = 0; m2 < mmax2; m2++)
        for (int m1 = 0; m1 < mmax1; m1++)
            for (int m0 = 0; m0 < mmax0; m0++) {
                const int m[3] = {m0, m1, m2};
                double wgt = 1.0;
                for (int k = 0; k < 3; k++)
                    if (k < d) wgt *= lag(3, m[k], t[k]);
                val += wgt * pv[m2][m1][m0];
            }
    return val;
}

// block in the box and made of INSIDE/GHOST nodes (Neumann rows also take
// BOXDIR nodes, whose values g_B are known)
__device__ bool block_valid(const uint8_t *cls, int n, int d, const int I[3], const int s[3], const int w[3], int bc) {
    for (int m2 = 0; m2 < w[2]; m2++)
        for (int m1 = 0; m1 < w[1]; m1++)
            for (int m0 = 0; m0 < w[0]; m0++) {
                const int J[3] = {I[0] - m0 * s[0], I[1] - m1 * s[1], I[2] - m2 * s[2]};
                if (!in_box(J, n - 1, d)) return false;
                const uint8_t c = cls[index_of(J, n, d)];
                if (c == C_BOXDIR && bc == BCMG_BC_NEUMANN) continue;
                if (c != C_INSIDE && c != C_GHOST) return false;
            }
    return true;
}

__device__ int first_inside_neighbour(const uint8_t *cls, long long p, const int I[3], int N, int n, int d,
                                      int &side);

// upwind signs at node J (index q): s_k = +1 where the discrete gradient's
// k-th component is >= 0; a zero gradient takes the direction from the first
// INSIDE axis neighbour to J
__device__ void upwind_signs(const double *phi, const uint8_t *cls, int N, int n, int d, double h, const int J[3],
                             long long q, int sJ[3]) {
    double g[3];
    grad_at(phi, n, d, h, J, q, g);
    double gn = 0.0;
    for (int k = 0; k < d; k++) gn += g[k] * g[k];
    gn = sqrt(gn);
    sJ[0] = sJ[1] = sJ[2] = 1;
    if (gn > 0.0) {
        for (int k = 0; k < d; k++) sJ[k] = g[k] >= 0.0 ? 1 : -1;
    } else {
        int side = 0;
        const int ax = first_inside_neighbour(cls, q, J, N, n, d, side);
        for (int k = 0; k < d; k++) sJ[k] = (k == ax ? (double)side : 0.0) >= 0.0 ? 1 : -1;
    }
}

// Admissibility beyond validity: c_0 >= sum of |w_m| over the block's other
// GHOST nodes whose upwind signs differ from G's (every closed loop of ghost
// rows holding each other has such a coupling) plus half the sum over those
// oriented like G (one-way couplings); a Neumann row also needs c_0 > 0
__device__ bool block_dominant(const double *phi, const uint8_t *cls, int N, int n, int d, double h, const int I[3],
                               const int s[3], const int w[3], const double tau[3], const double nd[3], int bc) {
    double c0 = 0.0, off = 0.0;
    for (int m2 = 0; m2 < w[2]; m2++)
        for (int m1 = 0; m1 < w[1]; m1++)
            for (int m0 = 0; m0 < w[0]; m0++) {
                const int m[3] = {m0, m1, m2};
                const int J[3] = {I[0] - m0 * s[0], I[1] - m1 * s[1], I[2] - m2 * s[2]};
                const double wgt = row_weight(bc, w, tau, nd, m);
                const long long q = index_of(J, n, d);
                if (m0 == 0 && m1 == 0 && m2 == 0) {
                    c0 = wgt;
                } else if (cls[q] == C_GHOST) {
                    int sJ[3];
                    upwind_signs(phi, cls, N, n, d, h, J, q, sJ);
                    if (sJ[0] != s[0] || sJ[1] != s[1] || sJ[2] != s[2])
                        off += fabs(wgt);
                    else
                        off += 0.5 * fabs(wgt);
                }
            }
    if (bc == BCMG_BC_NEUMANN && !(c0 > 0.0)) return false;
    return c0 >= off;
}

__device__ double dtau_of(int d, double theta, int mode, double cnst) {
    if (mode == BCMG_DTAU_CONST) return cnst;
    double t = theta < 1.0 ? theta : 1.0;
    if (t < 0.0) t = 0.0;
    if (d == 1) return 1.0;
    double gmin = INFINITY, gmax = -INFINITY;
    for (int v = 0; v < d; v++) {
        const double p = v < d - 1 ? acosh(2.0 + v) : acosh(2.0 * d - 1.0);
        double g;
        if (mode == BCMG_DTAU_OPT_EXP) {
            g = exp(-p * t);
        } else {
            const double c0 = (1.0 - t) * (2.0 - t) / 2.0, c1 = t * (2.0 - t), c2 = t * (t - 1.0) / 2.0;
            g = fabs(c2 * exp(-2.0 * p) + c1 * exp(-p) + c0);
        }
        gmin = fmin(gmin, g);
        gmax = fmax(gmax, g);
    }
    return 2.0 / (gmin + gmax);
}

// First INSIDE axis neighbour of node p in the order -x, +x, -y, +y, -z, +z:
// returns its axis (or -1) and sets side = +1 when it is p - e_k, -1 when it
// is p + e_k.  Written as a chain of selects: an if / else-if pair that
// assigned the axis in both branches was compiled for gfx950 so that the
// else-if branch kept the old axis.
__device__ int first_inside_neighbour(const uint8_t *cls, long long p, const int I[3], int N, int n, int d,
                                      int &side) {
    int axis = -1, sd = 0;
    long long str = 1;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const bool lo = k < d && axis < 0 && I[k] > 0 && cls[p - str] == C_INSIDE;
        const bool hi = k < d && axis < 0 && !lo && I[k] < N && cls[p + str] == C_INSIDE;
        sd = lo ? 1 : (hi ? -1 : sd);
        axis = (lo || hi) ? k : axis;
        str *= n;
    }
    side = sd;
    return axis;
}

// dtau / h of a Neumann row (Prop. optN / opt3DN with eq. coeffN; the
// exponential form G0 = p e^{-p t} of Remark exptheta2D over p in
// [acosh 2, acosh(2d-1)], whose maximum lies at p = 1/t when that is inside;
// 1D: HUGE_VAL, capped below at the row's Gauss-Seidel step)
__device__ double dtau_neumann_of(int d, double theta, int mode, double cnst) {
    if (mode == BCMG_DTAU_CONST) return cnst;
    double t = theta < 1.0 ? theta : 1.0;
    if (t < 0.0) t = 0.0;
    if (d == 1) return HUGE_VAL;
    const double p_lo = acosh(2.0), p_hi = acosh(2.0 * d - 1.0);
    double gmin = INFINITY, gmax = -INFINITY;
    for (int v = 0; v <= d; v++) {
        double p;
        if (v < d) {
            p = v < d - 1 ? acosh(2.0 + v) : p_hi;
        } else {  // the interior maximum of p e^{-p t}
            if (mode != BCMG_DTAU_OPT_EXP || !(t > 0.0)) break;
            p = 1.0 / t;
            if (!(p > p_lo && p < p_hi)) break;
        }
        double g;
        if (mode == BCMG_DTAU_OPT_EXP) {
            g = p * exp(-p * t);
        } else {
            const double c0 = 1.5 - t, c1 = 2.0 * (t - 1.0), c2 = 0.5 - t;
            g = fabs(c2 * exp(-2.0 * p) + c1 * exp(-p) + c0);
        }
        gmin = fmin(gmin, g);
        gmax = fmax(gmax, g);
    }
    return 2.0 / (gmin + gmax);
}

// One ghost G: discrete normal, upwind signs, axis dominance, root eta in
// [0,1] of phi~(G - eta h n) = 0 (bracket at 1, 60 bisections), first
// admissible stencil widths (in the box, INSIDE/GHOST nodes only, and
// block_dominant), Q, tau and dtau(theta~) bounded by the row's Gauss-Seidel
// step 1/c_0, with theta~ the normal distance from G to the row's
// interpolation point.  Sec. 3.3 eqs. BCh, rel,
// DtauOptTheta, Remark exptheta2D.  Neumann rows (bc): the derivative
// coefficients gnd, blocks that may hold BOXDIR nodes, c_0 > 0, and with no
// admissible block the difference (u_G - u_J)/h towards the first INSIDE axis
// neighbour J (fb bit 1); dtau = h * dtau_neumann_of.
__global__ __launch_bounds__(128) void k_ghost_geometry(int d, int N, int level, double h, const double *phi, const uint8_t *cls,
                                 const int *gidx, int ng, int dtau_mode, double dtau_const, int bc, int *gcode,
                                 double *gtau, double *gdtau, double *geta, double *gn, double *gq, int *gfb,
                                 double *gnd) {
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= ng) return;
    const int n = N + 1;
    const long long p = gidx[gi];
    int I[3];
    coords(p, n, d, I);
    double g[3];
    grad_at(phi, n, d, h, I, p, g);
    double gnorm = 0.0;
    for (int k = 0; k < d; k++) gnorm += g[k] * g[k];
    gnorm = sqrt(gnorm);
    double nv[3] = {0.0, 0.0, 0.0}, key[3] = {0.0, 0.0, 0.0};
    if (gnorm > 0.0) {
        for (int k = 0; k < d; k++) {
            nv[k] = g[k] / gnorm;
            key[k] = fabs(g[k]);
        }
    } else {  // unit vector from the first INSIDE axis neighbour to G
        int side = 0;
        const int ax = first_inside_neighbour(cls, p, I, N, n, d, side);
        for (int k = 0; k < d; k++) nv[k] = k == ax ? (double)side : 0.0;
        for (int k = 0; k < d; k++) key[k] = fabs(nv[k]);
    }
    int s[3] = {1, 1, 1};
    for (int k = 0; k < d; k++) s[k] = (gnorm > 0.0 ? g[k] : nv[k]) >= 0.0 ? 1 : -1;
    int ord[3] = {0, 1, 2};
    for (int a = 1; a < d; a++)
        for (int b = a; b > 0 && key[ord[b - 1]] < key[ord[b]]; b--) {
            const int tmp = ord[b - 1];
            ord[b - 1] = ord[b];
            ord[b] = tmp;
        }
    int sp[3] = {s[0], s[1], s[2]};
    for (int k = 0; k < d; k++) {
        const int far = I[k] - 2 * s[k];
        if (far < 0 || far > N) sp[k] = -s[k];
    }
    const double phiG = phi[p];
    double pv[3][3][3];
    for (int m2 = 0; m2 < (d >= 3 ? 3 : 1); m2++)
        for (int m1 = 0; m1 < (d >= 2 ? 3 : 1); m1++)
            for (int m0 = 0; m0 < 3; m0++) {
                const int J[3] = {I[0] - m0 * sp[0], I[1] - m1 * sp[1], I[2] - m2 * sp[2]};
                pv[m2][m1][m0] = phi[index_of(J, n, d)];
            }
    double eta;
    int fb = 0;
    if (phiG == 0.0) {
        eta = 0.0;
    } else {
        double hi = -1.0;  // eta is sought in [0, 1]: bracket at eta = 1
        {
            double t[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < d; k++) t[k] = nv[k] * sp[k];
            if (phi_tilde_vals(pv, d, t) < 0.0) hi = 1.0;
        }
        if (hi > 0.0) {
            double lo = 0.0;
            for (int it = 0; it < 60; it++) {
                const double mid = 0.5 * (lo + hi);
                double t[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < d; k++) t[k] = mid * nv[k] * sp[k];
                if (phi_tilde_vals(pv, d, t) < 0.0)
                    hi = mid;
                else
                    lo = mid;
            }
            eta = 0.5 * (lo + hi);
        } else {
            eta = phiG / (h * gnorm);
            if (!(eta < 1.0)) eta = 1.0;
            fb = 1;
        }
    }
    const int cand3[7][3] = {{3, 3, 3}, {2, 2, 2}, {3, 3, 1}, {2, 2, 1}, {3, 1, 1}, {2, 1, 1}, {1, 1, 1}};
    const int cand2[5][3] = {{3, 3, 1}, {2, 2, 1}, {3, 1, 1}, {2, 1, 1}, {1, 1, 1}};
    const int cand1[3][3] = {{3, 1, 1}, {2, 1, 1}, {1, 1, 1}};
    const int ncand = d == 3 ? 7 : (d == 2 ? 5 : 3);
    double nd[3] = {0.0, 0.0, 0.0};
    if (bc == BCMG_BC_NEUMANN)
        for (int k = 0; k < d; k++) nd[k] = -(double)s[k] * nv[k] / h;
    int w[3] = {1, 1, 1};
    bool chosen = false;
    for (int c = 0; c < ncand; c++) {
        const int *cd = d == 3 ? cand3[c] : (d == 2 ? cand2[c] : cand1[c]);
        int wt[3] = {1, 1, 1};
        for (int r = 0; r < d; r++) wt[ord[r]] = cd[r];
        if (!block_valid(cls, n, d, I, s, wt, bc)) continue;
        double tt[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < d; k++) tt[k] = wt[k] >= 2 ? eta * fabs(nv[k]) : 0.0;
        if (!block_dominant(phi, cls, N, n, d, h, I, s, wt, tt, nd, bc)) continue;
        w[0] = wt[0];
        w[1] = wt[1];
        w[2] = wt[2];
        chosen = true;
        break;
    }
    int axis = -1;  // Neumann row with no admissible block: one-sided difference along this axis
    if (!chosen && bc == BCMG_BC_NEUMANN) {
        int side = 0;
        axis = first_inside_neighbour(cls, p, I, N, n, d, side);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            w[k] = k == axis ? 2 : 1;
            nd[k] = k == axis ? -1.0 / h : 0.0;
            s[k] = k == axis ? side : s[k];
        }
        fb |= 2;
    }
    int code = 0;
    double tq[3];
    for (int k = 0; k < 3; k++) {
        code |= (w[k] & 3) << (2 * k);
        if (s[k] < 0) code |= 1 << (6 + k);
        gn[3 * gi + k] = nv[k];
        const double xk = k < d ? -1.0 + I[k] * h : 0.0;
        gq[3 * gi + k] = k < d ? xk - eta * h * nv[k] : 0.0;
        tq[k] = (k < d && w[k] >= 2 && axis < 0) ? eta * fabs(nv[k]) : 0.0;
        gtau[3 * gi + k] = tq[k];
        if (gnd) gnd[3 * gi + k] = nd[k];
    }
    gcode[gi] = code;
    geta[gi] = eta;
    gfb[gi] = fb;
    // theta~: the distance along n from G to the point the row interpolates
    // at; eta for a full-width row, eta * (sum of n_k^2 over the kept axes)
    // for a row with width-1 axes (Q projected onto the span of the others)
    double theta = eta;
    if (axis < 0) {
        bool shortened = false;
        double nn2 = 0.0;
        for (int k = 0; k < d; k++) {
            if (w[k] >= 2)
                nn2 += nv[k] * nv[k];
            else
                shortened = true;
        }
        if (shortened) theta = eta * nn2;
    }
    double dt = bc == BCMG_BC_NEUMANN ? h * dtau_neumann_of(d, theta, dtau_mode, dtau_const)
                                      : dtau_of(d, theta, dtau_mode, dtau_const);
    if (dtau_mode != BCMG_DTAU_CONST) {  // at most the row's Gauss-Seidel step 1/c_0
        const int m0[3] = {0, 0, 0};
        const double c0 = row_weight(bc, w, tq, nd, m0);
        if (c0 > 0.0 && dt * c0 > 1.0) dt = 1.0 / c0;
    }
    gdtau[gi] = dt;
}

void launch_ghost_geometry(int d, int N, int level, double h, const double *phi, const uint8_t *cls, const int *gidx,
                           int ng, int dtau_mode, double dtau_const, int bc, int *gcode, double *gtau, double *gdtau,
                           double *geta, double *gn, double *gq, int *gfb, double *gnd, hipStream_t s) {
    if (ng <= 0) return;
    hipLaunchKernelGGL(k_ghost_geometry, dim3((ng + 127) / 128), dim3(128), 0, s, d, N, level, h, phi, cls, gidx, ng,
                       dtau_mode, dtau_const, bc, gcode, gtau, gdtau, geta, gn, gq, gfb, gnd);
}

// ----------------------------------------------------------- extension band
// OUTSIDE nodes within Chebyshev distance K of a ghost: the only nodes the
// K extension sweeps can make non-zero.
__global__ void k_band_mark(int d, int N, const uint8_t *cls, const int *gidx, int ng, int K, uint8_t *mark) {
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= ng) return;
    const int n = N + 1;
    int I[3];
    coords(gidx[gi], n, d, I);
    const int r2 = d >= 3 ? K : 0, r1 = d >= 2 ? K : 0;
    for (int m2 = -r2; m2 <= r2; m2++)
        for (int m1 = -r1; m1 <= r1; m1++)
            for (int m0 = -K; m0 <= K; m0++) {
                const int J[3] = {I[0] + m0, I[1] + m1, I[2] + m2};
                if (!in_box(J, N, d)) continue;
                const long long q = index_of(J, n, d);
                if (cls[q] == C_OUTSIDE) mark[q] = 1;
            }
}

void launch_band_mark(int d, int N, const uint8_t *cls, const int *gidx, int ng, int K, uint8_t *mark,
                      hipStream_t s) {
    if (ng <= 0) return;
    hipLaunchKernelGGL(k_band_mark, dim3((ng + 127) / 128), dim3(128), 0, s, d, N, cls, gidx, ng, K, mark);
}

__device__ int band_find(const int *bidx, int nb, int q) {
    int lo = 0, hi = nb - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = bidx[mid];
        if (v == q) return mid;
        if (v < q)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

// Per band node X: its upwind neighbours X - s_k e_k with weights |n_k|:
// reference >= 0: band entry; -1 - q: a GHOST node q (read from the field);
// kRefZero: value 0 (BOXDIR, or OUTSIDE beyond the band), weight kept;
// out-of-box terms get weight 0.  kRefFallback when the weights sum to 0.
__global__ void k_band_records(int d, int N, double h, const double *phi, const uint8_t *cls, const int *bidx, int nb,
                               int *bref, double *bw) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int n = N + 1;
    const long long p = bidx[b];
    int I[3];
    coords(p, n, d, I);
    double g[3];
    grad_at(phi, n, d, h, I, p, g);
    double gnorm = 0.0;
    for (int k = 0; k < d; k++) gnorm += g[k] * g[k];
    gnorm = sqrt(gnorm);
    double den = 0.0;
    for (int k = 0; k < 3; k++) {
        bref[3 * b + k] = kRefZero;
        bw[3 * b + k] = 0.0;
    }
    if (gnorm > 0.0) {
        for (int k = 0; k < d; k++) {
            const double nk = g[k] / gnorm;
            const int sk = g[k] >= 0.0 ? 1 : -1;
            int J[3] = {I[0], I[1], I[2]};
            J[k] -= sk;
            if (!in_box(J, N, d)) continue;
            const long long q = index_of(J, n, d);
            const uint8_t c = cls[q];
            int ref = kRefZero;
            if (c == C_GHOST) {
                ref = -1 - (int)q;
            } else if (c == C_OUTSIDE) {
                const int bi = band_find(bidx, nb, (int)q);
                ref = bi >= 0 ? bi : kRefZero;
            }
            bref[3 * b + k] = ref;
            bw[3 * b + k] = fabs(nk);
            den += fabs(nk);
        }
    }
    if (!(den > 0.0)) bref[3 * b] = kRefFallback;
}

void launch_band_records(int d, int N, double h, const double *phi, const uint8_t *cls, const int *bidx, int nb,
                         int *bref, double *bw, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_band_records, dim3((nb + 127) / 128), dim3(128), 0, s, d, N, h, phi, cls, bidx, nb, bref, bw);
}

// ------------------------------------------------- extension and restriction rows
// The normal extension (K upwind Jacobi sweeps from zero, Sec. 3.3 transfer
// operators) is linear in the ghost values, so its result on the band is a
// fixed sparse map v(X) = sum_j c_j u(G_j).  The rows are built sweep by sweep
// (count, prefix sum, write): the row of sweep j at a band node combines, with
// the weights |n_k| / sum_k |n_k|, the ghosts it references directly and the
// rows of sweep j-1 of the band nodes it references; a node whose weights sum
// to zero takes the mean of the GHOST nodes of its 3^d box.  Rows are sorted
// by ghost-list index without repeats.

constexpr int kMaxSrc = 27;

__device__ int find_sorted(const int *a, int n, int q) {
    int lo = 0, hi = n - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = a[mid];
        if (v == q) return mid;
        if (v < q)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

// Sources of a merged row, one fixed slot each (slots of a 3^d box, or
// the upwind references), so that every loop over them unrolls into
// registers: a sorted row (ip, cp, len) or a single entry `one` with
// coefficient 1; each with weight w.
template <int NS>
struct Srcs {
    const int *ip[NS];
    const double *cp[NS];
    int len[NS];
    int one[NS];
    double w[NS];
};

template <int NS>
__device__ __forceinline__ void srcs_clear(Srcs<NS> &S) {
#pragma unroll
    for (int t = 0; t < NS; t++) {
        S.ip[t] = nullptr;
        S.cp[t] = nullptr;
        S.len[t] = 0;
        S.one[t] = -1;
        S.w[t] = 0.0;
    }
}

// Merge of the sorted source rows: returns the number of distinct indices;
// writes them (mapped through map when given) and their coefficients
// sum_t w_t c_t (in slot order) when oidx is not null.
template <int NS>
__device__ int merge_srcs(const Srcs<NS> &S, const int *map, int *oidx, double *ocf) {
    int pos[NS], head[NS];
#pragma unroll
    for (int t = 0; t < NS; t++) {
        pos[t] = 0;
        head[t] = S.len[t] > 0 ? (S.one[t] >= 0 ? S.one[t] : S.ip[t][0]) : INT32_MAX;
    }
    int n = 0;
    while (true) {
        int m = INT32_MAX;
#pragma unroll
        for (int t = 0; t < NS; t++) m = head[t] < m ? head[t] : m;
        if (m == INT32_MAX) break;
        double c = 0.0;
#pragma unroll
        for (int t = 0; t < NS; t++)
            if (head[t] == m) {
                c += S.w[t] * (S.one[t] >= 0 ? 1.0 : S.cp[t][pos[t]]);
                pos[t]++;
                head[t] = (S.one[t] < 0 && pos[t] < S.len[t]) ? S.ip[t][pos[t]] : INT32_MAX;
            }
        if (oidx) {
            oidx[n] = map ? map[m] : m;
            ocf[n] = c;
        }
        n++;
    }
    return n;
}

// Sweep j (1..K) of the extension rows of every band node b.  Count mode
// when optr is null (counts[b] = row length), else write mode.
__global__ __launch_bounds__(128) void k_erow(int d, int N, const uint8_t *cls, const int *gidx, int ng, const int *bidx, int nb,
                       const int *bref, const double *bw, int j, const int *pptr, const int *pidx,
                       const double *pcf, const int *optr, int *counts, int *oidx, double *ocf) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    int n;
    int *oi = optr ? oidx + optr[b] : nullptr;
    double *oc = optr ? ocf + optr[b] : nullptr;
    if (bref[3 * b] == kRefFallback) {
        // the mean of the GHOST nodes of the 3^d box, one slot per box position
        Srcs<27> S;
        srcs_clear(S);
        const int nn1 = N + 1;
        int I[3];
        coords(bidx[b], nn1, d, I);
        int cnt = 0;
#pragma unroll
        for (int m2 = -1; m2 <= 1; m2++)
#pragma unroll
            for (int m1 = -1; m1 <= 1; m1++)
#pragma unroll
                for (int m0 = -1; m0 <= 1; m0++) {
                    const int t = (m2 + 1) * 9 + (m1 + 1) * 3 + (m0 + 1);
                    if ((d < 3 && m2 != 0) || (d < 2 && m1 != 0)) continue;
                    const int J[3] = {I[0] + m0, I[1] + m1, I[2] + m2};
                    if (!in_box(J, N, d)) continue;
                    const long long q = index_of(J, nn1, d);
                    if (cls[q] != C_GHOST) continue;
                    S.one[t] = find_sorted(gidx, ng, (int)q);
                    S.len[t] = 1;
                    cnt++;
                }
#pragma unroll
        for (int t = 0; t < 27; t++) S.w[t] = S.len[t] ? 1.0 / cnt : 0.0;
        n = merge_srcs(S, nullptr, oi, oc);
    } else {
        Srcs<3> S;
        srcs_clear(S);
        double den = 0.0;
        for (int k = 0; k < d; k++) den += bw[3 * b + k];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            if (k >= d) continue;
            const int ref = bref[3 * b + k];
            if (ref == kRefZero) continue;
            if (ref >= 0) {
                if (j < 2) continue;  // v^0 = 0 on the band
                S.ip[k] = pidx + pptr[ref];
                S.cp[k] = pcf + pptr[ref];
                S.len[k] = pptr[ref + 1] - pptr[ref];
            } else {
                S.one[k] = find_sorted(gidx, ng, -1 - ref);
                S.len[k] = 1;
            }
            S.w[k] = bw[3 * b + k] / den;
        }
        n = merge_srcs(S, nullptr, oi, oc);
    }
    if (!optr) counts[b] = n;
}

// Restriction rows of the ghosts of a coarse level (Sec. 3.3: full weighting
// over the non-INSIDE, non-BOXDIR nodes of the extended fine residual,
// renormalised unless the fine 3^d box is complete and has no INSIDE node;
// or the plain mean).  Fine OUTSIDE nodes contribute through their extension
// rows; the result is a row over fine ghost nodes (node indices, ascending).
__global__ __launch_bounds__(128) void k_rrow(int d, int Nc, const int *gidx_c, int ngc, int Nf, const uint8_t *cls_f, const int *gidx_f,
                       int ngf, const int *bidx_f, int nbf, const int *eptr_f, const int *eidx_f, const double *ecf_f,
                       int restrict_mode, const int *optr, int *counts, int *oidx, double *ocf) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngc) return;
    const int nc = Nc + 1, nf = Nf + 1;
    int P[3];
    coords(gidx_c[g], nc, d, P);
    Srcs<27> S;
    srcs_clear(S);
    bool all_ok = true;
    double selw = 0.0;
    int cnt = 0;  // admissible nodes of the box (beyond-band OUTSIDE nodes included)
#pragma unroll
    for (int m2 = -1; m2 <= 1; m2++)
#pragma unroll
        for (int m1 = -1; m1 <= 1; m1++)
#pragma unroll
            for (int m0 = -1; m0 <= 1; m0++) {
                const int t = (m2 + 1) * 9 + (m1 + 1) * 3 + (m0 + 1);
                if ((d < 3 && m2 != 0) || (d < 2 && m1 != 0)) continue;
                const int J[3] = {2 * P[0] + m0, 2 * P[1] + m1, 2 * P[2] + m2};
                if (!in_box(J, Nf, d)) {
                    all_ok = false;
                    continue;
                }
                double wgt = m0 == 0 ? 0.5 : 0.25;
                if (d >= 2) wgt *= m1 == 0 ? 0.5 : 0.25;
                if (d >= 3) wgt *= m2 == 0 ? 0.5 : 0.25;
                const long long q = index_of(J, nf, d);
                const uint8_t c = cls_f[q];
                if (c == C_INSIDE) {
                    all_ok = false;
                    continue;
                }
                if (c == C_BOXDIR) continue;
                selw += wgt;
                cnt++;
                if (c == C_GHOST) {
                    S.one[t] = find_sorted(gidx_f, ngf, (int)q);
                    S.len[t] = 1;
                } else {
                    const int bb = find_sorted(bidx_f, nbf, (int)q);
                    if (bb < 0) continue;  // beyond the band: extended value 0
                    S.ip[t] = eidx_f + eptr_f[bb];
                    S.cp[t] = ecf_f + eptr_f[bb];
                    S.len[t] = eptr_f[bb + 1] - eptr_f[bb];
                }
                S.w[t] = wgt;
            }
    if (!all_ok) {
#pragma unroll
        for (int t = 0; t < 27; t++) {
            if (restrict_mode == BCMG_RESTRICT_PLAIN_MEAN)
                S.w[t] = S.len[t] ? 1.0 / cnt : 0.0;
            else
                S.w[t] = S.w[t] / selw;
        }
    }
    if (!optr) {
        counts[g] = merge_srcs(S, gidx_f, nullptr, nullptr);
        return;
    }
    merge_srcs(S, gidx_f, oidx + optr[g], ocf + optr[g]);
}

void launch_erow(int d, int N, const uint8_t *cls, const int *gidx, int ng, const int *bidx, int nb, const int *bref,
                 const double *bw, int j, const int *pptr, const int *pidx, const double *pcf, const int *optr,
                 int *counts, int *oidx, double *ocf, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_erow, dim3((nb + 127) / 128), dim3(128), 0, s, d, N, cls, gidx, ng, bidx, nb, bref, bw, j,
                       pptr, pidx, pcf, optr, counts, oidx, ocf);
}

void launch_rrow(int d, int Nc, const int *gidx_c, int ngc, int Nf, const uint8_t *cls_f, const int *gidx_f, int ngf,
                 const int *bidx_f, int nbf, const int *eptr_f, const int *eidx_f, const double *ecf_f,
                 int restrict_mode, const int *optr, int *counts, int *oidx, double *ocf, hipStream_t s) {
    if (ngc <= 0) return;
    hipLaunchKernelGGL(k_rrow, dim3((ngc + 127) / 128), dim3(128), 0, s, d, Nc, gidx_c, ngc, Nf, cls_f, gidx_f, ngf,
                       bidx_f, nbf, eptr_f, eidx_f, ecf_f, restrict_mode, optr, counts, oidx, ocf);
}

// Exclusive prefix sum of n counts into ptr[0..n-1], total into ptr[n].
hipError_t launch_scan(const int *counts, int n, int *ptr, hipStream_t s) { return scan_exclusive(counts, n, ptr, ptr + n, s); }

// Coarse OUTSIDE nodes that the prolongation reads: the corners of the
// coarse cells holding fine INSIDE / GHOST nodes.  Only these band nodes
// need the extended coarse error during a cycle.
__global__ void k_need_mark(int d, int Nf, const uint8_t *cls_f, const uint8_t *cls_c, uint8_t *mark_c,
                            long long nnf) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnf) return;
    const uint8_t c = cls_f[p];
    if (c != C_INSIDE && c != C_GHOST) return;
    const int nf = Nf + 1, nc = Nf / 2 + 1;
    int I[3];
    coords(p, nf, d, I);
    int B[3] = {0, 0, 0}, h[3] = {0, 0, 0};
    for (int k = 0; k < d; k++) {
        h[k] = I[k] & 1;
        B[k] = (I[k] - h[k]) / 2;
    }
    for (int m2 = 0; m2 <= h[2]; m2++)
        for (int m1 = 0; m1 <= h[1]; m1++)
            for (int m0 = 0; m0 <= h[0]; m0++) {
                const int J[3] = {B[0] + m0, B[1] + m1, B[2] + m2};
                const long long q = index_of(J, nc, d);
                if (cls_c[q] == C_OUTSIDE) mark_c[q] = 1;
            }
}

// flag[b] = mark[bidx[b]] over the band entries
__global__ void k_need_flags(const int *bidx, int nb, const uint8_t *mark, uint8_t *flag) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) flag[b] = mark[bidx[b]];
}

void launch_need_mark(int d, int Nf, const uint8_t *cls_f, const uint8_t *cls_c, uint8_t *mark_c, long long nnf,
                      hipStream_t s) {
    if (nnf <= 0) return;
    hipLaunchKernelGGL(k_need_mark, dim3((unsigned)((nnf + 255) / 256)), dim3(256), 0, s, d, Nf, cls_f, cls_c,
                       mark_c, nnf);
}

void launch_need_flags(const int *bidx, int nb, const uint8_t *mark, uint8_t *flag, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_need_flags, dim3((nb + 255) / 256), dim3(256), 0, s, bidx, nb, mark, flag);
}

// x-extent of the INSIDE/GHOST nodes of each grid row (-1 if none).
// Per row: first and last INSIDE or GHOST node (-1 if none), and the first
// and last INSIDE node when the row's INSIDE nodes are consecutive (ib = -1
// if they are not, or there are none).
__global__ void k_row_extent(int d, int n, const uint8_t *cls, int *xmin, int *xmax, int *ia, int *ib,
                             long long rows) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const uint8_t *row = cls + r * n;
    int lo = -1, hi = -1, ilo = -1, ihi = -1, icount = 0;
    for (int x = 0; x < n; x++) {
        const uint8_t c = row[x];
        if (c == C_INSIDE || c == C_GHOST) {
            if (lo < 0) lo = x;
            hi = x;
        }
        if (c == C_INSIDE) {
            if (ilo < 0) ilo = x;
            ihi = x;
            icount++;
        }
    }
    xmin[r] = lo;
    xmax[r] = hi;
    ia[r] = ilo;
    ib[r] = icount > 0 && icount == ihi - ilo + 1 ? ihi : -1;
}

void launch_row_extent(int d, int n, const uint8_t *cls, int *xmin, int *xmax, int *ia, int *ib, hipStream_t s) {
    long long rows = 1;
    for (int k = 1; k < d; k++) rows *= n;
    hipLaunchKernelGGL(k_row_extent, dim3((unsigned)((rows + 127) / 128)), dim3(128), 0, s, d, n, cls, xmin, xmax, ia,
                       ib, rows);
}

// ----------------------------------------------------- coarsest-level inverse
// One workgroup: unknowns INSIDE (ascending) then GHOST (ascending), dense
// matrix of the interior and ghost rows, Gauss-Jordan with partial pivoting
// on [A | I].  info[0] = unknowns, info[1] = 1 if a pivot falls below
// 1e-14 max|A| (singular: the cycle then smooths instead).
__global__ void k_coarse_setup(int d, int N, double h, const uint8_t *cls, const int *gidx, int ng, const int *gcode,
                               const double *gtau, int bc, const double *gnd, double reaction, double *work,
                               double *ainv, int *cmap, int *info) {
    const int n = N + 1;
    int nn = 1;
    for (int k = 0; k < d; k++) nn *= n;
    __shared__ int pos[kCoarseMax];
    __shared__ int s_nc, s_piv, s_sing;
    __shared__ double s_amax;
    const int t = threadIdx.x;
    if (t == 0) {
        int c = 0;
        for (int p = 0; p < nn; p++) {
            pos[p] = -1;
            if (cls[p] == C_INSIDE) {
                pos[p] = c;
                cmap[c++] = p;
            }
        }
        for (int g = 0; g < ng; g++) {
            pos[gidx[g]] = c;
            cmap[c++] = gidx[g];
        }
        s_nc = c;
        s_sing = 0;
    }
    __syncthreads();
    const int nc = s_nc;
    const int W = 2 * nc;
    for (int i = t; i < nc * W; i += blockDim.x) {
        const int r = i / W, c = i % W;
        work[i] = (c >= nc && c - nc == r) ? 1.0 : 0.0;
    }
    __syncthreads();
    const double ih2 = 1.0 / (h * h);
    if (t == 0) {
        for (int row = 0; row < nc; row++) {
            const int p = cmap[row];
            if (cls[p] == C_INSIDE) {
                work[row * W + row] += 2.0 * d * ih2 + reaction;
                int str = 1;
                for (int k = 0; k < d; k++) {
                    if (pos[p - str] >= 0) work[row * W + pos[p - str]] -= ih2;
                    if (pos[p + str] >= 0) work[row * W + pos[p + str]] -= ih2;
                    str *= n;
                }
            }
        }
        for (int g = 0; g < ng; g++) {
            const int row = pos[gidx[g]];
            int I[3];
            coords(gidx[g], n, d, I);
            const int code = gcode[g];
            int w[3], s[3];
            double tau[3], nd[3];
            for (int k = 0; k < 3; k++) {
                w[k] = k < d ? code_w(code, k) : 1;
                s[k] = code_s(code, k);
                tau[k] = k < d ? gtau[3 * g + k] : 0.0;
                nd[k] = bc == BCMG_BC_NEUMANN ? gnd[3 * g + k] : 0.0;
            }
            for (int m2 = 0; m2 < w[2]; m2++)
                for (int m1 = 0; m1 < w[1]; m1++)
                    for (int m0 = 0; m0 < w[0]; m0++) {
                        const int m[3] = {m0, m1, m2};
                        const int J[3] = {I[0] - m0 * s[0], I[1] - m1 * s[1], I[2] - m2 * s[2]};
                        const int q = pos[index_of(J, n, d)];
                        // BOXDIR nodes of Neumann blocks carry 0 on coarse levels
                        if (q >= 0) work[row * W + q] += row_weight(bc, w, tau, nd, m);
                    }
        }
        double amax = 0.0;
        for (int r = 0; r < nc; r++)
            for (int c = 0; c < nc; c++) amax = fmax(amax, fabs(work[r * W + c]));
        s_amax = amax;
    }
    __syncthreads();
    for (int k = 0; k < nc; k++) {
        if (t == 0) {
            int pr = k;
            for (int i = k + 1; i < nc; i++)
                if (fabs(work[i * W + k]) > fabs(work[pr * W + k])) pr = i;
            s_piv = pr;
            if (fabs(work[pr * W + k]) < 1e-14 * s_amax) s_sing = 1;
        }
        __syncthreads();
        if (s_sing) break;
        const int pr = s_piv;
        if (pr != k)
            for (int c = t; c < W; c += blockDim.x) {
                const double tmp = work[k * W + c];
                work[k * W + c] = work[pr * W + c];
                work[pr * W + c] = tmp;
            }
        __syncthreads();
        const double piv = work[k * W + k];
        __syncthreads();
        for (int c = t; c < W; c += blockDim.x) work[k * W + c] /= piv;
        __syncthreads();
        for (int i = t; i < nc * W; i += blockDim.x) {
            const int r = i / W, c = i % W;
            if (r == k || c == k) continue;
            work[i] -= work[r * W + k] * work[k * W + c];
        }
        __syncthreads();
        for (int r = t; r < nc; r += blockDim.x)
            if (r != k) work[r * W + k] = 0.0;
        __syncthreads();
    }
    for (int i = t; i < nc * nc; i += blockDim.x) ainv[i] = work[(i / nc) * W + nc + (i % nc)];
    if (t == 0) {
        info[0] = nc;
        info[1] = s_sing;
    }
}

void launch_coarse_setup(int d, int N, double h, const uint8_t *cls, const int *gidx, int ng, const int *gcode,
                         const double *gtau, int bc, const double *gnd, double reaction, double *work, double *ainv,
                         int *cmap, int *info, hipStream_t s) {
    hipLaunchKernelGGL(k_coarse_setup, dim3(1), dim3(kBlock), 0, s, d, N, h, cls, gidx, ng, gcode, gtau, bc, gnd,
                       reaction, work, ainv, cmap, info);
}

// ------------------------------------------------------------- data movement
__global__ void k_set_rhs(long long nn, const uint8_t *cls, const double *f, double *rhs) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nn) return;
    rhs[p] = (f && cls[p] == C_INSIDE) ? f[p] : 0.0;
}

void launch_set_rhs(long long nn, const uint8_t *cls, const double *f, double *rhs, hipStream_t s) {
    hipLaunchKernelGGL(k_set_rhs, dim3((unsigned)((nn + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, nn, cls, f, rhs);
}

__global__ void k_scatter_ghosts(const int *gidx, int ng, const double *gq, double *rhs) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ng) rhs[gidx[g]] = gq[g];
}

void launch_scatter_ghosts(const int *gidx, int ng, const double *gq, double *rhs, hipStream_t s) {
    if (ng <= 0) return;
    hipLaunchKernelGGL(k_scatter_ghosts, dim3((ng + kBlock - 1) / kBlock), dim3(kBlock), 0, s, gidx, ng, gq, rhs);
}

__global__ void k_fill_boundary(long long nn, const uint8_t *cls, const double *gbox, double *u) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nn) return;
    if (cls[p] == C_BOXDIR) u[p] = gbox ? gbox[p] : 0.0;
}

void launch_fill_boundary(long long nn, const uint8_t *cls, const double *gbox, double *u, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_boundary, dim3((unsigned)((nn + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, nn, cls,
                       gbox, u);
}

}  // namespace bcmg
