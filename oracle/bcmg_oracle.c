/*
 * bcmg_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * Plain, slow, FP64 CPU reference of the ghost-point geometric multigrid of
 * Coco, Mazza & Semplice, "A ghost-point smoothing strategy for geometric
 * multigrid on curved boundaries" (arXiv 2207.14208).  Only the test-suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library: every step
 * below is written from the paper (section / equation cited per function)
 * plus the readings listed in the design notes where the paper is silent.
 *
 * Every loop runs over the whole node box in lexicographic order (x fastest),
 * exactly as the definitions read; nothing is blocked, fused or reordered.
 *
 * Node classes (Sec. 3.3 "Non-rectangular domains", partition of D_h):
 *   OUTSIDE  inactive node (I_h)
 *   INSIDE   phi < 0 and not on a face of the box (Omega_h)
 *   GHOST    not INSIDE, phi >= 0, with an INSIDE axis neighbour (Gamma_h)
 *   BOXDIR   phi < 0 on a face of the box: eliminated Dirichlet node
 *            (Sec. 3, eq. (mainProblem2D), value g_B)
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_OUTSIDE 0
#define OR_INSIDE 1
#define OR_GHOST 2
#define OR_BOXDIR 3

#define OR_DTAU_OPT_EXP 0
#define OR_DTAU_OPT_POLY 1
#define OR_DTAU_CONST 2

#define OR_RESTRICT_RENORM_FW 0
#define OR_RESTRICT_PLAIN_MEAN 1

#define OR_SMOOTH_RB 0
#define OR_SMOOTH_LEX 1
#define OR_SMOOTH_JAC 2

#define OR_CYCLE_V 0
#define OR_CYCLE_TGCS 1
#define OR_CYCLE_W 2

#define OR_BC_DIRICHLET 0
#define OR_BC_NEUMANN 1

#define OR_MAXLEV 16

typedef struct {
    int nu1, nu2;        /* pre- and post-smoothing steps (Sec. 2.1) */
    int coarsest_N;      /* intervals per axis on the coarsest grid */
    int max_cycles;
    int dtau_mode;       /* OPT_EXP (Remark exptheta2D), OPT_POLY (eq. dtauoptLFA), CONST */
    double dtau_const;
    int ext_iters;       /* K: sweeps of the normal extension */
    int restrict_mode;   /* RENORM_FW or PLAIN_MEAN */
    int smoother;        /* RB (red-black GS), LEX (GS-LEX) or JAC (weighted Jacobi) for the interior */
    int cycle;           /* V-cycle, two-grid correction scheme or W-cycle */
    int bc;              /* condition on Gamma: DIRICHLET (B u = u) or NEUMANN (B u = grad u . n), Sec. 3.3 */
    double reaction;     /* c >= 0 in c u - Laplace u = f (c = 1: the reaction-diffusion tests of Sec. 3.3 / 4.2) */
    int ghost_dominance; /* 1: stencil widths must pass or_block_dominant; 0: validity only (test mode) */
} or_options;

typedef struct {
    int d, N, n;         /* dimension, intervals, nodes per axis n = N+1 */
    long nn;             /* n^d */
    long st[3];          /* index strides, 0 beyond d */
    double h;
    double *phi;
    unsigned char *cls;
    long ni, ng;
    long *gidx;          /* ghost node indices, ascending */
    int *gw;             /* [ng][3] stencil widths, 1 beyond d */
    int *gs;             /* [ng][3] upwind signs s_k */
    int *gfb;            /* 1 if the root search fell back to the first-order distance */
    double *geta;        /* eta = theta~ */
    double *gn;          /* [ng][3] unit normal */
    double *gq;          /* [ng][3] projection Q */
    double *gtau;        /* [ng][3] local coordinates of Q in the stencil */
    double *gdtau;       /* fictitious time step */
    double *gnd;         /* [ng][3] Neumann rows: coefficient of d/dt_k of the interpolant (t_k local) */
    int bc;              /* boundary row type of every ghost (OR_BC_*) */
    double reaction;     /* c of the interior row */
    double *u, *rhs, *r, *e; /* work arrays (coarse levels own u and rhs) */
} or_level;

typedef struct {
    int d, L;            /* levels 0..L-1, level L-1 is the coarsest */
    or_options opt;
    or_level lev[OR_MAXLEV];
    /* coarsest-level dense LU (partial pivoting) */
    long nc;             /* unknowns on the coarsest level */
    long *cmap;          /* unknown -> node index (INSIDE ascending, then GHOST ascending) */
    double *lu;
    long *piv;
    int coarse_singular;
    long coarse_fallbacks;
} or_problem;

/* ------------------------------------------------------------------------- */
/* small helpers                                                              */

static void or_coords(const or_level *L, long p, int I[3]) {
    I[0] = I[1] = I[2] = 0;
    for (int k = 0; k < L->d; k++) {
        I[k] = (int)(p % L->n);
        p /= L->n;
    }
}

static long or_index(const or_level *L, const int I[3]) {
    long p = 0;
    for (int k = L->d - 1; k >= 0; k--) p = p * L->n + I[k];
    return p;
}

static int or_in_box(const or_level *L, const int I[3]) {
    for (int k = 0; k < L->d; k++)
        if (I[k] < 0 || I[k] > L->N) return 0;
    return 1;
}

static int or_on_face(const or_level *L, const int I[3]) {
    for (int k = 0; k < L->d; k++)
        if (I[k] == 0 || I[k] == L->N) return 1;
    return 0;
}

double or_version(void) { return 1.0; }

void or_default_options(or_options *o) {
    o->nu1 = 2;
    o->nu2 = 1;
    o->coarsest_N = 4;
    o->max_cycles = 100;
    o->dtau_mode = OR_DTAU_OPT_EXP;
    o->dtau_const = 1.0;
    o->ext_iters = 4;
    o->restrict_mode = OR_RESTRICT_RENORM_FW;
    o->smoother = OR_SMOOTH_RB;
    o->cycle = OR_CYCLE_V;
    o->bc = OR_BC_DIRICHLET;
    o->reaction = 0.0;
    o->ghost_dominance = 1;
}

/* ------------------------------------------------------------------------- */
/* Fictitious time step.                                                      */
/* Coefficients of the quadratic Dirichlet boundary row, eq. (coeff) / (BC1D) */
static void or_coeff(double t, double c[3]) {
    c[0] = (1.0 - t) * (2.0 - t) / 2.0; /* c_0    */
    c[1] = t * (2.0 - t);               /* c_{-1} */
    c[2] = t * (t - 1.0) / 2.0;         /* c_{-2} */
}

/*
 * Delta tau as a function of theta~ (eq. DtauOptTheta).
 *  POLY: Prop. opt (2D) / Prop. opt3D (3D) / the d-dimensional remark:
 *        2 / (min_V |G0(V)| + max_V |G0(V)|), G0 = sum_r c_{-r} e^{-r p(V)},
 *        vertices V = A_1..A_d with p(A_i) = acosh(1+i) (i<d), p(A_d) = acosh(2d-1).
 *  EXP:  Remark exptheta2D: G0 = exp(-p theta); G0 is monotone in p so the
 *        extremes are at p = acosh(2) and p = acosh(2d-1).
 *  theta is clamped to [0,1] (the analysis assumes 0 <= theta < 1, Sec. 2).
 *  d = 1: p = acosh(1) = 0 and every form gives 1.
 */
double or_dtau(int d, double theta, int mode, double dtau_const) {
    if (mode == OR_DTAU_CONST) return dtau_const;
    double t = theta < 1.0 ? theta : 1.0;
    if (t < 0.0) t = 0.0;
    if (d == 1) return 1.0;
    double pv[4];
    int nv = 0;
    for (int i = 1; i < d; i++) pv[nv++] = acosh(1.0 + i);
    pv[nv++] = acosh(2.0 * d - 1.0);
    double gmin = INFINITY, gmax = -INFINITY;
    for (int v = 0; v < nv; v++) {
        double g;
        if (mode == OR_DTAU_OPT_EXP) {
            g = exp(-pv[v] * t);
        } else {
            double c[3];
            or_coeff(t, c);
            g = fabs(c[2] * exp(-2.0 * pv[v]) + c[1] * exp(-pv[v]) + c[0]);
        }
        if (g < gmin) gmin = g;
        if (g > gmax) gmax = g;
    }
    return 2.0 / (gmin + gmax);
}

/* Coefficients of the quadratic Neumann boundary row in units of 1/h,
 * eq. (coeffN): c_0, c_{-1}, c_{-2}. */
static void or_coeff_n(double t, double c[3]) {
    c[0] = 1.5 - t;
    c[1] = 2.0 * (t - 1.0);
    c[2] = 0.5 - t;
}

/*
 * Delta tau / h for Neumann rows as a function of theta~ (eq. DtauOptTheta
 * with Prop. optN in 2D and Prop. opt3DN in 3D); the caller multiplies by h.
 *  POLY:  2 / (min G0 + max G0), G0 = sum_r c_{-r} e^{-r p} with the
 *         coefficients of eq. (coeffN), over the same vertices as the
 *         Dirichlet form.  G0 is monotone in p (Lemma fnostatN) and positive
 *         (Lemma G0posN), so the vertices give the extremes.
 *  EXP:   Remark exptheta2D: G0 = p exp(-p theta) over p in
 *         [acosh(2), acosh(2d-1)].  This G0 is not monotone in p: its maximum
 *         over the interval is at p = 1/theta when that point lies inside,
 *         its minimum at an end.
 *  CONST: dtau_const (the constant is given in units of h).
 *  d = 1: p = 0 makes both optimal forms vanish; the ghost row is then
 *         relaxed by its own Gauss-Seidel step (returns HUGE_VAL, which the
 *         caller caps at 1/c_0).
 */
double or_dtau_neumann(int d, double theta, int mode, double dtau_const) {
    if (mode == OR_DTAU_CONST) return dtau_const;
    double t = theta < 1.0 ? theta : 1.0;
    if (t < 0.0) t = 0.0;
    if (d == 1) return HUGE_VAL;
    double pv[5];
    int nv = 0;
    for (int i = 1; i < d; i++) pv[nv++] = acosh(1.0 + i);
    pv[nv++] = acosh(2.0 * d - 1.0);
    if (mode == OR_DTAU_OPT_EXP && t > 0.0) {
        double pstar = 1.0 / t;
        if (pstar > pv[0] && pstar < pv[nv - 1]) pv[nv++] = pstar;
    }
    double gmin = INFINITY, gmax = -INFINITY;
    for (int v = 0; v < nv; v++) {
        double g;
        if (mode == OR_DTAU_OPT_EXP) {
            g = pv[v] * exp(-pv[v] * t);
        } else {
            double c[3];
            or_coeff_n(t, c);
            g = fabs(c[2] * exp(-2.0 * pv[v]) + c[1] * exp(-pv[v]) + c[0]);
        }
        if (g < gmin) gmin = g;
        if (g > gmax) gmax = g;
    }
    return 2.0 / (gmin + gmax);
}

/* ------------------------------------------------------------------------- */
/* Classification (Sec. 3.3: D_h = Omega_h U Gamma_h U I_h; Sec. 3 eliminated */
/* Dirichlet nodes on the box faces).                                         */
void or_classify(int d, int N, const double *phi, unsigned char *cls) {
    or_level L;
    memset(&L, 0, sizeof L);
    L.d = d;
    L.N = N;
    L.n = N + 1;
    L.nn = 1;
    for (int k = 0; k < d; k++) L.nn *= L.n;
    int I[3];
    for (long p = 0; p < L.nn; p++) {
        or_coords(&L, p, I);
        if (phi[p] < 0.0)
            cls[p] = or_on_face(&L, I) ? OR_BOXDIR : OR_INSIDE;
        else
            cls[p] = OR_OUTSIDE;
    }
    for (long p = 0; p < L.nn; p++) {
        if (cls[p] != OR_OUTSIDE) continue;
        or_coords(&L, p, I);
        int ghost = 0;
        for (int k = 0; k < d && !ghost; k++) {
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                int J[3] = {I[0], I[1], I[2]};
                J[k] += sgn;
                if (!or_in_box(&L, J)) continue;
                if (cls[or_index(&L, J)] == OR_INSIDE) ghost = 1;
            }
        }
        if (ghost) cls[p] = OR_GHOST;
    }
}

/* Discrete gradient of phi at a node: central differences, one-sided on a
 * box face (Sec. 3.3: the normal is a finite-difference approximation of
 * grad phi / |grad phi| centred at the ghost point). */
static void or_grad(const or_level *L, const int I[3], double g[3]) {
    g[0] = g[1] = g[2] = 0.0;
    for (int k = 0; k < L->d; k++) {
        int Jp[3] = {I[0], I[1], I[2]}, Jm[3] = {I[0], I[1], I[2]};
        Jp[k] += 1;
        Jm[k] -= 1;
        if (I[k] > 0 && I[k] < L->N)
            g[k] = (L->phi[or_index(L, Jp)] - L->phi[or_index(L, Jm)]) / (2.0 * L->h);
        else if (I[k] == 0)
            g[k] = (L->phi[or_index(L, Jp)] - L->phi[or_index(L, I)]) / L->h;
        else
            g[k] = (L->phi[or_index(L, I)] - L->phi[or_index(L, Jm)]) / L->h;
    }
}

/*
 * Discrete unit normal at node I (Sec. 3.3: n = grad_h phi / |grad_h phi|),
 * the axis-dominance key |grad_h phi_k| and the upwind signs s_k (+1 when
 * grad_h phi_k >= 0).  A zero discrete gradient takes the unit vector from
 * the first INSIDE axis neighbour (order -x,+x,-y,+y,-z,+z) to I.  Returns
 * |grad_h phi|.
 */
static double or_normal(const or_level *L, const int I[3], double n[3], double key[3], int s[3]) {
    int d = L->d;
    double g[3];
    or_grad(L, I, g);
    double gnorm = 0.0;
    for (int k = 0; k < d; k++) gnorm += g[k] * g[k];
    gnorm = sqrt(gnorm);
    for (int k = 0; k < 3; k++) {
        n[k] = 0.0;
        key[k] = 0.0;
        s[k] = 1;
    }
    if (gnorm > 0.0) {
        for (int k = 0; k < d; k++) {
            n[k] = g[k] / gnorm;
            key[k] = fabs(g[k]);
        }
    } else {
        int found = 0;
        for (int k = 0; k < d && !found; k++) {
            for (int sgn = -1; sgn <= 1 && !found; sgn += 2) {
                int J[3] = {I[0], I[1], I[2]};
                J[k] += sgn;
                if (!or_in_box(L, J)) continue;
                if (L->cls[or_index(L, J)] == OR_INSIDE) {
                    n[k] = -(double)sgn;
                    found = 1;
                }
            }
        }
        for (int k = 0; k < d; k++) key[k] = fabs(n[k]);
    }
    for (int k = 0; k < d; k++) s[k] = (gnorm > 0.0 ? g[k] : n[k]) >= 0.0 ? 1 : -1;
    return gnorm;
}

/* Lagrange basis on nodes 0..w-1 evaluated at t (eq. coeff for w = 3,
 * the s = 2 coefficients of Sec. 2 for w = 2). */
static double or_lagrange(int w, int m, double t) {
    if (w == 1) return 1.0;
    if (w == 2) return m == 0 ? 1.0 - t : t;
    if (m == 0) return (1.0 - t) * (2.0 - t) / 2.0;
    if (m == 1) return t * (2.0 - t);
    return t * (t - 1.0) / 2.0;
}

/* d/dt of the Lagrange basis on nodes 0..w-1 at t */
static double or_lagrange_dt(int w, int m, double t) {
    if (w == 1) return 0.0;
    if (w == 2) return m == 0 ? -1.0 : 1.0;
    if (m == 0) return t - 1.5;
    if (m == 1) return 2.0 - 2.0 * t;
    return t - 0.5;
}

/*
 * Weight of block node m (node G - m o s) in the ghost row B u~(Q) (eq. BCh),
 * u~ the tensor-product interpolant of widths w at local coordinates tau:
 *   Dirichlet: u~(Q)            = sum_m prod_k L_{m_k}(tau_k) u_m
 *   Neumann:   grad u~(Q) . n   = sum_m sum_k nd_k L'_{m_k}(tau_k) prod_{j!=k} L_{m_j}(tau_j) u_m
 * with nd_k = dt_k/dx_k n_k = -s_k n_k / h (t_k grows along -s_k).
 */
static double or_row_weight(int bc, const int w[3], const double tau[3], const double nd[3], const int m[3]) {
    if (bc == OR_BC_DIRICHLET) {
        double wgt = 1.0;
        for (int k = 0; k < 3; k++) wgt *= or_lagrange(w[k], m[k], tau[k]);
        return wgt;
    }
    double acc = 0.0;
    for (int k = 0; k < 3; k++) {
        double term = nd[k] * or_lagrange_dt(w[k], m[k], tau[k]);
        for (int j = 0; j < 3; j++)
            if (j != k) term *= or_lagrange(w[j], m[j], tau[j]);
        acc += term;
    }
    return acc;
}

/* Tensor-product quadratic interpolant of phi on the 3^d block
 * {I - m o s : m_k in 0..2} evaluated at local coordinates t. */
static double or_phi_tilde(const or_level *L, const int I[3], const int s[3], const double t[3]) {
    double val = 0.0;
    int m[3] = {0, 0, 0};
    int mmax[3] = {1, 1, 1};
    for (int k = 0; k < L->d; k++) mmax[k] = 3;
    for (m[2] = 0; m[2] < mmax[2]; m[2]++)
        for (m[1] = 0; m[1] < mmax[1]; m[1]++)
            for (m[0] = 0; m[0] < mmax[0]; m[0]++) {
                int J[3];
                double wgt = 1.0;
                for (int k = 0; k < 3; k++) {
                    J[k] = I[k] - m[k] * s[k];
                    if (k < L->d) wgt *= or_lagrange(3, m[k], t[k]);
                }
                val += wgt * L->phi[or_index(L, J)];
            }
    return val;
}

/* Is the block {I - m o s : 0 <= m_k < w_k} made of in-box INSIDE/GHOST
 * nodes?  Neumann rows also admit BOXDIR nodes (known values g_B): a ghost
 * where Gamma meets a box face otherwise has no block with a derivative
 * along the normal. */
static int or_block_valid(const or_level *L, const int I[3], const int s[3], const int w[3]) {
    int m[3];
    for (m[2] = 0; m[2] < w[2]; m[2]++)
        for (m[1] = 0; m[1] < w[1]; m[1]++)
            for (m[0] = 0; m[0] < w[0]; m[0]++) {
                int J[3];
                for (int k = 0; k < 3; k++) J[k] = I[k] - m[k] * s[k];
                if (!or_in_box(L, J)) return 0;
                unsigned char c = L->cls[or_index(L, J)];
                if (c == OR_BOXDIR && L->bc == OR_BC_NEUMANN) continue;
                if (c != OR_INSIDE && c != OR_GHOST) return 0;
            }
    return 1;
}

/*
 * Admissibility of a ghost row's block beyond validity: the row's own weight
 * c_0 must be at least the sum of |w_m| over the block's other GHOST nodes
 * whose upwind signs differ from G's, plus half the sum over those oriented
 * like G.
 * Blocks extend against the signs, so a closed loop of ghost rows, each
 * holding the next in its block, needs a sign change between two
 * consecutive ghosts of the loop: every loop has a coupling of the first
 * kind, and with full dominance there the ghost rows relaxed together
 * cannot form a nearly singular (or expanding) block.  Couplings between
 * ghosts of one orientation run one way; a row whose weight sits mostly on
 * such ghosts still relaxes slowly (they do not respond to it within the
 * step), which the half-weight term bounds.  A Neumann row also needs
 * c_0 > 0 (a width-1 axis carries no derivative).
 */
static int or_block_dominant(const or_level *L, const int I[3], const int s[3], const int w[3], const double tau[3],
                             const double nd[3]) {
    double c0 = 0.0, off = 0.0;
    int m[3];
    for (m[2] = 0; m[2] < w[2]; m[2]++)
        for (m[1] = 0; m[1] < w[1]; m[1]++)
            for (m[0] = 0; m[0] < w[0]; m[0]++) {
                int J[3];
                for (int k = 0; k < 3; k++) J[k] = I[k] - m[k] * s[k];
                double wgt = or_row_weight(L->bc, w, tau, nd, m);
                if (m[0] == 0 && m[1] == 0 && m[2] == 0) {
                    c0 = wgt;
                } else if (L->cls[or_index(L, J)] == OR_GHOST) {
                    double nJ[3], kJ[3];
                    int sJ[3];
                    or_normal(L, J, nJ, kJ, sJ);
                    if (sJ[0] != s[0] || sJ[1] != s[1] || sJ[2] != s[2]) off += fabs(wgt);
                    else off += 0.5 * fabs(wgt);
                }
            }
    if (L->bc == OR_BC_NEUMANN && !(c0 > 0.0)) return 0;
    return c0 >= off;
}

/*
 * Geometry of one ghost point G (Sec. 3.3, eqs. (BCh), (rel), (DtauOptTheta)):
 * normal n, upwind signs, stencil widths, projection Q = G - eta h n with
 * phi~(Q) = 0, local coordinates tau of Q, theta~ (eta for a full-width row)
 * and Delta tau.
 */
static void or_ghost_geometry(or_level *L, long gi, const or_options *o) {
    static const int cand3[7][3] = {{3, 3, 3}, {2, 2, 2}, {3, 3, 1}, {2, 2, 1}, {3, 1, 1}, {2, 1, 1}, {1, 1, 1}};
    static const int cand2[5][3] = {{3, 3, 1}, {2, 2, 1}, {3, 1, 1}, {2, 1, 1}, {1, 1, 1}};
    static const int cand1[3][3] = {{3, 1, 1}, {2, 1, 1}, {1, 1, 1}};
    int d = L->d;
    long p = L->gidx[gi];
    int I[3];
    or_coords(L, p, I);

    double n[3], key[3]; /* unit normal, axis-dominance key */
    int s[3];
    double gnorm = or_normal(L, I, n, key, s);

    /* axes by dominance, descending; ties keep the lower axis first */
    int ord[3] = {0, 1, 2};
    for (int a = 1; a < d; a++) {
        int b = a;
        while (b > 0 && key[ord[b - 1]] < key[ord[b]]) {
            int tmp = ord[b - 1];
            ord[b - 1] = ord[b];
            ord[b] = tmp;
            b--;
        }
    }

    /* root of phi~(G - eta h n) = 0 on the 3^d upwind block; an axis whose
     * block leaves the box is flipped for the interpolant only */
    int sp[3] = {s[0], s[1], s[2]};
    for (int k = 0; k < d; k++) {
        int far = I[k] - 2 * s[k];
        if (far < 0 || far > L->N) sp[k] = -s[k];
    }
    double phiG = L->phi[p];
    double eta;
    int fb = 0;
    if (phiG == 0.0) {
        eta = 0.0;
    } else {
        /* eta is sought in [0, 1] (Sec. 3.3): bracket at eta = 1 */
        double hi = -1.0;
        {
            double t[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < d; k++) t[k] = n[k] * sp[k];
            if (or_phi_tilde(L, I, sp, t) < 0.0) hi = 1.0;
        }
        if (hi > 0.0) {
            double lo = 0.0;
            for (int it = 0; it < 60; it++) {
                double mid = 0.5 * (lo + hi);
                double t[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < d; k++) t[k] = mid * n[k] * sp[k];
                if (or_phi_tilde(L, I, sp, t) < 0.0)
                    hi = mid;
                else
                    lo = mid;
            }
            eta = 0.5 * (lo + hi);
        } else {
            eta = phiG / (L->h * gnorm);
            if (!(eta < 1.0)) eta = 1.0;
            fb = 1;
        }
    }

    /* first admissible width vector (entries assigned to axes in dominance
     * order): block inside the box, made of INSIDE/GHOST nodes, and a row
     * whose own weight c_0 is at least the sum of the |weights| of the other
     * ghosts of the block (or_block_dominant; the option ghost_dominance = 0
     * drops this second test, for the test that shows why it is needed) */
    const int(*cand)[3] = d == 3 ? cand3 : (d == 2 ? cand2 : cand1);
    int ncand = d == 3 ? 7 : (d == 2 ? 5 : 3);
    /* Neumann rows: coefficient of d/dt_k in n . grad (t_k = (x_G - x)_k s_k / h) */
    double nd[3] = {0.0, 0.0, 0.0};
    if (L->bc == OR_BC_NEUMANN)
        for (int k = 0; k < d; k++) nd[k] = -(double)s[k] * n[k] / L->h;
    int w[3] = {1, 1, 1};
    int found = 0;
    for (int c = 0; c < ncand; c++) {
        int wt[3] = {1, 1, 1};
        for (int r = 0; r < d; r++) wt[ord[r]] = cand[c][r];
        if (!or_block_valid(L, I, s, wt)) continue;
        double tt[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < d; k++) tt[k] = wt[k] >= 2 ? eta * fabs(n[k]) : 0.0;
        if (o->ghost_dominance && !or_block_dominant(L, I, s, wt, tt, nd)) continue;
        w[0] = wt[0];
        w[1] = wt[1];
        w[2] = wt[2];
        found = 1;
        break;
    }
    /* a Neumann row with no admissible block (every candidate has a width-1
     * axis along the whole normal, or fails the test above): the one-sided
     * difference (u_G - u_J) / h towards the first INSIDE axis neighbour J
     * (order -x, +x, -y, +y, -z, +z), flagged in fb with bit 2 */
    int last_resort = -1;
    if (!found && L->bc == OR_BC_NEUMANN) {
        for (int k = 0; k < d && last_resort < 0; k++)
            for (int sgn = -1; sgn <= 1 && last_resort < 0; sgn += 2) {
                int J[3] = {I[0], I[1], I[2]};
                J[k] += sgn;
                if (or_in_box(L, J) && L->cls[or_index(L, J)] == OR_INSIDE) {
                    last_resort = k;
                    s[k] = -sgn;
                }
            }
        for (int k = 0; k < 3; k++) {
            w[k] = k == last_resort ? 2 : 1;
            nd[k] = k == last_resort ? -1.0 / L->h : 0.0;
        }
        fb |= 2;
    }

    for (int k = 0; k < 3; k++) {
        L->gw[3 * gi + k] = w[k];
        L->gs[3 * gi + k] = s[k];
        L->gn[3 * gi + k] = n[k];
        double xk = k < d ? -1.0 + I[k] * L->h : 0.0;
        L->gq[3 * gi + k] = k < d ? xk - eta * L->h * n[k] : 0.0;
        L->gtau[3 * gi + k] = (k < d && w[k] >= 2 && last_resort < 0) ? eta * fabs(n[k]) : 0.0;
        L->gnd[3 * gi + k] = nd[k];
    }
    L->geta[gi] = eta;
    L->gfb[gi] = fb;
    /* theta~ of eq. (DtauOptTheta): the distance, along the normal, from G
     * to the point where the row interpolates.  Remark (exptheta2D) reads
     * G_0 as the value there of an error mode exp(-p (x_G - x).n / h) that
     * decays along the normal.  A full-width row interpolates at Q itself,
     * so theta~ = |G - Q| / h = eta.  A row with width-1 axes interpolates
     * at Q projected onto the span of its other axes (tau_k = 0 on the
     * width-1 ones), whose distance from G along n is eta * sum of n_k^2
     * over the kept axes. */
    double theta = eta;
    if (last_resort < 0) {
        int shortened = 0;
        double nn2 = 0.0;
        for (int k = 0; k < d; k++) {
            if (w[k] >= 2)
                nn2 += n[k] * n[k];
            else
                shortened = 1;
        }
        if (shortened) theta = eta * nn2;
    }
    double dt = L->bc == OR_BC_NEUMANN ? L->h * or_dtau_neumann(d, theta, o->dtau_mode, o->dtau_const)
                                       : or_dtau(d, theta, o->dtau_mode, o->dtau_const);
    /* never relax a ghost row beyond its own Gauss-Seidel step dtau = 1/c_0
     * (the value the relaxation reduces to at theta = 0, Sec. 2.1); on the
     * quadratic row of the BLFA this bound is inactive in 2D and within 3%
     * in 3D, it only tames the shortened stencils */
    if (o->dtau_mode != OR_DTAU_CONST) {
        const int m0[3] = {0, 0, 0};
        double c0 = or_row_weight(L->bc, w, &L->gtau[3 * gi], nd, m0);
        if (c0 > 0.0 && dt * c0 > 1.0) dt = 1.0 / c0;
    }
    L->gdtau[gi] = dt;
}

/* ------------------------------------------------------------------------- */
/* Operators                                                                  */

/* sum_m w_m u(G - m o s) over the ghost block (eq. BCh; the weights of
 * or_row_weight for the level's boundary type) */
static double or_ghost_row(const or_level *L, long gi, const double *u) {
    long p = L->gidx[gi];
    int I[3];
    or_coords(L, p, I);
    const int *w = &L->gw[3 * gi];
    const int *s = &L->gs[3 * gi];
    const double *tau = &L->gtau[3 * gi];
    const double *nd = &L->gnd[3 * gi];
    double acc = 0.0;
    int m[3];
    for (m[2] = 0; m[2] < w[2]; m[2]++)
        for (m[1] = 0; m[1] < w[1]; m[1]++)
            for (m[0] = 0; m[0] < w[0]; m[0]++) {
                int J[3];
                for (int k = 0; k < 3; k++) J[k] = I[k] - m[k] * s[k];
                double wgt = or_row_weight(L->bc, w, tau, nd, m);
                acc += wgt * u[or_index(L, J)];
            }
    return acc;
}

/* the part of the ghost row on BOXDIR block nodes (Neumann rows only) */
static double or_ghost_row_boxdir(const or_level *L, long gi, const double *u) {
    long p = L->gidx[gi];
    int I[3];
    or_coords(L, p, I);
    const int *w = &L->gw[3 * gi];
    const int *s = &L->gs[3 * gi];
    double acc = 0.0;
    int m[3];
    for (m[2] = 0; m[2] < w[2]; m[2]++)
        for (m[1] = 0; m[1] < w[1]; m[1]++)
            for (m[0] = 0; m[0] < w[0]; m[0]++) {
                int J[3];
                for (int k = 0; k < 3; k++) J[k] = I[k] - m[k] * s[k];
                long q = or_index(L, J);
                if (L->cls[q] == OR_BOXDIR) acc += or_row_weight(L->bc, w, &L->gtau[3 * gi], &L->gnd[3 * gi], m) * u[q];
            }
    return acc;
}

/* interior row (eq. Laph and its 1D/3D analogues) of c u - Laplace u:
 * (2d u_P - sum nbrs)/h^2 + c u_P  (c = 0: the Poisson problem) */
static double or_lap(const or_level *L, long p, const double *u) {
    double s = 0.0;
    for (int k = 0; k < L->d; k++) s += u[p + L->st[k]] + u[p - L->st[k]];
    double v = (2.0 * L->d * u[p] - s) / (L->h * L->h);
    if (L->reaction != 0.0) v += L->reaction * u[p];
    return v;
}

/* A u on INSIDE and GHOST rows, 0 elsewhere (the system A_h u_h = f_h) */
void or_apply_A(or_problem *P, int l, const double *u, double *Au) {
    or_level *L = &P->lev[l];
    for (long p = 0; p < L->nn; p++) Au[p] = 0.0;
    for (long p = 0; p < L->nn; p++)
        if (L->cls[p] == OR_INSIDE) Au[p] = or_lap(L, p, u);
    for (long gi = 0; gi < L->ng; gi++) Au[L->gidx[gi]] = or_ghost_row(L, gi, u);
}

/* Residual r = rhs - A u on INSIDE and GHOST rows, 0 elsewhere (Sec. 2.1) */
void or_residual(or_problem *P, int l, const double *u, const double *rhs, double *r) {
    or_level *L = &P->lev[l];
    for (long p = 0; p < L->nn; p++) r[p] = 0.0;
    for (long p = 0; p < L->nn; p++)
        if (L->cls[p] == OR_INSIDE) r[p] = rhs[p] - or_lap(L, p, u);
    for (long gi = 0; gi < L->ng; gi++) {
        long p = L->gidx[gi];
        r[p] = rhs[p] - or_ghost_row(L, gi, u);
    }
}

/* Euclidean norm of r over INSIDE and GHOST rows, serial lexicographic sum */
double or_norm(or_problem *P, int l, const double *r) {
    or_level *L = &P->lev[l];
    double s = 0.0;
    for (long p = 0; p < L->nn; p++)
        if (L->cls[p] == OR_INSIDE || L->cls[p] == OR_GHOST) s += r[p] * r[p];
    return sqrt(s);
}

/*
 * One smoothing step (the REL-ALL preconditioner, eq. 2Ddiri:P): Gauss-Seidel
 * on the interior (eq. GSLEX_2D, or its red-black ordering), or weighted
 * Jacobi (Sec. 2.1: P = omega diag + (1 - omega) I with omega = 2/3 in 1D;
 * here omega = 2d/(2d+1), the d-dimensional form of that choice: 4/5 in 2D,
 * 6/7 in 3D), then one
 * fictitious-time relaxation of every ghost row (eq. rel with DtauOptTheta)
 * using the new interior values and the old ghost values (P_GG = I/dtau).
 */
void or_smooth(or_problem *P, int l, double *u, const double *rhs) {
    or_level *L = &P->lev[l];
    double h2 = L->h * L->h;
    double diag = 2.0 * L->d + L->reaction * h2; /* h^2 times the row's own coefficient */
    int I[3];
    if (P->opt.smoother == OR_SMOOTH_JAC) {
        double omega = 2.0 * L->d / (2.0 * L->d + 1.0);
        double *unew = (double *)malloc(sizeof(double) * L->nn); /* new INSIDE values from the old field */
        for (long p = 0; p < L->nn; p++) {
            if (L->cls[p] != OR_INSIDE) continue;
            double s = 0.0;
            for (int k = 0; k < L->d; k++) s += u[p + L->st[k]] + u[p - L->st[k]];
            unew[p] = u[p] + omega * ((h2 * rhs[p] + s) / diag - u[p]);
        }
        for (long p = 0; p < L->nn; p++)
            if (L->cls[p] == OR_INSIDE) u[p] = unew[p];
        free(unew);
    } else if (P->opt.smoother == OR_SMOOTH_LEX) {
        for (long p = 0; p < L->nn; p++) {
            if (L->cls[p] != OR_INSIDE) continue;
            double s = 0.0;
            for (int k = 0; k < L->d; k++) s += u[p + L->st[k]] + u[p - L->st[k]];
            u[p] = (h2 * rhs[p] + s) / diag;
        }
    } else {
        for (int colour = 0; colour < 2; colour++) {
            for (long p = 0; p < L->nn; p++) {
                if (L->cls[p] != OR_INSIDE) continue;
                or_coords(L, p, I);
                if (((I[0] + I[1] + I[2]) & 1) != colour) continue;
                double s = 0.0;
                for (int k = 0; k < L->d; k++) s += u[p + L->st[k]] + u[p - L->st[k]];
                u[p] = (h2 * rhs[p] + s) / diag;
            }
        }
    }
    double *delta = L->e; /* scratch */
    for (long gi = 0; gi < L->ng; gi++) {
        long p = L->gidx[gi];
        delta[gi] = L->gdtau[gi] * (rhs[p] - or_ghost_row(L, gi, u));
    }
    for (long gi = 0; gi < L->ng; gi++) u[L->gidx[gi]] += delta[gi];
}

/*
 * Extension of ghost values into the inactive nodes along the normal
 * (Sec. 3.3 "Transfer operators": a few pseudo-time steps of
 * dr/dsigma + dr/dn = 0).  Reading: K Jacobi sweeps of the steady upwind
 * form v(X) = sum_k |n_k| v(X - s_k e_k) / sum_k |n_k| on every OUTSIDE
 * node, starting from v = 0; out-of-box terms dropped, BOXDIR values 0,
 * GHOST and INSIDE values never changed; zero weight sum -> mean of the
 * GHOST nodes of the 3^d box (0 if none).
 */
void or_extend(or_problem *P, int l, double *v) {
    or_level *L = &P->lev[l];
    int d = L->d;
    double *old = (double *)malloc(sizeof(double) * L->nn);
    int I[3];
    for (long p = 0; p < L->nn; p++)
        if (L->cls[p] == OR_OUTSIDE) v[p] = 0.0;
    for (int it = 0; it < P->opt.ext_iters; it++) {
        memcpy(old, v, sizeof(double) * L->nn);
        for (long p = 0; p < L->nn; p++) {
            if (L->cls[p] != OR_OUTSIDE) continue;
            or_coords(L, p, I);
            double g[3];
            or_grad(L, I, g);
            double gnorm = 0.0;
            for (int k = 0; k < d; k++) gnorm += g[k] * g[k];
            gnorm = sqrt(gnorm);
            double num = 0.0, den = 0.0;
            if (gnorm > 0.0) {
                for (int k = 0; k < d; k++) {
                    double nk = g[k] / gnorm;
                    int sk = g[k] >= 0.0 ? 1 : -1;
                    int J[3] = {I[0], I[1], I[2]};
                    J[k] -= sk;
                    if (!or_in_box(L, J)) continue;
                    long q = or_index(L, J);
                    double val = L->cls[q] == OR_BOXDIR ? 0.0 : old[q];
                    num += fabs(nk) * val;
                    den += fabs(nk);
                }
            }
            if (den > 0.0) {
                v[p] = num / den;
            } else {
                double sum = 0.0;
                int cnt = 0;
                int m[3], lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
                for (int k = 0; k < d; k++) {
                    lo[k] = -1;
                    hi[k] = 1;
                }
                for (m[2] = lo[2]; m[2] <= hi[2]; m[2]++)
                    for (m[1] = lo[1]; m[1] <= hi[1]; m[1]++)
                        for (m[0] = lo[0]; m[0] <= hi[0]; m[0]++) {
                            int J[3] = {I[0] + m[0], I[1] + m[1], I[2] + m[2]};
                            if (!or_in_box(L, J)) continue;
                            long q = or_index(L, J);
                            if (L->cls[q] == OR_GHOST) {
                                sum += old[q];
                                cnt++;
                            }
                        }
                v[p] = cnt > 0 ? sum / cnt : 0.0;
            }
        }
    }
    free(old);
}

/*
 * Restriction fine level l -> coarse level l+1 (Sec. 2.1 eq. coarseFW,
 * Sec. 3.2 nine-point FW, Sec. 3.3 "Transfer operators").  rfine must hold
 * the residual of level l already extended into the OUTSIDE nodes.
 *   coarse INSIDE: FW over the 3^d fine box around X = 2J if all of it is
 *     INSIDE, else the FW weights of its INSIDE nodes renormalised to 1.
 *   coarse GHOST: FW if the box holds no INSIDE node and lies in the box,
 *     else renormalised FW over its non-INSIDE, non-BOXDIR in-box nodes.
 *   PLAIN_MEAN replaces the renormalised weights by an unweighted mean.
 *   other coarse nodes: 0.
 */
void or_restrict(or_problem *P, int l, const double *rfine, double *rc) {
    or_level *F = &P->lev[l];
    or_level *C = &P->lev[l + 1];
    int d = F->d;
    int Jc[3];
    for (long pc = 0; pc < C->nn; pc++) {
        rc[pc] = 0.0;
        unsigned char cc = C->cls[pc];
        if (cc != OR_INSIDE && cc != OR_GHOST) continue;
        or_coords(C, pc, Jc);
        int X[3] = {2 * Jc[0], 2 * Jc[1], 2 * Jc[2]};
        double full = 0.0, sel = 0.0, selw = 0.0, selcnt = 0.0;
        int all_ok = 1; /* every box node in-box and (INSIDE | non-INSIDE) */
        int m[3], lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int k = 0; k < d; k++) {
            lo[k] = -1;
            hi[k] = 1;
        }
        for (m[2] = lo[2]; m[2] <= hi[2]; m[2]++)
            for (m[1] = lo[1]; m[1] <= hi[1]; m[1]++)
                for (m[0] = lo[0]; m[0] <= hi[0]; m[0]++) {
                    int J[3] = {X[0] + m[0], X[1] + m[1], X[2] + m[2]};
                    double wgt = 1.0;
                    for (int k = 0; k < d; k++) wgt *= (m[k] == 0 ? 0.5 : 0.25);
                    if (!or_in_box(F, J)) {
                        all_ok = 0;
                        continue;
                    }
                    long q = or_index(F, J);
                    unsigned char fc = F->cls[q];
                    int take;
                    if (cc == OR_INSIDE) {
                        take = fc == OR_INSIDE;
                        if (!take) all_ok = 0;
                    } else {
                        take = fc != OR_INSIDE && fc != OR_BOXDIR;
                        if (fc == OR_INSIDE) all_ok = 0;
                    }
                    full += wgt * rfine[q];
                    if (take) {
                        sel += wgt * rfine[q];
                        selw += wgt;
                        selcnt += 1.0;
                    }
                }
        (void)selcnt;
        if (all_ok) {
            rc[pc] = full;
        } else if (P->opt.restrict_mode == OR_RESTRICT_PLAIN_MEAN) {
            double s = 0.0, c = 0.0;
            for (m[2] = lo[2]; m[2] <= hi[2]; m[2]++)
                for (m[1] = lo[1]; m[1] <= hi[1]; m[1]++)
                    for (m[0] = lo[0]; m[0] <= hi[0]; m[0]++) {
                        int J[3] = {X[0] + m[0], X[1] + m[1], X[2] + m[2]};
                        if (!or_in_box(F, J)) continue;
                        long q = or_index(F, J);
                        unsigned char fc = F->cls[q];
                        int take = cc == OR_INSIDE ? fc == OR_INSIDE : (fc != OR_INSIDE && fc != OR_BOXDIR);
                        if (take) {
                            s += rfine[q];
                            c += 1.0;
                        }
                    }
            rc[pc] = c > 0.0 ? s / c : 0.0;
        } else {
            rc[pc] = selw > 0.0 ? sel / selw : 0.0;
        }
    }
}

/*
 * Prolongation and correction, coarse level l+1 -> fine level l (Sec. 2.1
 * interpolation operator, Sec. 3.2 bilinear interpolation, Sec. 3.3: after
 * extending the coarse error into the inactive nodes).  ec is modified:
 * BOXDIR entries are set to 0 and OUTSIDE entries receive the extension.
 */
void or_prolong(or_problem *P, int l, double *ec, double *u) {
    or_level *F = &P->lev[l];
    or_level *C = &P->lev[l + 1];
    int d = F->d;
    for (long pc = 0; pc < C->nn; pc++)
        if (C->cls[pc] == OR_BOXDIR) ec[pc] = 0.0;
    or_extend(P, l + 1, ec);
    int I[3];
    for (long p = 0; p < F->nn; p++) {
        unsigned char c = F->cls[p];
        if (c != OR_INSIDE && c != OR_GHOST) continue;
        or_coords(F, p, I);
        int m[3], hi[3] = {0, 0, 0};
        for (int k = 0; k < d; k++) hi[k] = I[k] & 1;
        double e = 0.0;
        for (m[2] = 0; m[2] <= hi[2]; m[2]++)
            for (m[1] = 0; m[1] <= hi[1]; m[1]++)
                for (m[0] = 0; m[0] <= hi[0]; m[0]++) {
                    int J[3] = {0, 0, 0};
                    double wgt = 1.0;
                    for (int k = 0; k < d; k++) {
                        J[k] = (I[k] - (I[k] & 1)) / 2 + m[k];
                        if (I[k] & 1) wgt *= 0.5;
                    }
                    e += wgt * ec[or_index(C, J)];
                }
        u[p] += e;
    }
}

/* ------------------------------------------------------------------------- */
/* Coarsest-level solve: Gaussian elimination with partial pivoting on the   */
/* dense INSIDE U GHOST rows (Sec. 2.1: solved exactly on the coarse grid).  */

static void or_coarse_factor(or_problem *P) {
    or_level *L = &P->lev[P->L - 1];
    long nc = L->ni + L->ng;
    P->nc = nc;
    P->cmap = (long *)malloc(sizeof(long) * (nc > 0 ? nc : 1));
    long *pos = (long *)malloc(sizeof(long) * L->nn);
    long c = 0;
    for (long p = 0; p < L->nn; p++) {
        pos[p] = -1;
        if (L->cls[p] == OR_INSIDE) {
            pos[p] = c;
            P->cmap[c++] = p;
        }
    }
    for (long gi = 0; gi < L->ng; gi++) {
        pos[L->gidx[gi]] = c;
        P->cmap[c++] = L->gidx[gi];
    }
    P->lu = (double *)calloc((size_t)(nc > 0 ? nc * nc : 1), sizeof(double));
    P->piv = (long *)malloc(sizeof(long) * (nc > 0 ? nc : 1));
    double ih2 = 1.0 / (L->h * L->h);
    for (long row = 0; row < L->ni; row++) {
        long p = P->cmap[row];
        P->lu[row * nc + row] += 2.0 * L->d * ih2 + L->reaction;
        for (int k = 0; k < L->d; k++) {
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                long q = p + sgn * L->st[k];
                if (pos[q] >= 0) P->lu[row * nc + pos[q]] -= ih2;
            }
        }
    }
    for (long gi = 0; gi < L->ng; gi++) {
        long row = L->ni + gi;
        long p = L->gidx[gi];
        int I[3];
        or_coords(L, p, I);
        const int *w = &L->gw[3 * gi];
        const int *s = &L->gs[3 * gi];
        const double *tau = &L->gtau[3 * gi];
        const double *nd = &L->gnd[3 * gi];
        int m[3];
        for (m[2] = 0; m[2] < w[2]; m[2]++)
            for (m[1] = 0; m[1] < w[1]; m[1]++)
                for (m[0] = 0; m[0] < w[0]; m[0]++) {
                    int J[3];
                    for (int k = 0; k < 3; k++) J[k] = I[k] - m[k] * s[k];
                    double wgt = or_row_weight(L->bc, w, tau, nd, m);
                    long q = or_index(L, J);
                    if (pos[q] >= 0) P->lu[row * nc + pos[q]] += wgt; /* BOXDIR: right-hand side */
                }
    }
    free(pos);
    double amax = 0.0;
    for (long i = 0; i < nc * nc; i++)
        if (fabs(P->lu[i]) > amax) amax = fabs(P->lu[i]);
    P->coarse_singular = 0;
    double *A = P->lu;
    for (long k = 0; k < nc; k++) {
        long pr = k;
        for (long i = k + 1; i < nc; i++)
            if (fabs(A[i * nc + k]) > fabs(A[pr * nc + k])) pr = i;
        P->piv[k] = pr;
        if (pr != k)
            for (long j = 0; j < nc; j++) {
                double t = A[k * nc + j];
                A[k * nc + j] = A[pr * nc + j];
                A[pr * nc + j] = t;
            }
        if (fabs(A[k * nc + k]) < 1e-14 * amax) {
            P->coarse_singular = 1;
            return;
        }
        for (long i = k + 1; i < nc; i++) {
            double f = A[i * nc + k] / A[k * nc + k];
            A[i * nc + k] = f;
            for (long j = k + 1; j < nc; j++) A[i * nc + j] -= f * A[k * nc + j];
        }
    }
}

/* Solve on the coarsest level: u (unknown entries) such that A u = rhs,
 * BOXDIR values of u moved to the right-hand side. */
void or_coarse_solve(or_problem *P, double *u, const double *rhs) {
    int l = P->L - 1;
    or_level *L = &P->lev[l];
    long nc = P->nc;
    if (nc == 0) return;
    if (P->coarse_singular) {
        for (int it = 0; it < 50; it++) or_smooth(P, l, u, rhs);
        P->coarse_fallbacks++;
        return;
    }
    double *b = (double *)malloc(sizeof(double) * nc);
    double ih2 = 1.0 / (L->h * L->h);
    for (long row = 0; row < nc; row++) {
        long p = P->cmap[row];
        b[row] = rhs[p];
        if (row < L->ni)
            for (int k = 0; k < L->d; k++)
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    long q = p + sgn * L->st[k];
                    if (L->cls[q] == OR_BOXDIR) b[row] += u[q] * ih2;
                }
        else
            b[row] -= or_ghost_row_boxdir(L, row - L->ni, u);
    }
    const double *A = P->lu;
    /* the factorisation swapped whole rows, multipliers included (P A = L U
     * with P the interchanges in order): permute b first, then L y = P b */
    for (long k = 0; k < nc; k++) {
        long pr = P->piv[k];
        if (pr != k) {
            double t = b[k];
            b[k] = b[pr];
            b[pr] = t;
        }
    }
    for (long k = 0; k < nc; k++)
        for (long i = k + 1; i < nc; i++) b[i] -= A[i * nc + k] * b[k];
    for (long k = nc - 1; k >= 0; k--) {
        double s = b[k];
        for (long j = k + 1; j < nc; j++) s -= A[k * nc + j] * b[j];
        b[k] = s / A[k * nc + k];
    }
    for (long row = 0; row < nc; row++) u[P->cmap[row]] = b[row];
    free(b);
}

/* ------------------------------------------------------------------------- */
/* Cycles (Sec. 2.1: TGCS, and its recursion with gamma = 1, the V-cycle, or  */
/* gamma = 2, the W-cycle)                                                    */

static void or_vcycle_level(or_problem *P, int l, double *u, const double *rhs);

/* Solve level l to a relative residual of tol by V-cycles from u = 0 */
static void or_solve_level(or_problem *P, int l, double *u, const double *rhs, double tol) {
    or_level *L = &P->lev[l];
    or_residual(P, l, u, rhs, L->r);
    double r0 = or_norm(P, l, L->r);
    if (r0 == 0.0) return;
    for (int it = 0; it < 200; it++) {
        or_vcycle_level(P, l, u, rhs);
        or_residual(P, l, u, rhs, L->r);
        if (or_norm(P, l, L->r) <= tol * r0) break;
    }
}

static void or_vcycle_level(or_problem *P, int l, double *u, const double *rhs) {
    if (l == P->L - 1) {
        or_coarse_solve(P, u, rhs);
        return;
    }
    or_level *F = &P->lev[l];
    or_level *C = &P->lev[l + 1];
    for (int i = 0; i < P->opt.nu1; i++) or_smooth(P, l, u, rhs);
    or_residual(P, l, u, rhs, F->r);
    or_extend(P, l, F->r);
    or_restrict(P, l, F->r, C->rhs);
    for (long p = 0; p < C->nn; p++) C->u[p] = 0.0;
    int inner_cycle = l + 1 < P->L - 1;
    if (P->opt.cycle == OR_CYCLE_TGCS && l == 0 && inner_cycle) {
        or_solve_level(P, 1, C->u, C->rhs, 1e-14);
    } else {
        /* gamma cycles on the coarse residual equation; the coarsest level
         * is solved exactly, once */
        int gamma = P->opt.cycle == OR_CYCLE_W && inner_cycle ? 2 : 1;
        for (int g = 0; g < gamma; g++) or_vcycle_level(P, l + 1, C->u, C->rhs);
    }
    memcpy(C->e, C->u, sizeof(double) * C->nn);
    or_prolong(P, l, C->e, u);
    for (int i = 0; i < P->opt.nu2; i++) or_smooth(P, l, u, rhs);
}

void or_vcycle(or_problem *P, double *u) { or_vcycle_level(P, 0, u, P->lev[0].rhs); }

/*
 * Solve from the given u (BOXDIR entries hold g_B) until
 * |r_m| / |r_0| <= tol (Sec. 3.3, comparison with AGMG: residual normalised
 * by the first iteration).  hist (max_cycles+1 entries, may be NULL)
 * receives |r_m|.  Returns the number of cycles, or -1 without convergence.
 */
int or_solve(or_problem *P, double *u, double tol, int max_cycles, double *hist) {
    or_level *L = &P->lev[0];
    or_residual(P, 0, u, L->rhs, L->r);
    double r0 = or_norm(P, 0, L->r);
    if (hist) hist[0] = r0;
    if (!isfinite(r0)) return -1; /* NaN or Inf in the data: diverged before any cycle */
    if (r0 == 0.0) return 0;
    for (int m = 1; m <= max_cycles; m++) {
        or_vcycle(P, u);
        or_residual(P, 0, u, L->rhs, L->r);
        double rm = or_norm(P, 0, L->r);
        if (hist) hist[m] = rm;
        if (!isfinite(rm)) return -1;
        if (rm <= tol * r0) return m;
        /* divergence: non-finite, or growth past 1e3 x the larger of the first
         * two norms (the first cycle may raise the unscaled norm by O(h^-2)
         * when the initial residual lives on the ghost rows only) */
        double ref = hist ? (m >= 2 ? fmax(hist[0], hist[1]) : hist[0]) : r0;
        if (!isfinite(rm) || (m >= 2 && rm > 1e3 * ref)) return -1;
    }
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Setup / teardown                                                           */

static void or_level_alloc(or_level *L, int d, int N) {
    memset(L, 0, sizeof *L);
    L->d = d;
    L->N = N;
    L->n = N + 1;
    L->nn = 1;
    for (int k = 0; k < 3; k++) L->st[k] = 0;
    long s = 1;
    for (int k = 0; k < d; k++) {
        L->st[k] = s;
        s *= L->n;
    }
    L->nn = s;
    L->h = 2.0 / N;
    L->phi = (double *)calloc(L->nn, sizeof(double));
    L->cls = (unsigned char *)calloc(L->nn, 1);
    L->u = (double *)calloc(L->nn, sizeof(double));
    L->rhs = (double *)calloc(L->nn, sizeof(double));
    L->r = (double *)calloc(L->nn, sizeof(double));
    L->e = (double *)calloc(L->nn, sizeof(double));
}

static void or_level_geometry(or_level *L, const or_options *o) {
    or_classify(L->d, L->N, L->phi, L->cls);
    L->ni = L->ng = 0;
    for (long p = 0; p < L->nn; p++) {
        if (L->cls[p] == OR_INSIDE) L->ni++;
        if (L->cls[p] == OR_GHOST) L->ng++;
    }
    long ng = L->ng > 0 ? L->ng : 1;
    L->gidx = (long *)malloc(sizeof(long) * ng);
    L->gw = (int *)malloc(sizeof(int) * 3 * ng);
    L->gs = (int *)malloc(sizeof(int) * 3 * ng);
    L->gfb = (int *)malloc(sizeof(int) * ng);
    L->geta = (double *)malloc(sizeof(double) * ng);
    L->gn = (double *)malloc(sizeof(double) * 3 * ng);
    L->gq = (double *)malloc(sizeof(double) * 3 * ng);
    L->gtau = (double *)malloc(sizeof(double) * 3 * ng);
    L->gdtau = (double *)malloc(sizeof(double) * ng);
    L->gnd = (double *)malloc(sizeof(double) * 3 * ng);
    L->bc = o->bc;
    L->reaction = o->reaction;
    long c = 0;
    for (long p = 0; p < L->nn; p++)
        if (L->cls[p] == OR_GHOST) L->gidx[c++] = p;
    for (long gi = 0; gi < L->ng; gi++) or_ghost_geometry(L, gi, o);
}

/*
 * Build the hierarchy from phi sampled at the finest nodes ((N+1)^d,
 * x fastest).  Coarse phi is injected from the finer level (coarse nodes
 * are a subset of the fine nodes), and every level is classified and
 * given its own ghost geometry.  N must be a power of two with at least
 * two levels down to opt->coarsest_N.  Returns NULL on bad arguments.
 */
or_problem *or_setup(int d, int N, const double *phi, const or_options *opt) {
    if (d < 1 || d > 3 || N < 4 || opt->coarsest_N < 4) return NULL; /* 3-node interpolants need N >= 4 */
    if (N & (N - 1)) return NULL;
    or_problem *P = (or_problem *)calloc(1, sizeof(or_problem));
    P->d = d;
    P->opt = *opt;
    int L = 0;
    for (int NN = N; NN >= opt->coarsest_N; NN /= 2) {
        L++;
        if (NN == opt->coarsest_N) break;
        if (NN % 2) {
            free(P);
            return NULL;
        }
    }
    if (L < 2 || L > OR_MAXLEV) {
        free(P);
        return NULL;
    }
    P->L = L;
    for (int l = 0; l < L; l++) or_level_alloc(&P->lev[l], d, N >> l);
    memcpy(P->lev[0].phi, phi, sizeof(double) * P->lev[0].nn);
    for (int l = 1; l < L; l++) {
        or_level *F = &P->lev[l - 1], *C = &P->lev[l];
        int J[3];
        for (long pc = 0; pc < C->nn; pc++) {
            or_coords(C, pc, J);
            int I[3] = {2 * J[0], 2 * J[1], 2 * J[2]};
            C->phi[pc] = F->phi[or_index(F, I)];
        }
    }
    for (int l = 0; l < L; l++) or_level_geometry(&P->lev[l], opt);
    or_coarse_factor(P);
    return P;
}

void or_destroy(or_problem *P) {
    if (!P) return;
    for (int l = 0; l < P->L; l++) {
        or_level *L = &P->lev[l];
        free(L->phi);
        free(L->cls);
        free(L->u);
        free(L->rhs);
        free(L->r);
        free(L->e);
        free(L->gidx);
        free(L->gw);
        free(L->gs);
        free(L->gfb);
        free(L->geta);
        free(L->gn);
        free(L->gq);
        free(L->gtau);
        free(L->gdtau);
        free(L->gnd);
    }
    free(P->cmap);
    free(P->lu);
    free(P->piv);
    free(P);
}

/* ------------------------------------------------------------------------- */
/* Accessors for the Python side                                              */

int or_num_levels(or_problem *P) { return P->L; }
int or_level_N(or_problem *P, int l) { return P->lev[l].N; }
long or_level_nodes(or_problem *P, int l) { return P->lev[l].nn; }
void or_counts(or_problem *P, int l, long *ni, long *ng) {
    *ni = P->lev[l].ni;
    *ng = P->lev[l].ng;
}
int or_coarse_singular(or_problem *P) { return P->coarse_singular; }
long or_coarse_fallbacks(or_problem *P) { return P->coarse_fallbacks; }
long or_coarse_unknowns(or_problem *P) { return P->nc; }

void or_get_phi(or_problem *P, int l, double *out) { memcpy(out, P->lev[l].phi, sizeof(double) * P->lev[l].nn); }
void or_get_classes(or_problem *P, int l, unsigned char *out) { memcpy(out, P->lev[l].cls, P->lev[l].nn); }

/* ghost arrays: idx[ng], w[ng*3], s[ng*3], fb[ng], eta[ng], n[ng*3], q[ng*3], tau[ng*3], dtau[ng] */
void or_get_ghosts(or_problem *P, int l, long *idx, int *w, int *s, int *fb, double *eta, double *n, double *q,
                   double *tau, double *dtau) {
    or_level *L = &P->lev[l];
    long ng = L->ng;
    if (idx) memcpy(idx, L->gidx, sizeof(long) * ng);
    if (w) memcpy(w, L->gw, sizeof(int) * 3 * ng);
    if (s) memcpy(s, L->gs, sizeof(int) * 3 * ng);
    if (fb) memcpy(fb, L->gfb, sizeof(int) * ng);
    if (eta) memcpy(eta, L->geta, sizeof(double) * ng);
    if (n) memcpy(n, L->gn, sizeof(double) * 3 * ng);
    if (q) memcpy(q, L->gq, sizeof(double) * 3 * ng);
    if (tau) memcpy(tau, L->gtau, sizeof(double) * 3 * ng);
    if (dtau) memcpy(dtau, L->gdtau, sizeof(double) * ng);
}

/* Neumann derivative coefficients nd[ng*3] (0 for Dirichlet rows) */
void or_get_ghost_nd(or_problem *P, int l, double *nd) {
    memcpy(nd, P->lev[l].gnd, sizeof(double) * 3 * P->lev[l].ng);
}

/* Finest-level right-hand side: f on INSIDE nodes, g(Q) on ghost rows
 * (given in ghost-list order). */
void or_set_rhs(or_problem *P, const double *f, const double *gq) {
    or_level *L = &P->lev[0];
    for (long p = 0; p < L->nn; p++) L->rhs[p] = L->cls[p] == OR_INSIDE ? f[p] : 0.0;
    for (long gi = 0; gi < L->ng; gi++) L->rhs[L->gidx[gi]] = gq[gi];
}

void or_get_rhs(or_problem *P, int l, double *out) { memcpy(out, P->lev[l].rhs, sizeof(double) * P->lev[l].nn); }
void or_set_level_rhs(or_problem *P, int l, const double *in) {
    memcpy(P->lev[l].rhs, in, sizeof(double) * P->lev[l].nn);
}

/* smoothing steps on level l with the level's own right-hand side array */
void or_smooth_n(or_problem *P, int l, double *u, const double *rhs, int nsteps) {
    for (int i = 0; i < nsteps; i++) or_smooth(P, l, u, rhs);
}

/* one V-cycle starting at level l (u, rhs of that level) */
void or_vcycle_at(or_problem *P, int l, double *u, const double *rhs) { or_vcycle_level(P, l, u, rhs); }
