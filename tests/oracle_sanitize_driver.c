/*
 * Host sanitizer run of the oracle (test infrastructure): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitize.py, it sets up and solves small problems through
 * every option of the oracle (2D and 3D, Dirichlet and Neumann rows, the
 * three dtau forms, the three smoothers and cycles, a sphere union with
 * crossed ghost pairs, a one-node domain) and destroys them.  Any invalid
 * access or undefined operation aborts the run.
 */
#include "../oracle/bcmg_oracle.c"

static double *sample(int d, int N, double (*fn)(const double *)) {
    long nn = 1;
    for (int k = 0; k < d; k++) nn *= N + 1;
    double *a = (double *)malloc(sizeof(double) * nn);
    for (long p = 0; p < nn; p++) {
        double x[3] = {0, 0, 0};
        long q = p;
        for (int k = 0; k < d; k++) {
            x[k] = -1.0 + 2.0 * (double)(q % (N + 1)) / N;
            q /= N + 1;
        }
        a[p] = fn(x);
    }
    return a;
}

static double circle(const double *x) { return sqrt((x[0] - 0.02) * (x[0] - 0.02) + (x[1] - 0.03) * (x[1] - 0.03)) - 0.5; }
static double sphere(const double *x) { return sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) - 0.55; }
static double spheres(const double *x) {
    static const double c[4][4] = {{0.1, 0.1, 0.0, 0.3}, {-0.35, 0.0, 0.1, 0.2}, {0.3, -0.3, 0.2, 0.12}, {0.0, 0.4, -0.3, 0.07}};
    double v = 1e9;
    for (int i = 0; i < 4; i++) {
        double r = sqrt((x[0] - c[i][0]) * (x[0] - c[i][0]) + (x[1] - c[i][1]) * (x[1] - c[i][1]) +
                        (x[2] - c[i][2]) * (x[2] - c[i][2])) - c[i][3];
        if (r < v) v = r;
    }
    return v;
}
static double one_node(const double *x) { return sqrt((x[0] - 0.13) * (x[0] - 0.13) + (x[1] - 0.13) * (x[1] - 0.13)) - 0.3 * 0.125; }
static double line1d(const double *x) { return x[0] - 0.3137; }

static int run(int d, int N, double (*fn)(const double *), or_options o, int cycles) {
    double *phi = sample(d, N, fn);
    or_problem *P = or_setup(d, N, phi, &o);
    free(phi);
    if (!P) return 1;
    or_level *L = &P->lev[0];
    double *f = (double *)calloc(L->nn, sizeof(double));
    double *gq = (double *)calloc(L->ng > 0 ? L->ng : 1, sizeof(double));
    double *u = (double *)calloc(L->nn, sizeof(double));
    double *hist = (double *)calloc(cycles + 1, sizeof(double));
    for (long p = 0; p < L->nn; p++) f[p] = 1.0;
    for (long g = 0; g < L->ng; g++) gq[g] = 0.5;
    or_set_rhs(P, f, gq);
    or_solve(P, u, 1e-12, cycles, hist);
    /* the single steps the tests call */
    for (int l = 0; l + 1 < P->L; l++) {
        or_level *F = &P->lev[l];
        double *r = (double *)calloc(F->nn, sizeof(double));
        double *rc = (double *)calloc(P->lev[l + 1].nn, sizeof(double));
        or_residual(P, l, F->u, F->rhs, r);
        or_extend(P, l, r);
        or_restrict(P, l, r, rc);
        or_prolong(P, l, rc, F->u);
        free(r);
        free(rc);
    }
    free(f);
    free(gq);
    free(u);
    free(hist);
    or_destroy(P);
    return 0;
}

int main(void) {
    int bad = 0;
    or_options o;
    or_default_options(&o);
    for (int mode = 0; mode < 3; mode++) {
        or_options m = o;
        m.dtau_mode = mode;
        m.dtau_const = 1.5;
        bad |= run(2, 32, circle, m, 6);
    }
    for (int sm = 0; sm < 3; sm++)
        for (int cy = 0; cy < 3; cy++) {
            or_options m = o;
            m.smoother = sm;
            m.cycle = cy;
            bad |= run(2, 16, circle, m, 3);
        }
    bad |= run(3, 16, sphere, o, 5);
    bad |= run(3, 32, spheres, o, 5);
    {
        or_options m = o;
        m.ghost_dominance = 0;
        bad |= run(3, 32, spheres, m, 3);
        m = o;
        m.bc = OR_BC_NEUMANN;
        m.reaction = 1.0;
        bad |= run(3, 16, sphere, m, 5);
        bad |= run(2, 32, circle, m, 5);
        m = o;
        m.restrict_mode = OR_RESTRICT_PLAIN_MEAN;
        bad |= run(1, 64, line1d, m, 5);
    }
    bad |= run(2, 16, one_node, o, 5);
    printf("sanitized oracle runs: %s\n", bad ? "setup failed" : "ok");
    return bad;
}
