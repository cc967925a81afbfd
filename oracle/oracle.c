/*
 * Plain FP64 CPU oracle of the explicit-implicit scheme of arXiv 1408.5853.
 *
 * TEST INFRASTRUCTURE ONLY: it exists to check the GPU library, and only the
 * tests, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *  - Face conductivities are the layer law evaluated at the mean of the two
 *    node temperatures (Sec. 3, definitions after eq. (11)), all at the old
 *    time level (the scheme is linear per step, no iterations, Sec. 3.1).
 *  - An r-face takes the layer holding that interval; z-faces take the node's
 *    layer (layers are stacked along r).
 *  - Interface rows come from eq. (18) with the flux quotients on the new
 *    level and lambda* at the old interface temperature; they carry no heat
 *    capacity, no z-conduction and no source.  Eq. (12) applied to this row
 *    reproduces eq. (20).
 *  - Boundary rows in r follow eq. (15) (insulated) or hold the wall value
 *    (fixed).  The z-boundary lines are not solved: after all interior lines
 *    they copy their neighbour line (insulated) or hold the wall value.
 *  - The pulse gate of eq. (4) enters each step as its average over
 *    [t_k, t_k + dt); pulse times are taken in step units and snapped to the
 *    nearest integer when within 1e-9 relative.  The source is the amplitude
 *    times that average on the heater layer's capacity nodes (p(t) = 1).
 *  - Axial spacing is uniform, eta = height / (nz - 1).
 *  - Transient turn-on model (Sec. 3.2, eq. (22)), when enabled: the
 *    exponential is taken decaying, p^2(t) = 1 - exp(-(t - t_n) / (7 tau*)),
 *    so that p^2 rises from 0 towards 1 as the text describes (as printed
 *    it is negative).  Pulse n starts at t_n = t_on + n P, which must fall on
 *    a step boundary; the step [t_n, t_n + tau) is taken as 100 sub-steps of
 *    tau* = tau / 100, sub-step i with the gate averaged over the sub-step
 *    times p^2 at its start, 1 - exp(-i / 7).  All other steps are unchanged
 *    (p^2 = 1), and the surface mean is reported once per step.
 *  - Stepped domain (eq. (9): N_j radial nodes on line j), when set: lines
 *    j <= z_full span all nr nodes (the layered section up to z_0), lines
 *    above span nodes 0..nr_top-1 only (the terminal up to z_max).  The
 *    terminal's outer wall and the step face are insulated: a node of line
 *    z_full exchanges axial heat only with a capacity node above it, so the
 *    face is closed from node nr_top - 1 on (above that node sits the
 *    terminal's wall node, which only copies its neighbour); nodes outside
 *    the domain are not solved and keep their values; the surface mean runs
 *    over the lines of the layered section, z in [0, z_0].
 *  - Polynomial laws (eqs. (23), (24)), when given, replace the power laws
 *    term for term (lambda still times the layer's conductivity scale); the
 *    Joule source (eqs. (2), (25)), when enabled, multiplies the heater's
 *    source by sqrt(joule_tref / T) at the node's old temperature.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ROW_BC = 0, ROW_CAP = 1, ROW_IFACE = 2 };

typedef struct {
    int nr, L;
    double *r;    /* node radii */
    double *h;    /* h[i] = r_i - r_{i-1}, i >= 1 (eq. (9)) */
    int *lay;     /* layer of interval i (i >= 1) */
    int *kind;    /* row class of node i */
    int *mat;     /* capacity: its layer; interface: the inner layer */
    double *dr;   /* [nr][L]  d r_i / d thick_m */
    double *dh;   /* [nr][L]  d h_i / d thick_m */
} geom;

static void geom_free(geom *g)
{
    free(g->r); free(g->h); free(g->lay); free(g->kind); free(g->mat);
    free(g->dr); free(g->dh);
}

static int check_cell(const ocell *c)
{
    if (c->nr < 3 || c->nz < 3 || c->n_layers < 1) return 1;
    if (!(c->dt > 0) || !(c->height > 0) || !(c->r_inner >= 0)) return 1;
    if (c->heater < 0 || c->heater >= c->n_layers) return 1;
    if (c->width < 0 || c->period <= 0 || c->width > c->period) return 1;
    long tot = 0;
    for (int m = 0; m < c->n_layers; m++) {
        if (c->intervals[m] < 2 || !(c->thick[m] > 0)) return 1;
        tot += c->intervals[m];
    }
    if (tot != c->nr - 1) return 1;
    if (c->r_inner == 0 && c->bc_kind[0] != 0) return 1;
    if (c->z_full < 0 || c->z_full > c->nz - 2) return 1;
    if (c->z_full > 0 && (c->nr_top < 3 || c->nr_top > c->nr)) return 1;
    return 0;
}

/* eq. (9): r_{i+1} = r_i + h_{i+1}, with layer m cut into equal intervals */
static int geom_build(const ocell *c, geom *g)
{
    int nr = c->nr, L = c->n_layers;
    memset(g, 0, sizeof(*g));
    g->nr = nr; g->L = L;
    g->r = calloc(nr, sizeof(double));
    g->h = calloc(nr + 1, sizeof(double));
    g->lay = calloc(nr + 1, sizeof(int));
    g->kind = calloc(nr, sizeof(int));
    g->mat = calloc(nr, sizeof(int));
    g->dr = calloc((size_t)nr * L, sizeof(double));
    g->dh = calloc((size_t)(nr + 1) * L, sizeof(double));
    if (!g->r || !g->h || !g->lay || !g->kind || !g->mat || !g->dr || !g->dh) {
        geom_free(g);
        return 1;
    }
    int i = 0;
    for (int m = 0; m < L; m++)
        for (int k = 0; k < c->intervals[m]; k++) {
            i++;
            g->lay[i] = m;
            g->h[i] = c->thick[m] / c->intervals[m];
            g->dh[(size_t)i * L + m] = 1.0 / c->intervals[m];
        }
    g->r[0] = c->r_inner;
    for (i = 1; i < nr; i++) {
        g->r[i] = g->r[i - 1] + g->h[i];
        for (int m = 0; m < L; m++)
            g->dr[(size_t)i * L + m] = g->dr[(size_t)(i - 1) * L + m] + g->dh[(size_t)i * L + m];
    }
    g->kind[0] = g->kind[nr - 1] = ROW_BC;
    for (i = 1; i < nr - 1; i++) {
        g->mat[i] = g->lay[i];
        g->kind[i] = (g->lay[i] != g->lay[i + 1]) ? ROW_IFACE : ROW_CAP;
    }
    return 0;
}

/* sum_{k<n} coef[k] T^k, term by term */
static double poly(const double *coef, int n, double T)
{
    double s = 0.0, Tk = 1.0;
    for (int k = 0; k < n; k++) {
        s += coef[k] * Tk;
        Tk *= T;
    }
    return s;
}

/* d/dT of sum_{k<n} coef[k] T^k, term by term */
static double dpoly(const double *coef, int n, double T)
{
    double s = 0.0, Tk = 1.0;
    for (int k = 1; k < n; k++) {
        s += k * coef[k] * Tk;
        Tk *= T;
    }
    return s;
}

/* material laws: the workloads' power laws, or the polynomial fits of
 * eqs. (23) (c, cubic) and (24) (lambda, quartic) when given; and their
 * T-derivatives (the adjoint's) */
static double lam(const ocell *c, int m, double T)
{
    if (c->poly_b) return c->kscale[m] * poly(c->poly_b + 5 * m, 5, T);
    return c->kscale[m] * c->k0[m] * pow(T / c->tref[m], c->p[m]);
}
static double dlam(const ocell *c, int m, double T)
{
    if (c->poly_b) return c->kscale[m] * dpoly(c->poly_b + 5 * m, 5, T);
    return c->p[m] * lam(c, m, T) / T;
}
static double cap(const ocell *c, int m, double T)
{
    if (c->poly_a) return poly(c->poly_a + 4 * m, 4, T);
    return c->c0[m] * pow(T / c->tref[m], c->q[m]);
}
static double dcap(const ocell *c, int m, double T)
{
    if (c->poly_a) return dpoly(c->poly_a + 4 * m, 4, T);
    return c->q[m] * cap(c, m, T) / T;
}

int oc_radii(const ocell *c, double *r)
{
    geom g;
    if (check_cell(c) || geom_build(c, &g)) return 1;
    memcpy(r, g.r, sizeof(double) * c->nr);
    geom_free(&g);
    return 0;
}

static double snap(double x)
{
    double n = nearbyint(x);
    return fabs(x - n) <= 1e-9 * fmax(1.0, fabs(x)) ? n : x;
}

/* eq. (4): time the gate nu(t) = 1 on [t_on + nP, t_on + nP + w) is open
 * within [lo, hi), all in step units */
static double gate_overlap(const ocell *c, double lo, double hi)
{
    if (!(c->width > 0)) return 0.0;
    double b0 = snap(c->t_on / c->dt), W = snap(c->width / c->dt);
    double P = snap(c->period / c->dt);
    double s = 0.0;
    long n = (long)floor((lo - b0 - W) / P);
    if (n < 0) n = 0;
    for (;; n++) {
        double b = b0 + n * P, e = b + W;
        if (b >= hi) break;
        double o = fmin(hi, e) - fmax(lo, b);
        if (o > 0) s += o;
    }
    return s;
}

/* eq. (4) averaged over step k */
double oc_source_fraction(const ocell *c, long k)
{
    return gate_overlap(c, (double)k, (double)k + 1.0);
}

/* eq. (22): does step k start a pulse (t_on + n P = k dt)?  -1 when the
 * model is on but pulse starts do not fall on step boundaries */
static int pulse_start(const ocell *c, long k)
{
    double b0 = snap(c->t_on / c->dt), P = snap(c->period / c->dt);
    if (b0 != floor(b0) || P != floor(P) || !(P >= 1)) return -1;
    long kb = (long)b0, kp = (long)P;
    return k >= kb && (k - kb) % kp == 0;
}

/* source factor of sub-step i of a pulse-start step k: the gate's average
 * over [k + i/100, k + (i+1)/100) times p^2 = 1 - exp(-i/7) (eq. (22)) */
double oc_turn_on_source(const ocell *c, long k, int i)
{
    double lo = (double)k + (double)i / 100.0, hi = (double)k + (double)(i + 1) / 100.0;
    return gate_overlap(c, lo, hi) / (hi - lo) * (1.0 - exp(-(double)i / 7.0));
}

/* its derivative with respect to the pulse width [1/s]: a pulse end inside
 * the sub-step counts fully, one on its boundary half (as for whole steps) */
static double turn_on_source_dwidth(const ocell *c, long k, int i)
{
    if (!(c->width > 0)) return 0.0;
    double b0 = snap(c->t_on / c->dt), W = snap(c->width / c->dt);
    double P = snap(c->period / c->dt);
    double lo = (double)k + (double)i / 100.0, hi = (double)k + (double)(i + 1) / 100.0, d = 0.0;
    long n = (long)floor((lo - b0 - W) / P);
    if (n < 0) n = 0;
    for (;; n++) {
        double b = b0 + n * P, e = b + W;
        if (b >= hi) break;
        if (e > lo && e < hi) d += 1.0;
        else if (e == lo || e == hi) d += 0.5;
    }
    return d / ((hi - lo) * c->dt) * (1.0 - exp(-(double)i / 7.0));
}

/* d/d(width) of the step average: 1/dt while a pulse ends inside the step,
 * half of that on each side when it ends exactly on a step boundary (the
 * mean of the one-sided derivatives, which a central difference sees) */
double oc_source_fraction_dwidth(const ocell *c, long k)
{
    if (!(c->width > 0)) return 0.0;
    double b0 = snap(c->t_on / c->dt), W = snap(c->width / c->dt);
    double P = snap(c->period / c->dt);
    double lo = (double)k, hi = (double)k + 1.0, d = 0.0;
    long n = (long)floor((lo - b0 - W) / P);
    if (n < 0) n = 0;
    for (;; n++) {
        double b = b0 + n * P, e = b + W;
        if (b >= hi) break;
        if (e > lo && e < hi) d += 1.0;
        else if (e == lo || e == hi) d += 0.5;
    }
    return d / c->dt;
}

/* radial node count N_j of line j (eq. (9)) */
static int line_len(const ocell *c, int j)
{
    return (c->z_full > 0 && j > c->z_full) ? c->nr_top : c->nr;
}

/* Rows of eq. (13) for line j (capacity), eq. (18) (interface), eq. (15)
 * (r boundaries); the explicit z operator eq. (11) sits in F. */
static void line_rows(const ocell *c, const geom *g, const double *T, double tau,
                      double s, int j, double *A, double *B, double *C, double *F)
{
    int nr = c->nr, n = line_len(c, j);
    double eta = c->height / (c->nz - 1);
    const double *Tj = T + (size_t)j * nr;
    const double *Tn = Tj + nr, *Ts = Tj - nr;
    const double *r = g->r, *h = g->h;
    for (int i = 1; i < n - 1; i++) {
        if (g->kind[i] == ROW_CAP) {
            int m = g->mat[i];
            double lw = lam(c, m, 0.5 * (Tj[i] + Tj[i - 1]));   /* lambda_{i-1/2,j} */
            double le = lam(c, m, 0.5 * (Tj[i] + Tj[i + 1]));   /* lambda_{i+1/2,j} */
            double rw = 0.5 * (r[i] + r[i - 1]);                 /* r_{i-1/2} */
            double re = 0.5 * (r[i] + r[i + 1]);                 /* r_{i+1/2} */
            double hb = 0.5 * (h[i + 1] + h[i]);                 /* hbar_i */
            double rc = c->rho[m] * cap(c, m, Tj[i]) / tau;
            A[i] = -rw * lw / (r[i] * hb * h[i]);
            C[i] = -re * le / (r[i] * hb * h[i + 1]);
            B[i] = (rw * lw / h[i] + re * le / h[i + 1]) / (r[i] * hb) + rc;
            double ln = lam(c, m, 0.5 * (Tj[i] + Tn[i]));       /* lambda_{i,j+1/2} */
            /* the step face: no capacity node above */
            if (c->z_full > 0 && j == c->z_full && i >= c->nr_top - 1) ln = 0.0;
            double ls = lam(c, m, 0.5 * (Tj[i] + Ts[i]));       /* lambda_{i,j-1/2} */
            double Lz = (ln * (Tn[i] - Tj[i]) / eta - ls * (Tj[i] - Ts[i]) / eta) / eta;
            double X = (m == c->heater) ? c->amplitude * s : 0.0;
            /* Joule heating, eqs. (2), (25): resistivity proportional to
             * T^(-1/2), taken at the old level like every coefficient */
            if (c->joule_tref > 0) X *= sqrt(c->joule_tref / Tj[i]);
            F[i] = rc * Tj[i] + Lz + X;
        } else {
            int a = g->mat[i], b = a + 1;
            double la = lam(c, a, Tj[i]), lb = lam(c, b, Tj[i]);  /* lambda*_m, lambda*_{m+1} */
            A[i] = -la * h[i + 1];
            B[i] = la * h[i + 1] + lb * h[i];
            C[i] = -lb * h[i];
            F[i] = 0.0;
        }
    }
    A[0] = 0.0; B[0] = 1.0;
    if (c->bc_kind[0] == 0) { C[0] = -1.0; F[0] = 0.0; }
    else { C[0] = 0.0; F[0] = c->bc_value[0]; }
    C[n - 1] = 0.0; B[n - 1] = 1.0;
    /* the terminal's wall is insulated; the layered section's as given */
    if (c->bc_kind[1] == 0 || (c->z_full > 0 && j > c->z_full)) { A[n - 1] = -1.0; F[n - 1] = 0.0; }
    else { A[n - 1] = 0.0; F[n - 1] = c->bc_value[1]; }
}

int oc_line_rows(const ocell *c, const double *T, long k, int j,
                 double *A, double *B, double *C, double *F)
{
    geom g;
    if (check_cell(c) || j < 1 || j > c->nz - 2 || geom_build(c, &g)) return 1;
    line_rows(c, &g, T, c->dt, oc_source_fraction(c, k), j, A, B, C, F);
    geom_free(&g);
    return 0;
}

/* eq. (12) forward sweep, eq. (14) back substitution */
static void thomas(int n, const double *A, const double *B, const double *C,
                   const double *F, double *al, double *be, double *x)
{
    double ap = 0.0, bp = 0.0;
    for (int i = 0; i < n; i++) {
        double den = B[i] + A[i] * ap;
        al[i] = -C[i] / den;
        be[i] = (F[i] - A[i] * bp) / den;
        ap = al[i];
        bp = be[i];
    }
    x[n - 1] = be[n - 1];
    for (int i = n - 2; i >= 0; i--) x[i] = al[i] * x[i + 1] + be[i];
}

int oc_thomas(int n, const double *A, const double *B, const double *C,
              const double *F, double *x)
{
    if (n < 1) return 1;
    double *w = malloc(sizeof(double) * 2 * n);
    if (!w) return 1;
    thomas(n, A, B, C, F, w, w + n, x);
    free(w);
    return 0;
}

int oc_line_paper_sweep(const ocell *c, const double *T, long k, int j, double *x)
{
    geom g;
    if (check_cell(c) || c->bc_kind[0] != 0 || c->bc_kind[1] != 0) return 1;
    if (j < 1 || j > c->nz - 2 || geom_build(c, &g)) return 1;
    int nr = c->nr;
    double *A = malloc(sizeof(double) * 6 * nr);
    if (!A) { geom_free(&g); return 1; }
    double *B = A + nr, *C = B + nr, *F = C + nr, *al = F + nr, *be = al + nr;
    line_rows(c, &g, T, c->dt, oc_source_fraction(c, k), j, A, B, C, F);
    const double *Tj = T + (size_t)j * nr;
    al[0] = 1.0; be[0] = 0.0;                                   /* eq. (16) */
    for (int i = 1; i < nr - 1; i++) {
        if (g.kind[i] == ROW_IFACE) {                           /* eq. (20) */
            int a = g.mat[i], b = a + 1;
            double la = lam(c, a, Tj[i]), lb = lam(c, b, Tj[i]);
            double D = lb * g.h[i] + la * g.h[i + 1] * (1.0 - al[i - 1]);
            al[i] = lb * g.h[i] / D;
            be[i] = la * g.h[i + 1] * be[i - 1] / D;
        } else {                                                /* eq. (12) */
            double den = B[i] + A[i] * al[i - 1];
            al[i] = -C[i] / den;
            be[i] = (F[i] - A[i] * be[i - 1]) / den;
        }
    }
    x[nr - 1] = be[nr - 2] / (1.0 - al[nr - 2]);                /* eq. (17) */
    for (int i = nr - 2; i >= 1; i--) x[i] = al[i] * x[i + 1] + be[i];  /* (14),(19) */
    x[0] = x[1];                                                /* eq. (15) */
    free(A);
    geom_free(&g);
    return 0;
}

/* z-boundary lines after the interior solve: copy (insulated) or hold */
static void z_boundaries(const ocell *c, double *T)
{
    int nr = c->nr, nz = c->nz;
    if (c->bc_kind[2] == 0) memcpy(T, T + nr, sizeof(double) * nr);
    else for (int i = 0; i < nr; i++) T[i] = c->bc_value[2];
    double *top = T + (size_t)(nz - 1) * nr;
    if (c->bc_kind[3] == 0) memcpy(top, top - nr, sizeof(double) * nr);
    else for (int i = 0; i < nr; i++) top[i] = c->bc_value[3];
}

/* weight of line j in the surface mean: trapezoid over lines 0..J (J the
 * last line of the layered section), normalised to 1 */
static double surface_weight(const ocell *c, int j)
{
    int J = c->z_full > 0 ? c->z_full : c->nz - 1;
    if (j > J) return 0.0;
    return ((j == 0 || j == J) ? 0.5 : 1.0) / J;
}

/* trapezoid weights along the outer surface r = r_max (lines 0..J, J the
 * last line of the layered section), normalised to 1 */
static double surface_mean(const ocell *c, const double *T)
{
    int nr = c->nr, J = c->z_full > 0 ? c->z_full : c->nz - 1;
    double s = 0.0;
    for (int j = 0; j <= J; j++) {
        double w = (j == 0 || j == J) ? 0.5 : 1.0;
        s += w * T[(size_t)j * nr + nr - 1];
    }
    return s / J;
}

typedef struct { double *A, *B, *C, *F, *al, *be, *wa, *wb; } rows_t;

static int nthreads_of(int n)
{
#ifdef _OPENMP
    return n > 0 ? n : omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

static int thread_id(void)
{
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

/* one step of eq. (8) of length tau with gate factor s: T (old) -> Tn (new);
 * scratch per thread */
static void step_tau(const ocell *c, const geom *g, const double *T, double *Tn,
                     double tau, double s, rows_t *scr, int nth)
{
    int nr = c->nr, nz = c->nz;
#pragma omp parallel for num_threads(nth) schedule(static)
    for (int j = 1; j < nz - 1; j++) {
        rows_t *w = &scr[thread_id()];
        int n = line_len(c, j);
        line_rows(c, g, T, tau, s, j, w->A, w->B, w->C, w->F);
        thomas(n, w->A, w->B, w->C, w->F, w->al, w->be, Tn + (size_t)j * nr);
        for (int i = n; i < nr; i++) Tn[(size_t)j * nr + i] = T[(size_t)j * nr + i];
    }
    z_boundaries(c, Tn);
}

/* step k (p^2 = 1) */
static void step(const ocell *c, const geom *g, const double *T, double *Tn,
                 long k, rows_t *scr, int nth)
{
    step_tau(c, g, T, Tn, c->dt, oc_source_fraction(c, k), scr, nth);
}

static rows_t *scratch_alloc(int nth, int nr)
{
    rows_t *s = calloc(nth, sizeof(rows_t));
    if (!s) return NULL;
    for (int t = 0; t < nth; t++) {
        double *p = malloc(sizeof(double) * 8 * nr);
        if (!p) return NULL;
        s[t].A = p; s[t].B = p + nr; s[t].C = p + 2 * nr; s[t].F = p + 3 * nr;
        s[t].al = p + 4 * nr; s[t].be = p + 5 * nr;
        s[t].wa = p + 6 * nr; s[t].wb = p + 7 * nr;
    }
    return s;
}

static void scratch_free(rows_t *s, int nth)
{
    if (!s) return;
    for (int t = 0; t < nth; t++) free(s[t].A);
    free(s);
}

int oc_forward(const ocell *c, double *T, long k0, long nsteps, double *surf,
               int nthreads)
{
    geom g;
    if (check_cell(c) || nsteps < 0) return 1;
    if (c->turn_on && c->width > 0 && pulse_start(c, 0) < 0) return 1;
    if (geom_build(c, &g)) return 1;
    size_t n = (size_t)c->nr * c->nz;
    int nth = nthreads_of(nthreads);
    double *Tn = malloc(sizeof(double) * n);
    rows_t *scr = scratch_alloc(nth, c->nr);
    if (!Tn || !scr) { free(Tn); scratch_free(scr, nth); geom_free(&g); return 1; }
    for (long s = 0; s < nsteps; s++) {
        long k = k0 + s;
        if (c->turn_on && c->width > 0 && pulse_start(c, k) == 1) {
            /* eq. (22): the pulse's first step as 100 sub-steps */
            for (int i = 0; i < 100; i++) {
                step_tau(c, &g, T, Tn, c->dt / 100.0, oc_turn_on_source(c, k, i), scr, nth);
                memcpy(T, Tn, sizeof(double) * n);
            }
        } else {
            step(c, &g, T, Tn, k, scr, nth);
            memcpy(T, Tn, sizeof(double) * n);
        }
        if (surf) surf[s] = surface_mean(c, T);
    }
    free(Tn);
    scratch_free(scr, nth);
    geom_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------
 * Discrete adjoint.  The step maps T^n -> T^{n+1} through, per interior line,
 * the residual r = A(T^n) T^{n+1} - F(T^n) = 0, plus the z-boundary copies.
 * J = sum_{n=1..N} (S_n - target_n)^2 with S the surface mean.
 * With lam^{n+1} = dJ/dT^{n+1}:
 *   mu   = lam^{n+1} on interior lines, plus the boundary lines' entries
 *          moved onto the lines they copy,
 *   y_j  = A_j^{-T} mu_j (transposed tridiagonal solve per line),
 *   lam^n = dJ_n/dT^n - sum_j (dr_j/dT^n)^T y_j,
 *   dJ/dtheta -= sum_j y_j^T dr_j/dtheta.
 * ---------------------------------------------------------------------- */

typedef struct {
    const ocell *c;
    const geom *g;
    int L, ng;
} adj_ctx;

/* contributions of line j's rows; lamn rows j-1..j+1 updated; gl = grad part */
static void adjoint_line(const adj_ctx *x, const double *T, const double *Tn,
                         double tau, double s, double sd, int j, const double *y,
                         double *lamn, double *gl)
{
    const ocell *c = x->c;
    const geom *g = x->g;
    int nr = c->nr, L = x->L;
    double eta = c->height / (c->nz - 1), e2 = eta * eta;
    const double *Tj = T + (size_t)j * nr, *Tnn = Tj + nr, *Tss = Tj - nr;
    const double *X = Tn + (size_t)j * nr;   /* new values of line j */
    double *lj = lamn + (size_t)j * nr, *ln_ = lj + nr, *ls_ = lj - nr;
    const double *r = g->r, *h = g->h;
    int n = line_len(c, j);
    for (int i = 1; i < n - 1; i++) {
        double yi = y[i];
        if (yi == 0.0) continue;
        double Dw = X[i] - X[i - 1], De = X[i] - X[i + 1];
        if (g->kind[i] == ROW_CAP) {
            int m = g->mat[i];
            double Tw = 0.5 * (Tj[i] + Tj[i - 1]), Te = 0.5 * (Tj[i] + Tj[i + 1]);
            double lw = lam(c, m, Tw), le = lam(c, m, Te);
            double dlw = dlam(c, m, Tw), dle = dlam(c, m, Te);
            double rw = 0.5 * (r[i] + r[i - 1]), re = 0.5 * (r[i] + r[i + 1]);
            double hb = 0.5 * (h[i + 1] + h[i]);
            double aw = rw / (r[i] * hb * h[i]), ae = re / (r[i] * hb * h[i + 1]);
            double rc = c->rho[m] * cap(c, m, Tj[i]) / tau;
            double drc = c->rho[m] * dcap(c, m, Tj[i]) / tau;
            double Tzn = 0.5 * (Tj[i] + Tnn[i]), Tzs = 0.5 * (Tj[i] + Tss[i]);
            double lzn = lam(c, m, Tzn), lzs = lam(c, m, Tzs);
            double dlzn = dlam(c, m, Tzn), dlzs = dlam(c, m, Tzs);
            if (c->z_full > 0 && j == c->z_full && i >= c->nr_top - 1)
                lzn = dlzn = 0.0;                                    /* the step face */
            double gn = Tnn[i] - Tj[i], gs = Tj[i] - Tss[i];
            double Lz = (lzn * gn - lzs * gs) / e2;
            double dLn = (0.5 * dlzn * gn + lzn) / e2;               /* dLz/dT_{j+1} */
            double dLc = (0.5 * dlzn * gn - lzn - 0.5 * dlzs * gs - lzs) / e2;
            double dLs = (-0.5 * dlzs * gs + lzs) / e2;              /* dLz/dT_{j-1} */
            /* residual r = aw lw Dw + ae le De + rc (X_i - T_i) - Lz - Q s chi */
            lj[i - 1] -= yi * aw * Dw * 0.5 * dlw;
            lj[i + 1] -= yi * ae * De * 0.5 * dle;
            lj[i] -= yi * (aw * Dw * 0.5 * dlw + ae * De * 0.5 * dle
                           + drc * (X[i] - Tj[i]) - rc - dLc);
            ln_[i] -= yi * (-dLn);
            ls_[i] -= yi * (-dLs);
            if (m == c->heater) {
                /* the source Q s chi(T_i), chi = sqrt(tref / T_i) with the
                 * Joule source of eq. (25), else 1; its T_i-derivative
                 * -chi / (2 T_i) enters lam^n */
                double chi = 1.0;
                if (c->joule_tref > 0) {
                    chi = sqrt(c->joule_tref / Tj[i]);
                    lj[i] -= yi * 0.5 * c->amplitude * s * chi / Tj[i];
                }
                gl[0] += yi * s * chi;
                gl[1] += yi * c->amplitude * sd * chi;
            }
            gl[2 + L + m] -= yi * (aw * lw * Dw + ae * le * De - Lz) / c->kscale[m];
            for (int l = 0; l < L; l++) {
                double dri = g->dr[(size_t)i * L + l];
                double drw = 0.5 * (dri + g->dr[(size_t)(i - 1) * L + l]);
                double dre = 0.5 * (dri + g->dr[(size_t)(i + 1) * L + l]);
                double dhi = g->dh[(size_t)i * L + l], dhe = g->dh[(size_t)(i + 1) * L + l];
                double dhb = 0.5 * (dhi + dhe);
                double daw = aw * (drw / rw - dri / r[i] - dhb / hb - dhi / h[i]);
                double dae = ae * (dre / re - dri / r[i] - dhb / hb - dhe / h[i + 1]);
                gl[2 + l] -= yi * (daw * lw * Dw + dae * le * De);
            }
        } else {
            int a = g->mat[i], b = a + 1;
            double la = lam(c, a, Tj[i]), lb = lam(c, b, Tj[i]);
            double dla = dlam(c, a, Tj[i]), dlb = dlam(c, b, Tj[i]);
            /* residual r = la h_{i+1} Dw + lb h_i De */
            lj[i] -= yi * (dla * h[i + 1] * Dw + dlb * h[i] * De);
            gl[2 + L + a] -= yi * la * h[i + 1] * Dw / c->kscale[a];
            gl[2 + L + b] -= yi * lb * h[i] * De / c->kscale[b];
            for (int l = 0; l < L; l++)
                gl[2 + l] -= yi * (la * g->dh[(size_t)(i + 1) * L + l] * Dw
                                   + lb * g->dh[(size_t)i * L + l] * De);
        }
    }
}

/* The launches of a run of N steps: one per step, or the 100 sub-steps of a
 * pulse-start step under the turn-on model (eq. (22)).  Each has its time
 * step, source factor, its width derivative, and the step whose surface is
 * observed after it (1..N; 0 for none). */
typedef struct { double tau, s, sd; long obs; } launch_t;

static long launches(const ocell *c, long N, launch_t *out)
{
    long m = 0;
    for (long k = 0; k < N; k++) {
        if (c->turn_on && c->width > 0 && pulse_start(c, k) == 1) {
            for (int i = 0; i < 100; i++, m++)
                if (out) {
                    out[m].tau = c->dt / 100.0;
                    out[m].s = oc_turn_on_source(c, k, i);
                    out[m].sd = turn_on_source_dwidth(c, k, i);
                    out[m].obs = i == 99 ? k + 1 : 0;
                }
        } else {
            if (out) {
                out[m].tau = c->dt;
                out[m].s = oc_source_fraction(c, k);
                out[m].sd = oc_source_fraction_dwidth(c, k);
                out[m].obs = k + 1;
            }
            m++;
        }
    }
    return m;
}

int oc_gradient(const ocell *c, const double *T0, long N, const double *target,
                long ckpt, double *J, double *grad, double *surf, double *lam0,
                int nthreads)
{
    geom g;
    if (check_cell(c) || N < 1 || geom_build(c, &g))
        return 1;
    if (c->turn_on && c->width > 0 && pulse_start(c, 0) < 0) { geom_free(&g); return 1; }
    int nr = c->nr, nz = c->nz, L = c->n_layers, ng = 2 + 2 * L;
    size_t n = (size_t)nr * nz;
    long M = launches(c, N, NULL);
    launch_t *lh = malloc(sizeof(launch_t) * M);
    long K = ckpt > 0 ? ckpt : M;
    long nseg = (M + K - 1) / K;
    int nth = nthreads_of(nthreads);
    int rc_ = 1;
    double *ck = malloc(sizeof(double) * n * nseg);
    double *seg = malloc(sizeof(double) * n * (K + 1));
    double *S = malloc(sizeof(double) * (N + 1));
    double *lam_ = calloc(n, sizeof(double)), *lamn = calloc(n, sizeof(double));
    double *mu = calloc(n, sizeof(double)), *Y = calloc(n, sizeof(double));
    double *gl = calloc((size_t)nz * ng, sizeof(double));
    rows_t *scr = scratch_alloc(nth, nr);
    if (!lh || !ck || !seg || !S || !lam_ || !lamn || !mu || !Y || !gl || !scr) goto out;
    launches(c, N, lh);

    /* forward sweep over the launches with checkpoints */
    double *Tc = seg, *Tt = seg + n;
    memcpy(Tc, T0, sizeof(double) * n);
    double Jv = 0.0;
    for (long l = 0; l < M; l++) {
        if (l % K == 0) memcpy(ck + n * (l / K), Tc, sizeof(double) * n);
        step_tau(c, &g, Tc, Tt, lh[l].tau, lh[l].s, scr, nth);
        memcpy(Tc, Tt, sizeof(double) * n);
        long o = lh[l].obs;
        if (o > 0) {
            S[o] = surface_mean(c, Tc);
            if (surf) surf[o - 1] = S[o];
            double d = S[o] - target[o - 1];
            Jv += d * d;
        }
    }
    *J = Jv;
    for (int q = 0; q < ng; q++) grad[q] = 0.0;

    /* lam^M = dJ_N / dT^M (the last launch observes step N) */
    for (int j = 0; j < nz; j++)
        lam_[(size_t)j * nr + nr - 1] = 2.0 * (S[N] - target[N - 1]) * surface_weight(c, j);
    adj_ctx ax = { c, &g, L, ng };
    for (long sg = nseg - 1; sg >= 0; sg--) {
        long a = sg * K, b = (a + K < M) ? a + K : M;
        memcpy(seg, ck + n * sg, sizeof(double) * n);
        for (long l = a; l < b; l++)
            step_tau(c, &g, seg + n * (l - a), seg + n * (l - a + 1), lh[l].tau, lh[l].s, scr, nth);
        for (long l = b - 1; l >= a; l--) {
            const double *T = seg + n * (l - a), *Tn = seg + n * (l - a + 1);
            double tau = lh[l].tau, s = lh[l].s, sd = lh[l].sd;
            /* move the copied boundary lines' sensitivities onto their sources */
            memcpy(mu, lam_, sizeof(double) * n);
            if (c->bc_kind[2] == 0)
                for (int i = 0; i < nr; i++) mu[nr + i] += lam_[i];
            if (c->bc_kind[3] == 0)
                for (int i = 0; i < nr; i++)
                    mu[(size_t)(nz - 2) * nr + i] += lam_[(size_t)(nz - 1) * nr + i];
            /* transposed line solves */
#pragma omp parallel for num_threads(nth) schedule(static)
            for (int j = 1; j < nz - 1; j++) {
                rows_t *w = &scr[thread_id()];
                int ln = line_len(c, j);
                line_rows(c, &g, T, tau, s, j, w->A, w->B, w->C, w->F);
                /* A^T: sub-diagonal C_{i-1}, diagonal B_i, super-diagonal A_{i+1} */
                double *sub = w->F, *sup = w->al;
                sub[0] = 0.0;
                for (int i = 1; i < ln; i++) sub[i] = w->C[i - 1];
                for (int i = 0; i < ln - 1; i++) sup[i] = w->A[i + 1];
                sup[ln - 1] = 0.0;
                thomas(ln, sub, w->B, sup, mu + (size_t)j * nr, w->wa, w->wb,
                       Y + (size_t)j * nr);
                /* nodes outside the domain keep their values: no equation */
                for (int i = ln; i < nr; i++) Y[(size_t)j * nr + i] = 0.0;
            }
            /* the state before launch l is observed when launch l-1 ends a step */
            memset(lamn, 0, sizeof(double) * n);
            long o = l >= 1 ? lh[l - 1].obs : 0;
            if (o > 0)
                for (int j = 0; j < nz; j++)
                    lamn[(size_t)j * nr + nr - 1] = 2.0 * (S[o] - target[o - 1]) * surface_weight(c, j);
            memset(gl, 0, sizeof(double) * nz * ng);
            /* lines three apart touch disjoint rows of lamn */
            for (int phase = 0; phase < 3; phase++) {
#pragma omp parallel for num_threads(nth) schedule(static)
                for (int j = 1 + phase; j < nz - 1; j += 3)
                    adjoint_line(&ax, T, Tn, tau, s, sd, j, Y + (size_t)j * nr, lamn,
                                 gl + (size_t)j * ng);
            }
            for (int j = 1; j < nz - 1; j++)
                for (int q = 0; q < ng; q++) grad[q] += gl[(size_t)j * ng + q];
            double *t = lam_; lam_ = lamn; lamn = t;
        }
    }
    if (lam0) memcpy(lam0, lam_, sizeof(double) * n);
    rc_ = 0;
out:
    free(lh); free(ck); free(seg); free(S); free(lam_); free(lamn); free(mu); free(Y);
    free(gl);
    scratch_free(scr, nth);
    geom_free(&g);
    return rc_;
}
