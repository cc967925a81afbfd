/* Runs the CPU oracle on small cells under the compiler's address and
 * undefined-behaviour checks (built by tests/test_oracle_sanitize.py):
 * forward runs on 1 and 4 threads must agree bit for bit, the adjoint with
 * checkpoints must equal the adjoint that stores every state, and every
 * variant of the problem (held and insulated walls, the solid axis, the
 * stepped domain of eq. (9), the polynomial laws and Joule source of
 * eqs. (23)-(25), the turn-on model of eq. (22)) must run clean.
 * Test infrastructure only. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static unsigned long long rng_state = 88172645463325252ull;
static double urand(void) {            /* xorshift64: deterministic inputs */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

#define L 3
static double thick[L] = {4e-4, 1e-4, 5e-4};
static int intervals[L] = {8, 4, 10};
static double k0[L] = {2.0, 0.5, 5.0}, p[L] = {1.2, 0.8, 1.5}, ks[L] = {1.0, 1.0, 1.0};
static double c0[L] = {50.0, 120.0, 80.0}, q[L] = {3.0, 3.0, 3.0};
static double rho[L] = {3e3, 2e3, 8e3}, tref[L] = {30.0, 30.0, 30.0};
static double pa[4 * L], pb[5 * L];

static ocell base_cell(void) {
    ocell c;
    memset(&c, 0, sizeof c);
    c.r_inner = 1.2e-3;
    c.height = 2e-3;
    c.nr = 23;
    c.nz = 7;
    c.n_layers = L;
    c.heater = 1;
    c.thick = thick;
    c.intervals = intervals;
    c.k0 = k0;
    c.p = p;
    c.kscale = ks;
    c.c0 = c0;
    c.q = q;
    c.rho = rho;
    c.tref = tref;
    c.amplitude = 4e9;
    c.width = 5.5e-6;
    c.period = 2e-5;
    c.t_on = 2e-6;
    c.bc_kind[0] = 1; c.bc_value[0] = 28.0;
    c.bc_kind[1] = 0;
    c.bc_kind[2] = 0;
    c.bc_kind[3] = 1; c.bc_value[3] = 29.0;
    c.dt = 1e-6;
    return c;
}

static int failures = 0;
static void check(int ok, const char *what) {
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

static void run_case(const char *name, ocell c, int with_gradient) {
    const long n = 40;
    const size_t N = (size_t)c.nz * c.nr;
    double *T0 = malloc(N * sizeof(double)), *T1 = malloc(N * sizeof(double));
    double *T4 = malloc(N * sizeof(double));
    double *S1 = malloc(n * sizeof(double)), *S4 = malloc(n * sizeof(double));
    for (size_t i = 0; i < N; ++i) T0[i] = 28.0 + 2.0 * urand();
    memcpy(T1, T0, N * sizeof(double));
    memcpy(T4, T0, N * sizeof(double));
    check(oc_forward(&c, T1, 0, n, S1, 1) == 0, name);
    check(oc_forward(&c, T4, 0, n, S4, 4) == 0, name);
    check(memcmp(T1, T4, N * sizeof(double)) == 0, "1 and 4 threads give the same field");
    check(memcmp(S1, S4, n * sizeof(double)) == 0, "1 and 4 threads give the same trace");
    for (size_t i = 0; i < N; ++i) check(isfinite(T1[i]) && T1[i] > 0, "finite field");
    if (with_gradient) {
        double *tgt = malloc(n * sizeof(double)), *lam = malloc(N * sizeof(double));
        double g0[2 + 2 * L], g5[2 + 2 * L], J0 = 0, J5 = 0;
        for (long k = 0; k < n; ++k) tgt[k] = S1[k] + 0.05 * urand();
        check(oc_gradient(&c, T0, n, tgt, 0, &J0, g0, NULL, lam, 1) == 0, name);
        check(oc_gradient(&c, T0, n, tgt, 7, &J5, g5, NULL, NULL, 4) == 0, name);
        check(J0 == J5 && memcmp(g0, g5, sizeof g0) == 0,
              "checkpointed adjoint equals the stored-states adjoint");
        for (int i = 0; i < 2 + 2 * L; ++i) check(isfinite(g0[i]), "finite gradient");
        free(tgt);
        free(lam);
    }
    printf("%s: ok\n", name);
    free(T0); free(T1); free(T4); free(S1); free(S4);
}

int main(void) {
    ocell c = base_cell();
    run_case("held inner wall, held top", c, 1);

    c = base_cell();
    c.r_inner = 0.0;                       /* solid cylinder: the axis row */
    c.bc_kind[0] = 0;
    c.bc_kind[1] = 1; c.bc_value[1] = 28.5;
    run_case("solid axis, held outer wall", c, 1);

    c = base_cell();
    c.z_full = 3;                          /* stepped domain, eq. (9) */
    c.nr_top = 12;
    run_case("stepped domain", c, 1);

    c = base_cell();
    c.turn_on = 1;                         /* eq. (22): pulse starts on step boundaries */
    run_case("turn-on model", c, 1);

    c = base_cell();
    for (int m = 0; m < L; ++m) {          /* eqs. (23), (24) near the power laws */
        pa[4 * m + 0] = 0.0;
        pa[4 * m + 1] = 0.0;
        pa[4 * m + 2] = 0.0;
        pa[4 * m + 3] = c0[m] / (30.0 * 30.0 * 30.0);
        for (int k = 0; k < 5; ++k) pb[5 * m + k] = k == 1 ? k0[m] / 30.0 : 0.0;
        pb[5 * m + 0] = 0.1 * k0[m];
    }
    c.poly_a = pa;
    c.poly_b = pb;
    c.joule_tref = 30.0;                   /* eq. (25) */
    run_case("polynomial laws, Joule source", c, 1);

    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("all ok\n");
    return 0;
}
