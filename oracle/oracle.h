/*
 * Plain FP64 CPU oracle for the explicit-implicit heat-conduction scheme of
 * Ayriyan et al., "Algorithm and Simulation of Heat Conduction Process for
 * Design of a Thin Multilayer Technical Device" (arXiv 1408.5853).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; the two meet only at the
 * problem dictionary produced by the seeded generator.
 *
 * Everything is written for readability against the paper, not speed:
 * coefficients are re-evaluated per node and face, every line is assembled
 * into explicit (A, B, C, F) rows and solved with the Thomas algorithm exactly
 * as eqs. (12)-(14) state it.
 */
#ifndef CRYO_ORACLE_H
#define CRYO_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* One cell.  Arrays are per layer, inner to outer (length n_layers). */
typedef struct {
    double r_inner, height;
    int nr, nz, n_layers, heater;
    const double *thick;      /* layer thickness [m] */
    const int *intervals;     /* radial intervals per layer */
    const double *k0, *p, *kscale;   /* lambda_m(T) = kscale*k0*(T/tref)^p */
    const double *c0, *q, *rho, *tref; /* c_m(T) = c0*(T/tref)^q, rho const */
    double amplitude, width, period, t_on;  /* pulse train, eq. (4) */
    int bc_kind[4];           /* r_inner, r_outer, z_low, z_high: 0 insulated, 1 fixed */
    double bc_value[4];
    double dt;
    int turn_on;              /* eq. (22) turn-on model: 0 off, 1 on */
    const double *poly_a;     /* NULL, or [n_layers][4]: c_m(T) = sum a_k T^k, eq. (23) */
    const double *poly_b;     /* NULL, or [n_layers][5]: lambda_m(T) = kscale sum b_k T^k, eq. (24) */
    double joule_tref;        /* > 0: heater source times sqrt(joule_tref / T), eq. (25) */
    int z_full, nr_top;       /* z_full > 0: lines j > z_full span nodes 0..nr_top-1 (eq. (9)) */
} ocell;

/* node radii r_0..r_{nr-1}, eq. (9) */
int oc_radii(const ocell *c, double *r);
/* step-averaged pulse gate over [k dt, (k+1) dt), eq. (4) */
double oc_source_fraction(const ocell *c, long k);
/* source factor of sub-step i (0..99) of a pulse-start step k under the
 * turn-on model, eq. (22): gate average over the sub-step times p^2 */
double oc_turn_on_source(const ocell *c, long k, int i);
/* derivative of oc_source_fraction with respect to the pulse width [1/s] */
double oc_source_fraction_dwidth(const ocell *c, long k);
/* rows A,B,C,F (length nr) of line j for step k, from old field T [nz][nr] */
int oc_line_rows(const ocell *c, const double *T, long k, int j,
                 double *A, double *B, double *C, double *F);
/* Thomas algorithm, eqs. (12) and (14), generic rows (A[0] = C[n-1] = 0) */
int oc_thomas(int n, const double *A, const double *B, const double *C,
              const double *F, double *x);
/* One line solved the way the paper writes it out for insulated ends:
 * eq. (16) seed, eq. (12) on capacity rows, eq. (20) at interfaces,
 * eq. (17) closure, eqs. (14)/(19) back substitution. */
int oc_line_paper_sweep(const ocell *c, const double *T, long k, int j,
                        double *x);
/* advance T [nz][nr] from step k0 by nsteps steps; surf (nullable) receives
 * the surface mean after each step.  With turn_on set, each step that starts
 * a pulse runs as 100 sub-steps of dt/100 (eq. (22)); pulse starts must then
 * fall on step boundaries, else the call fails */
int oc_forward(const ocell *c, double *T, long k0, long nsteps, double *surf,
               int nthreads);
/* (with polynomial laws the adjoint takes their derivative polynomials, and
 * with the Joule source the derivative of its sqrt(tref / T) factor; with
 * the turn-on model the sub-steps are part of the sweep, and ckpt counts
 * kernel steps: sub-steps included)
 * J = sum_{n=1..N} (S_n - target_n)^2 and its gradient
 * grad = [dJ/dQ, dJ/dwidth, dJ/dthick[L], dJ/dkscale[L]] by the discrete
 * adjoint.  ckpt = 0 stores every state, else every ckpt-th with recompute.
 * lam0 (nullable, [nz][nr]) receives dJ/dT^0. */
int oc_gradient(const ocell *c, const double *T0, long nsteps,
                const double *target, long ckpt, double *J, double *grad,
                double *surf, double *lam0, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
