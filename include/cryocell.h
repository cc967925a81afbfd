/*
 * cryocell — time stepping of the pulsed, nonlinear heat equation in a
 * multilayer cylindrical (r, z) cell on one AMD Instinct MI355X (gfx950),
 * with the explicit-implicit finite-difference scheme of
 *   A. Ayriyan, J. Busa Jr., E. E. Donets, H. Grigorian, J. Pribis,
 *   "Algorithm and Simulation of Heat Conduction Process for Design of a
 *   Thin Multilayer Technical Device", arXiv:1408.5853.
 *
 * The problem is the paper's Sec. 2: eq. (1) with layer-wise material laws,
 * a periodic rectangular heating pulse (eqs. (2)-(4)), a uniform initial
 * temperature (eq. (5)), insulated or held boundaries (eq. (6)) and ideal
 * contact between layers (eq. (7)).  The scheme is Sec. 3: eq. (8) with the
 * r operator (10) implicit and the z operator (11) explicit, coefficients at
 * the old time level, one tridiagonal system per axial line (eqs. (12)-(14),
 * (16), (17)), interface rows from eqs. (18)-(20), and the explicit stability
 * bound (21).
 *
 * Units are SI throughout (m, s, K, W/m/K, J/kg/K, kg/m^3, W/m^3).
 *
 * Conventions shared by every call:
 *  - Status: every call returns cryo_status; CRYO_OK is 0.  On failure
 *    cryo_last_error() returns a thread-local message; nothing is thrown.
 *  - Ownership: descriptors are copied at create time.  The library owns only
 *    its opaque plan/batch objects, their host tables and a small read-only
 *    device copy of the per-radius tables (O(nr) bytes), made by the first
 *    call that runs on the device, on the device current then.  The
 *    temperature fields, the workspace and all outputs are device memory
 *    owned by the caller; the library allocates nothing on the step path.
 *  - Streams: `stream` is a hipStream_t passed as void*; NULL is the null
 *    stream.  All device work of a call is enqueued on that stream and the
 *    call returns without waiting, except where noted.  Buffers must stay
 *    alive until the stream reaches the end of the call's work.
 *  - Field layout: a CRYO_F64 temperature field is a dense row-major double
 *    array [nz][nr], r contiguous, so one radial line (one tridiagonal
 *    system) is one row.  A CRYO_F32 field is a compensated pair of such
 *    planes, float [2][nz][nr]: plane 0 holds T rounded to float and plane 1
 *    the residual T - plane0 (at most half an ulp of plane 0).  Arithmetic of
 *    an F32 plan is FP32; the pair only carries the state, because a lone
 *    float cannot accumulate per-step increments far below its ulp.
 */
#ifndef CRYOCELL_H
#define CRYOCELL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CRYO_OK = 0,
    CRYO_ERR_ARG = 1,          /* malformed descriptor or argument */
    CRYO_ERR_UNSTABLE = 2,     /* dt violates the explicit bound, eq. (21) */
    CRYO_ERR_DEVICE = 3,       /* a HIP runtime call failed */
    CRYO_ERR_NONFINITE = 4,    /* a non-finite temperature, or one outside
                                  [1/16 K, 2^20 K), was produced */
    CRYO_ERR_WORKSPACE = 5,    /* workspace missing or too small */
    CRYO_ERR_UNSUPPORTED = 6   /* valid problem outside the built kernels' range */
} cryo_status;

typedef enum { CRYO_F64 = 0, CRYO_F32 = 1 } cryo_dtype;

/* Boundary kinds of eq. (6): zero normal derivative, or a held temperature. */
typedef enum { CRYO_INSULATED = 0, CRYO_HELD = 1 } cryo_bc_kind;

/* Material laws of one layer (the workloads' power-law families standing in
 * for the paper's polynomial fits, eqs. (23)-(24)):
 *   lambda(T) = k_scale * k0 * (T / tref)^p     [W/m/K]
 *   c(T)      = c0 * (T / tref)^q               [J/kg/K],  rho constant. */
typedef struct {
    double k0, p, k_scale;
    double c0, q;
    double rho, tref;
} cryo_material;

/* One radial layer, listed inner to outer (Sec. 2: cooler, insulator,
 * heater, outer insulator, ...).  `intervals` >= 2 equal radial intervals. */
typedef struct {
    double thickness;
    int32_t intervals;
    cryo_material mat;
} cryo_layer;

/* The cell (eq. (9) grid): radial nodes r_0 = r_inner, then each layer cut
 * into equal intervals, nr = 1 + sum(intervals); axial nodes uniform over
 * [0, height], nz of them.  Node counts include the boundary nodes. */
typedef struct {
    double r_inner;            /* >= 0; 0 only with an insulated inner side */
    double height;
    int32_t nr, nz;            /* 3 <= nr <= 2048, nz >= 3 */
    int32_t n_layers;          /* 1..16 */
    const cryo_layer *layers;  /* n_layers entries, copied */
} cryo_geometry;

/* Heating pulse (eqs. (2)-(4) with p(t) = 1): volumetric source `amplitude`
 * on the heater layer's interior nodes while t - t_on lies in
 * [n period, n period + width) for some integer n >= 0.  Each step uses the
 * gate's average over [t_k, t_k + dt); t_k = k dt. */
typedef struct {
    int32_t layer;
    double amplitude, width, period, t_on;
} cryo_pulse;

/* Sides in the order r_inner, r_outer, z_low, z_high. */
typedef struct {
    int32_t kind[4];
    double value[4];
} cryo_boundary;

typedef struct {
    cryo_geometry geom;
    cryo_pulse pulse;
    cryo_boundary bc;
    double dt;                 /* time step tau */
    double T_init;             /* eq. (5) */
} cryo_problem;

typedef struct cryo_plan cryo_plan;
typedef struct cryo_batch cryo_batch;

/* Thread-local text of the last failure (never NULL). */
const char *cryo_last_error(void);

/* Library version string. */
const char *cryo_version(void);

/* Host-only check of a descriptor: geometry, layer counts, laws, pulse and
 * boundary kinds; T_init and held wall values must lie in the temperature
 * range of the FP64 law tables, [1/16 K, 2^20 K).  Law exponents (each
 * layer's p and q, and p_m - p_{m+1} of neighbouring layers) must lie where
 * the FP64 table powers' series truncation stays within 1e-14 relative,
 * about -5.3 <= e <= 12.5 (CRYO_ERR_UNSUPPORTED otherwise).  Does not test
 * stability.  No device calls. */
cryo_status cryo_validate(const cryo_problem *prob);

/* Largest dt allowed by the explicit z half, eq. (21):
 *   dt_max = (eta^2 / 2) * min over layers of rho c(T) / lambda(T)
 * evaluated at temperature T_min (> 0).  No device calls. */
cryo_status cryo_stability_dt_max(const cryo_problem *prob, double T_min,
                                  double *dt_max);

/* Create a plan: validates `prob`, rejects dt above eq. (21)'s bound at the
 * coldest prescribed temperature (min of T_init and held wall values) with
 * CRYO_ERR_UNSTABLE, and builds the grid tables.  Host only.  `dtype`
 * selects the field type (double or float). */
cryo_status cryo_plan_create(const cryo_problem *prob, cryo_dtype dtype,
                             cryo_plan **out);
void cryo_plan_destroy(cryo_plan *plan);

/* Launch shape of the stepping kernel: radial rows per lane, waves (of 64
 * lanes) per radial line, and interior lines marched by one line group per
 * step.  The plan picks one at create time; cryo_plan_set_shape overrides it
 * (the autotuner's hook) and must precede the plan's first device call.
 * Built shapes: one wave per line with 2, 3, 4, 5, 6, 7, 8, 10, 12 or 16
 * rows per lane, and (4,2) (8,2) (4,4) (8,4); 64 * waves * rows must cover
 * nr.  The gradient runs (2,1) (4,1) (8,1) (4,2) (8,2) (4,4) (8,4).  Other
 * shapes, lines per wave included, change only rounding: the chunks of the
 * line solve, and the order in which a line adds its two axial fluxes (its
 * line block's march direction), depend on the shape. */
cryo_status cryo_plan_shape(const cryo_plan *plan, int32_t *rows_per_lane,
                            int32_t *waves_per_line, int32_t *lines_per_wave);
cryo_status cryo_plan_set_shape(cryo_plan *plan, int32_t rows_per_lane,
                                int32_t waves_per_line, int32_t lines_per_wave);

/* Host copy of the node radii r_0..r_{nr-1} (eq. (9)). */
cryo_status cryo_grid_radii(const cryo_plan *plan, double *r);

/* Host copy of the per-step pulse averages s_k, k = k0..k0+n-1 (eq. (4)). */
cryo_status cryo_source_fraction(const cryo_plan *plan, int64_t k0, int64_t n,
                                 double *s);

/* Device workspace needed by cryo_forward for runs of up to `nsteps` steps
 * per call (bytes, 256-aligned base expected). */
cryo_status cryo_workspace_bytes(const cryo_plan *plan, int64_t nsteps,
                                 size_t *bytes);

/* Fill the field T (device, see Field layout) with T_init (eq. (5)); an F32
 * field's residual plane is set to zero. */
cryo_status cryo_init(const cryo_plan *plan, void *T, void *stream);

/* Advance T (device, [nz][nr], in: state after step k0, out: after step
 * k0 + nsteps) by nsteps steps of eq. (8).  `ws` is the workspace
 * (cryo_workspace_bytes).  `surf` (device double[nsteps], nullable) receives
 * the surface mean S after each step: the trapezoid mean of T over z on the
 * outer radius r = r_max.  Asynchronous on `stream`. */
cryo_status cryo_forward(const cryo_plan *plan, void *T, int64_t k0,
                         int64_t nsteps, void *ws, size_t ws_bytes,
                         double *surf, void *stream);

/* Stepped domain of eq. (9) (N_j radial nodes on line j): lines
 * j <= z_full span all nr radial nodes (the layered section, z <= z_0), lines
 * above span nodes 0..nr_top-1 only (the terminal, z_0 < z <= z_max).  The
 * terminal's outer wall (node nr_top - 1) and the step face are insulated: a
 * node of line z_full exchanges axial heat only with a capacity node above
 * it (nodes nr_top - 1 and beyond see a closed face).  The held or insulated
 * outer wall of the problem applies to the layered section, the inner wall
 * and the z-boundaries to every line.  Nodes outside the domain are not
 * solved: their values are whatever the field held (a z-boundary copy or
 * hold still writes them).  The surface output becomes the trapezoid mean of
 * T on r = r_max over z in [0, z_0] (lines 0..z_full).  1 <= z_full <= nz-2,
 * 3 <= nr_top <= nr (CRYO_ERR_ARG otherwise); must precede the plan's first
 * device call; FP64 and FP32; combines with the polynomial laws and the
 * turn-on model.  Gradients follow the stepped domain (the surface mean over
 * the layered section); a shape whose adjoint tables would not fit a
 * workgroup's LDS is refused there (CRYO_ERR_UNSUPPORTED).  Batches take the
 * domain per instance (cryo_batch_create_with). */
cryo_status cryo_plan_set_stepped(cryo_plan *plan, int32_t z_full, int32_t nr_top);

/* Polynomial material laws of eqs. (23) and (24) in place of the power laws,
 * and optionally the Joule source of eqs. (2) and (25).  FP64 and FP32
 * plans (FP32 evaluates the laws in float); must precede the plan's first
 * device call.  `a` holds 4 coefficients per layer (inner to outer):
 * c_m(T) = sum_{k=0..3} a[4m+k] T^k [J/(kg K)]; `b` holds 5 per layer:
 * lambda_m(T) = k_scale_m sum_{k=0..4} b[5m+k] T^k [W/(m K)]; rho and
 * k_scale come from the layers' cryo_material, whose power-law fields are
 * then unused.  joule_tref > 0 makes the heater's source
 * amplitude * (gate average) * sqrt(joule_tref / T) at each node's old
 * temperature (a resistivity proportional to T^(-1/2), eq. (25)); 0 keeps it
 * temperature-independent.  Both laws must be positive, and dt within
 * eq. (21)'s bound, at the coldest prescribed temperature (checked there
 * only: CRYO_ERR_ARG, CRYO_ERR_UNSTABLE).  Arrays are copied.  Gradients
 * follow the laws and the source (see cryo_gradient); batches take them per
 * instance (cryo_batch_create_with). */
cryo_status cryo_plan_set_poly_laws(cryo_plan *plan, const double *a, const double *b,
                                    double joule_tref);

/* Transient turn-on model of the source, Sec. 3.2, eq. (22), read with a
 * decaying exponential (p^2 = 1 - exp(-(t - t_n) / (7 tau*)), tau* = dt/100,
 * rising from 0 towards 1).  With on != 0, every step k of cryo_forward whose
 * interval starts a pulse (k dt = t_on + n period) runs as 100 sub-steps of
 * dt/100; sub-step i takes the gate of eq. (4) averaged over the sub-step
 * times 1 - exp(-i/7), the value of p^2 at its start.  Other steps are
 * unchanged, and `surf` keeps one value per step (after its last sub-step).
 * Requires t_on and period to be whole multiples of dt (CRYO_ERR_UNSUPPORTED
 * otherwise).  The plan builds host tables for dt/100 here (device tables at
 * its next forward call), follows later cryo_plan_set_shape calls, and frees
 * them with on = 0 or cryo_plan_destroy.  Gradients include the sub-steps
 * in their sweep (see cryo_gradient); batch instances take the model
 * through the turn_on field of their options, see cryo_batch_create_with. */
cryo_status cryo_plan_set_turn_on(cryo_plan *plan, int32_t on);

/* After the stream has finished a cryo_forward that used `ws`: returns
 * CRYO_ERR_NONFINITE if that call produced a non-finite temperature, else
 * CRYO_OK.  Synchronises `stream`. */
cryo_status cryo_poll(const cryo_plan *plan, const void *ws, void *stream);

/* ---- Resident state -----------------------------------------------------
 * cryo_forward converts the field to the kernels' internal layout (radial
 * rows lane-major per line, FP32 pairs interleaved per line) and back on
 * every call: two extra passes over the field.  A resident state keeps the
 * field in that layout in caller-owned device memory between calls, so that
 * many short runs (restarts, design loops, step-by-step drivers) pay the
 * conversion once.  The memory is a workspace of cryo_workspace_bytes
 * bytes (256-aligned); the state object only records it and which of its two
 * field buffers is current, so calls on one state must be ordered on one
 * stream (or synchronised).  cryo_poll(plan, mem, stream) reports a
 * non-finite temperature produced since the last cryo_state_load. */
typedef struct cryo_state cryo_state;
/* Record `mem` (bytes >= cryo_workspace_bytes) as a state of `plan`; makes
 * the plan's device tables if this is the plan's first device use.  No
 * other device work.  The plan must outlive the state. */
cryo_status cryo_state_create(const cryo_plan *plan, void *mem, size_t bytes,
                              cryo_state **out);
void cryo_state_destroy(cryo_state *state);
/* Load the field T (device, the Field layout above) into the state and clear
 * its error word.  Asynchronous on `stream`. */
cryo_status cryo_state_load(cryo_state *state, const void *T, void *stream);
/* Advance the state by nsteps steps of eq. (8) from global step k0, exactly
 * as cryo_forward does (same kernels, same results bit for bit); `surf` as
 * there.  Asynchronous on `stream`. */
cryo_status cryo_state_forward(cryo_state *state, int64_t k0, int64_t nsteps, double *surf,
                               void *stream);
/* Write the state's current field to T (device, the Field layout above);
 * a non-finite value sets the error word.  Asynchronous on `stream`. */
cryo_status cryo_state_store(const cryo_state *state, void *T, void *stream);

/* ---- Forward without allocation ------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * cryo_forward_noalloc does exactly what cryo_forward does (same kernels,
 * same results bit for bit) but keeps its workspace in a library-owned
 * device array of CRYO_NOALLOC_MAX_BYTES bytes instead of caller memory; it
 * calls no hipMalloc, hipFree or allocating library routine.  The caller
 * still passes the field T (device, the Field layout above) and `surf`
 * (device double[nsteps], nullable).  The array is part of the library's
 * device code object: every GPU the library runs on holds its own copy
 * until the process ends, and its address is looked up on the first call
 * on each device.
 *  - A plan whose workspace (cryo_workspace_bytes) exceeds the array is
 *    refused with CRYO_ERR_WORKSPACE (72 MiB holds the 1024 x 4096 FP64 cell).
 *  - The plan must already hold its device tables (made by its first
 *    cryo_forward or by cryo_state_create); otherwise CRYO_ERR_ARG.  The
 *    current device must be the plan's (CRYO_ERR_ARG).
 *  - Every call on one GPU shares that GPU's array, which keeps the last
 *    call's contents: calls that overlap on one GPU (other streams, other
 *    host threads) race and must be ordered by the caller.
 *  - The kernels' non-finite error word lives in the array and is not
 *    reported (cryo_poll needs a workspace): callers that need that check
 *    use cryo_forward.
 * Asynchronous on `stream`. */
#define CRYO_NOALLOC_MAX_BYTES (72u << 20)
cryo_status cryo_forward_noalloc(const cryo_plan *plan, void *T, int64_t k0, int64_t nsteps,
                                 double *surf, void *stream);

/* ---- Autotuning ---------------------------------------------------------
 * Time every built kernel shape (rows per lane x waves per line covering nr)
 * and lines per wave 1, 2, 4, 8 on `prob` for `steps` steps and return the
 * fastest as shape[3] (for cryo_plan_set_shape or cryo_batch_create), with
 * its time per step (or -1 when taken from the cache).  The tuner allocates
 * and frees its own trial field and workspaces.  `cache_path` (nullable)
 * names a text file of earlier results keyed by dtype, nr, nz, layer count
 * and law family (every capacity exponent 3, or not); new results are
 * appended.  Synchronous on `stream`. */
cryo_status cryo_autotune(const cryo_problem *prob, cryo_dtype dtype, int32_t steps,
                          const char *cache_path, void *stream, int32_t *shape,
                          double *us_per_step);

/* Launch shapes for a batch (cryo_batch_create's `shapes`, n x 3 values):
 * the n instances are grouped as cryo_batch_create groups them with default
 * shapes (rows per lane and waves per line covering nr, capacity-law family);
 * for each group every built shape covering its largest radial size with
 * fewer than twice as many rows (or at most 2 rows per lane), with lines per
 * wave 1, 2, 4 and 8, is timed as a batch of up to 8 of the group's
 * instances (spread over their sizes) for `steps` steps (rounded up to
 * whole captured blocks of 32), and the shape with the least time per node
 * and step is given to all of the group's instances (lines per wave capped
 * at nz - 2).  Then, with more than one group, the whole batch is timed:
 * each group in turn (most nodes first) tries lines per wave 1, 2 and 4
 * beside the others as picked and keeps a value that makes the batch at
 * least 1 % faster (the groups' launches share the chip), in a second sweep
 * too when the first changed any group.  `cache_path`
 * (nullable) names a text file keyed by dtype, the group's default shape,
 * law family and largest radial size for the first pass, and by a hash of
 * the instances' grids, layer counts and law families for the second; new
 * results are appended.  The tuner allocates and frees its own trial fields
 * and workspaces.  Synchronous on `stream`. */
cryo_status cryo_batch_autotune(int32_t n, const cryo_problem *probs, cryo_dtype dtype,
                                int32_t steps, const char *cache_path, void *stream,
                                int32_t *shapes);

/* ---- Gradient by the discrete adjoint -----------------------------------
 * J = sum_{n=1..N} (S_n - target_n)^2 with S_n the surface mean after step
 * n, and its gradient with respect to
 *   theta = [amplitude, width, thickness_0..L-1, k_scale_0..L-1]
 * (grad has 2 + 2L entries), from the exact discrete adjoint of the N steps
 * from T0 (steps 0..N-1): transposed line solves, the local stencil of the
 * lagged coefficients, the copied z-boundary lines, the radii that move with
 * the thicknesses, and the pulse-edge steps (a pulse end on a step boundary
 * takes the mean of the two one-sided derivatives).  With the turn-on model
 * (cryo_plan_set_turn_on) the sweep runs over kernel steps, the 100
 * sub-steps of each pulse-start step included, whose source factors carry
 * p^2 and a width derivative of their own; the surface is still observed
 * once per step.  The states of the last kernel steps are kept from the
 * forward as far as the plan's gradient store reaches
 * (cryo_plan_set_gradient_store; none by default); the steps before them
 * are checkpointed every ckpt kernel steps (0: the square root of their
 * count, rounded up) and each segment is recomputed.
 * FP64 plans with one of the gradient's shapes only (CRYO_ERR_UNSUPPORTED
 * otherwise, see cryo_plan_set_shape); polynomial laws and the Joule source
 * (cryo_plan_set_poly_laws: the derivative polynomials, the interface row's
 * quotient of two laws, the source's sqrt(tref / T) factor) and a stepped
 * domain (cryo_plan_set_stepped) are followed.  T0 is a device field;
 * target, J, grad and surf (nullable, N values) are host arrays.  Synchronous on `stream`; the same device work as
 * cryo_gradient_async (results equal bit for bit). */
cryo_status cryo_gradient_workspace_bytes(const cryo_plan *plan, int64_t nsteps, int64_t ckpt,
                                          size_t *bytes);
/* The gradient store of a plan: the last `steps` kernel steps of a gradient's
 * run (all of them if the run has fewer) keep their states from its forward
 * (one field of 8 nz np bytes, rounded up to 256, per step, plus one for the
 * final state), so their adjoint steps need no recompute; only the steps
 * before them are checkpointed and recomputed.  This trades device memory
 * for time: each stored step saves one recomputed step.  The workspace
 * (cryo_gradient_workspace_bytes) grows accordingly; results are the same
 * bit for bit for every store.  0 (the default) stores none.  The setting is
 * read by the later workspace queries and gradient calls on the plan.
 * CRYO_ERR_ARG for steps < 0.  (The paper's scheme has no adjoint; this is
 * the memory/recompute split of the discrete adjoint of Sec. 3's steps.) */
cryo_status cryo_plan_set_gradient_store(cryo_plan *plan, int64_t steps);
/* The largest gradient store (at most the run's kernel steps) for which the
 * workspace of a run of nsteps steps with checkpoint interval ckpt fits in
 * budget_bytes, into *steps; 0 when no store fits (the workspace without one
 * may still not).  Host-only; the plan's own setting is neither read nor
 * changed.  CRYO_ERR_ARG for a null pointer, nsteps < 1 or ckpt < 0. */
cryo_status cryo_gradient_store_steps(const cryo_plan *plan, int64_t nsteps, int64_t ckpt,
                                      size_t budget_bytes, int64_t *steps);
cryo_status cryo_gradient(const cryo_plan *plan, const void *T0, int64_t nsteps,
                          const double *target, int64_t ckpt, void *ws, size_t ws_bytes,
                          double *J, double *grad, double *surf, void *stream);

/* cryo_gradient on the caller's stream, with no host wait: target (N
 * values), J (1), grad (2 + 2L) and surf (N values, nullable) are device
 * arrays, and every phase (forward with checkpoints, J and the seeds dJ/dS_n,
 * the backward sweep, the fixed-order parameter sums) is a launch or a
 * device-to-device copy on `stream`, so a caller may capture it in a HIP
 * graph once the plan holds its device tables (made by any earlier call on
 * it; a capture must not be the plan's first device use).  Workspace as for
 * cryo_gradient; the buffers must stay alive until the stream has finished.
 * A non-finite temperature is not returned: cryo_poll(plan, ws, stream)
 * reports it afterwards.  Argument errors as cryo_gradient. */
cryo_status cryo_gradient_async(const cryo_plan *plan, const void *T0, int64_t nsteps,
                                const double *target, int64_t ckpt, void *ws, size_t ws_bytes,
                                double *J, double *grad, double *surf, void *stream);

/* Gradients of n designs (the batched design loop): the same as n calls of
 * cryo_gradient, design i with plans[i], T0[i], targets[i] (nsteps values),
 * ws[i] of ws_bytes[i] bytes (cryo_gradient_workspace_bytes of plans[i]),
 * results J[i], grad[i] (2 + 2 L_i values) and surf_out[i] (nullable array,
 * nullable entries).  Designs may share a workspace (the same ws[i]
 * pointer, large enough for each of them): those run one after another on
 * one stream, so k workspaces with a gradient store each can serve any
 * number of designs.  The designs run on n_streams streams (0: enough for
 * the launches of designs running side by side to cover the compute units,
 * at most 4, the hardware queues a process gets by default; never more than
 * the distinct workspaces) of default priority that the library makes on
 * first use and keeps per device (they do not wait for other streams: T0
 * must be ready when the call is made).  The targets are copied in at once
 * to a device block the call allocates (with room for each design's J,
 * gradient, trace and error word, copied there from its workspace when the
 * design ends); then each workspace's designs are enqueued in order on
 * stream q mod n_streams for the q-th distinct workspace (one host thread
 * per stream), then the block is read back and freed.  Results equal those
 * of the single calls bit for bit.  The plans' device tables are made first,
 * on the calling thread.  Synchronous; errors name the failing design (the
 * lowest index among the threads' first failures). */
cryo_status cryo_gradient_many(int32_t n, cryo_plan *const *plans, const void *const *T0,
                               int64_t nsteps, const double *const *targets, int64_t ckpt,
                               void *const *ws, const size_t *ws_bytes, int32_t n_streams,
                               double *J, double *const *grad, double *const *surf_out);

/* ---- Batched design sweeps ---------------------------------------------
 * Many independent cells (uneven grids, own dt, layers and pulse) stepped
 * together: instances are grouped by kernel shape; each step is one launch
 * per shape group over all of its instances, and blocks of 32 steps are
 * captured once in a HIP graph (on private capture streams: one branch per
 * shape group, so that groups may run side by side) and replayed on the
 * caller's stream.  The fields of all instances are packed in one device
 * buffer: instance i's field (the plan's field layout) starts at element
 * offsets[i] of the batch dtype.  Every instance uses the same global step
 * range k0 .. k0 + nsteps. */

/* Create a batch of n instances.  `shapes` (nullable) gives per instance
 * (rows_per_lane, waves_per_line, lines_per_wave), e.g. from cryo_autotune;
 * otherwise each plan's default chunk shape with 4 lines per wave.  Errors
 * name the failing instance. */
cryo_status cryo_batch_create(int32_t n, const cryo_problem *probs, cryo_dtype dtype,
                              const int32_t *shapes, cryo_batch **out);

/* Plan options of one batch instance: what cryo_plan_set_poly_laws,
 * cryo_plan_set_stepped and cryo_plan_set_turn_on set on a single plan
 * (same arguments and checks). */
typedef struct {
    const double *poly_a;    /* NULL, or [n_layers][4]: c(T) of eq. (23) */
    const double *poly_b;    /* NULL, or [n_layers][5]: lambda(T) / k_scale of
                              * eq. (24); given with poly_a */
    double joule_tref;       /* > 0 with the polynomial laws: the Joule source
                              * of eq. (25); else 0 */
    int32_t z_full, nr_top;  /* both 0: rectangular; else the stepped domain of
                              * eq. (9) */
    int32_t turn_on;         /* nonzero: the turn-on model of eq. (22) (pulse
                              * starts on whole steps, CRYO_ERR_UNSUPPORTED
                              * otherwise) */
} cryo_instance_options;
/* cryo_batch_create with per-instance options (`opts`: n entries, nullable
 * for none).  Instances are grouped by kernel shape, law family (cube
 * capacity, general power laws, polynomial laws) and domain (rectangular or
 * stepped), one launch per group and step as above; each instance steps
 * exactly as a plan with the same shape and options (bit for bit).  With
 * the turn-on model on some instances, cryo_batch_forward splits its step
 * range at every step where one of them starts a pulse: that step runs
 * eagerly, those instances through their 100 sub-steps of dt/100 and the
 * others through one step each (single-plan launches of the same kernels),
 * and the steps between such steps run as above.  Option errors name the
 * instance (CRYO_ERR_ARG, CRYO_ERR_UNSTABLE, CRYO_ERR_UNSUPPORTED, as the
 * plan setters). */
cryo_status cryo_batch_create_with(int32_t n, const cryo_problem *probs, cryo_dtype dtype,
                                   const int32_t *shapes, const cryo_instance_options *opts,
                                   cryo_batch **out);
/* cryo_batch_autotune for instances with plan options (`opts`: n entries,
 * nullable for none, as cryo_batch_create_with takes them): instances are
 * grouped as cryo_batch_create_with groups them (shape, law family, domain),
 * each trial batch is made with the instances' options, and the cache keys
 * add the law family "poly" and the word "stepped" for such groups and the
 * options to the batch hash (a batch without options keeps the keys of
 * cryo_batch_autotune, which is this call with opts NULL).  Shapes the
 * options' tables do not fit are skipped.  The turn-on model is not timed
 * (its sub-steps are rare and run on the instance's shape): trial batches
 * step without it. */
cryo_status cryo_batch_autotune_with(int32_t n, const cryo_problem *probs, cryo_dtype dtype,
                                     const cryo_instance_options *opts, int32_t steps,
                                     const char *cache_path, void *stream, int32_t *shapes);
void cryo_batch_destroy(cryo_batch *batch);
/* Element offsets of the instances' fields in the packed buffer (n + 1). */
cryo_status cryo_batch_offsets(const cryo_batch *batch, int64_t *offsets);
/* Kernel shape chosen for instance i (3 values, as cryo_plan_shape). */
cryo_status cryo_batch_shape(const cryo_batch *batch, int32_t i, int32_t *shape);
/* Device workspace of cryo_batch_forward (bytes, 256-aligned base). */
cryo_status cryo_batch_workspace_bytes(const cryo_batch *batch, size_t *bytes);
/* Fill every instance's field with its T_init. */
cryo_status cryo_batch_init(const cryo_batch *batch, void *T, void *stream);
/* Advance every instance by nsteps steps from global step k0.  The captured
 * graph is tied to `ws`; a call with another workspace re-captures it.
 * Asynchronous on `stream`.  No device allocation after the first call. */
cryo_status cryo_batch_forward(cryo_batch *batch, void *T, int64_t k0, int64_t nsteps,
                               void *ws, size_t ws_bytes, void *stream);
/* After a cryo_batch_forward: CRYO_ERR_NONFINITE if an instance produced a
 * non-finite or out-of-range temperature; *bad_instance (nullable) gets the
 * first such instance or -1.  Synchronises `stream`. */
cryo_status cryo_batch_poll(const cryo_batch *batch, const void *ws, void *stream,
                            int32_t *bad_instance);

#ifdef __cplusplus
}
#endif
#endif
