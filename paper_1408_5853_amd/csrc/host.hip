// Host side of the C ABI: descriptor validation, the explicit stability bound
// (eq. (21)), the radial grid and its per-row tables (eqs. (9), (10), (13),
// (18)), the pulse schedule (eq. (4)) and the forward driver.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "internal.h"

namespace cryo {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

cryo_status fail(cryo_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

static double snap(double x) {
    double n = nearbyint(x);
    return fabs(x - n) <= 1e-9 * fmax(1.0, fabs(x)) ? n : x;
}

// Time the rectangular gate of eq. (4) is open within [lo, hi), all times in
// step units: pulses occupy [b0 + n P, b0 + n P + W), n >= 0.
static double gate_open(const Pulse &p, double lo, double hi) {
    if (!(p.W > 0)) return 0.0;
    double s = 0.0;
    int64_t n = (int64_t)floor((lo - p.b0 - p.W) / p.P);
    if (n < 0) n = 0;
    for (;; ++n) {
        double b = p.b0 + (double)n * p.P;
        if (b >= hi) break;
        double e = b + p.W;
        double o = std::min(hi, e) - std::max(lo, b);
        if (o > 0) s += o;
    }
    return s;
}

// the gate's average over step k
double source_fraction(const Pulse &p, int64_t k) {
    return gate_open(p, (double)k, (double)k + 1.0);
}

// Turn-on model, eq. (22): pulse n starts at step b0 + n P, which needs b0
// and P whole.  Sub-step i (of 100) of a pulse-start step k spans
// [k + i/100, k + (i+1)/100) and starts i tau* after the pulse, where
// p^2 = 1 - exp(-i tau* / (7 tau*)).
bool pulse_starts_on_steps(const Pulse &p) {
    return p.b0 == floor(p.b0) && p.P == floor(p.P) && p.P >= 1.0;
}
bool pulse_start(const Pulse &p, int64_t k) {
    if (!(p.W > 0) || !pulse_starts_on_steps(p)) return false;
    const int64_t kb = (int64_t)p.b0, kp = (int64_t)p.P;
    return k >= kb && (k - kb) % kp == 0;
}
double turn_on_source(const Pulse &p, int64_t k, int i) {
    const double lo = (double)k + (double)i / 100.0, hi = (double)k + (double)(i + 1) / 100.0;
    return gate_open(p, lo, hi) / (hi - lo) * (1.0 - exp(-(double)i / 7.0));
}

// FP64 power tables (see POW_*): one block per law id, then the cube path's
// multipliers and addends (K T^3 + A)
static void fill_pow_blob(const Laws &lw, std::vector<double> &blob) {
    const int L = lw.L, nlaw = 3 * L + 2, UNIT = law_unit(L);
    blob.assign(pow_blob_doubles(L), 0.0);
    double *B = blob.data();
    double *CKA = B + (size_t)nlaw * POW_BLK;                     // {K, A} per id
    for (int id = 0; id < nlaw; ++id) {
        const double e = lw.e[id];
        double *R = B + (size_t)id * POW_BLK;
        for (int j = 0; j < POW_NM; ++j) {
            const double m0 = 1.0 + (j + 0.5) / POW_NM;
            R[2 * j] = pow(m0, e);
            R[2 * j + 1] = 2.0 / m0;          // applied to the frexp mantissa in [1/2, 1)
        }
        for (int x = 0; x < POW_NE; ++x) R[POW_BX + x] = lw.K[id] * exp2(e * (x + POW_EMIN));
        R[POW_BE] = e;
        // binomial coefficients of (1 + u)^e, k = 2..POW_DEG
        double c = e;
        for (int k = 2; k <= POW_DEG; ++k) {
            c = c * (e - (k - 1)) / k;
            R[POW_BE + k] = c;
        }
        CKA[2 * id] = (id >= 2 * L && id < 3 * L) ? lw.K[id] : 0.0;
        CKA[2 * id + 1] = id == UNIT ? 1.0 : 0.0;
    }
}

// Relative truncation bound of the FP64 table power T^e (see POW_*): the
// first term the binomial series of (1 + u)^e drops, |binom(e, POW_DEG + 1)|
// |u|^(POW_DEG + 1) with |u| <= 2^-(POW_MBITS + 1).
static double pow_trunc_bound(double e) {
    double c = 1.0;
    for (int k = 1; k <= POW_DEG + 1; ++k) c *= (e - (k - 1)) / k;
    return fabs(c) * exp2(-(double)(POW_DEG + 1) * (POW_MBITS + 1));
}

// Every exponent a plan's power tables hold: the layers' p and q, and the
// stepping kernel's interface ratio laws p_m - p_{m+1}.
static cryo_status check_exponents(const cryo_geometry &g) {
    for (int m = 0; m < g.n_layers; ++m) {
        const cryo_material &mt = g.layers[m].mat;
        const double ex[3] = {mt.p, mt.q,
                              m + 1 < g.n_layers ? mt.p - g.layers[m + 1].mat.p : 0.0};
        const char *what[3] = {"conductivity exponent p", "capacity exponent q",
                               "conductivity ratio exponent p_m - p_{m+1}"};
        for (int k = 0; k < 3; ++k)
            if (pow_trunc_bound(ex[k]) > POW_TRUNC_MAX)
                return fail(CRYO_ERR_UNSUPPORTED,
                            std::string(what[k]) + " = " + std::to_string(ex[k]) +
                                " of layer " + std::to_string(m) +
                                " lies outside the range where the FP64 power series meets "
                                "1e-14 (about -5.3 <= e <= 12.5)");
    }
    return CRYO_OK;
}

static cryo_status check_problem(const cryo_problem *pr) {
    if (!pr) return fail(CRYO_ERR_ARG, "null problem");
    const cryo_geometry &g = pr->geom;
    if (g.nr < 3 || g.nz < 3) return fail(CRYO_ERR_ARG, "nr and nz must be >= 3");
    if (g.nr > MAX_NR)
        return fail(CRYO_ERR_UNSUPPORTED, "nr above " + std::to_string(MAX_NR));
    if (g.n_layers < 1 || g.n_layers > MAX_LAYERS || !g.layers)
        return fail(CRYO_ERR_ARG, "n_layers must be 1..16 with a layer array");
    if (!(g.height > 0) || !(g.r_inner >= 0) || !std::isfinite(g.height) ||
        !std::isfinite(g.r_inner))
        return fail(CRYO_ERR_ARG, "height must be > 0 and r_inner >= 0");
    int64_t tot = 0;
    for (int m = 0; m < g.n_layers; ++m) {
        const cryo_layer &l = g.layers[m];
        if (l.intervals < 2) return fail(CRYO_ERR_ARG, "each layer needs >= 2 intervals");
        if (!(l.thickness > 0) || !std::isfinite(l.thickness))
            return fail(CRYO_ERR_ARG, "layer thickness must be > 0");
        const cryo_material &mt = l.mat;
        if (!(mt.k0 > 0) || !(mt.k_scale > 0) || !(mt.c0 > 0) || !(mt.rho > 0) ||
            !(mt.tref > 0) || !std::isfinite(mt.p) || !std::isfinite(mt.q))
            return fail(CRYO_ERR_ARG, "material constants must be positive and finite");
        tot += l.intervals;
    }
    if (tot != g.nr - 1) return fail(CRYO_ERR_ARG, "sum of layer intervals must be nr - 1");
    if (check_exponents(g) != CRYO_OK) return CRYO_ERR_UNSUPPORTED;
    const cryo_pulse &pu = pr->pulse;
    if (pu.layer < 0 || pu.layer >= g.n_layers)
        return fail(CRYO_ERR_ARG, "heater layer index out of range");
    if (!(pu.period > 0) || !(pu.width >= 0) || pu.width > pu.period || !(pu.t_on >= 0) ||
        !std::isfinite(pu.amplitude))
        return fail(CRYO_ERR_ARG, "pulse needs period > 0, 0 <= width <= period, t_on >= 0");
    for (int s = 0; s < 4; ++s) {
        if (pr->bc.kind[s] != CRYO_INSULATED && pr->bc.kind[s] != CRYO_HELD)
            return fail(CRYO_ERR_ARG, "boundary kind must be 0 or 1");
        if (pr->bc.kind[s] == CRYO_HELD &&
            !(pr->bc.value[s] >= POW_TLO && pr->bc.value[s] < POW_THI))
            return fail(CRYO_ERR_ARG, "held boundary temperature must lie in [1/16 K, 2^20 K)");
    }
    if (g.r_inner == 0 && pr->bc.kind[0] != CRYO_INSULATED)
        return fail(CRYO_ERR_ARG, "r_inner = 0 (the axis) must be insulated");
    if (!(pr->dt > 0) || !std::isfinite(pr->dt)) return fail(CRYO_ERR_ARG, "dt must be > 0");
    if (!(pr->T_init >= POW_TLO && pr->T_init < POW_THI))
        return fail(CRYO_ERR_ARG, "T_init must lie in [1/16 K, 2^20 K)");
    return CRYO_OK;
}

static double dt_bound(const cryo_problem *pr, double Tm) {
    const cryo_geometry &g = pr->geom;
    double eta = g.height / (g.nz - 1);
    double best = INFINITY;
    for (int m = 0; m < g.n_layers; ++m) {
        const cryo_material &mt = g.layers[m].mat;
        double x = Tm / mt.tref;
        double rc = mt.rho * mt.c0 * pow(x, mt.q);
        double lam = mt.k_scale * mt.k0 * pow(x, mt.p);
        best = std::min(best, rc / lam);
    }
    return 0.5 * eta * eta * best;
}

// Chunk shape of a line: rows per lane and waves per line.  One wave per line
// with the fewest rows per lane that cover nr (up to 1024 rows), then 8 rows
// per lane over more waves.
static void pick_shape(int nr, int *rpl, int *wpl) {
    for (int r : ONE_WAVE_RPL)
        if (WAVE * r >= nr) {
            *rpl = r;
            *wpl = 1;
            return;
        }
    int w = 1;
    while (WAVE * w * 8 < nr) w *= 2;
    *rpl = 8;
    *wpl = w;
}

// Lines per wave: about one workgroup per compute unit of an MI355X (256),
// so that every unit works and each line group amortises its start-up line.
static int pick_lpw(int nz, int wpl) {
    const int per_wg = STEP_WAVES_HOST / wpl;
    const double l = (double)(nz - 2) / ((double)per_wg * 256.0);
    return std::min(8, std::max(1, (int)std::lround(l)));
}

// Device copies of the per-row tables, made once on the first call that
// needs the device (on the device current at that time).
cryo_status ensure_device(cryo_plan *p) {
    if (p->d_info) return CRYO_OK;
    (void)hipGetDevice(&p->device);
    const int np = p->np;
    size_t es = p->dtype == CRYO_F64 ? sizeof(double) : sizeof(float);
    // one array of two planes: fgw, fge
    std::vector<double> rows(p->fgw);
    rows.insert(rows.end(), p->fge.begin(), p->fge.end());
    const std::vector<double> &blobs = p->fpow_blob;
    hipError_t e = hipMalloc(&p->d_rows, es * 2 * np);
    uint32_t *info = nullptr;
    if (e == hipSuccess) e = hipMalloc((void **)&info, sizeof(uint32_t) * np);
    if (e == hipSuccess) {
        if (p->dtype == CRYO_F64) {
            e = hipMemcpy(p->d_rows, rows.data(), es * 2 * np, hipMemcpyHostToDevice);
        } else {
            std::vector<float> a(rows.begin(), rows.end());
            e = hipMemcpy(p->d_rows, a.data(), es * 2 * np, hipMemcpyHostToDevice);
        }
    }
    if (e == hipSuccess)
        e = hipMemcpy(info, p->finfo.data(), sizeof(uint32_t) * np, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_pow, sizeof(double) * blobs.size());
    if (e == hipSuccess)
        e = hipMemcpy(p->d_pow, blobs.data(), sizeof(double) * blobs.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && p->stepped) {
        std::vector<double> t(p->tfgw);
        t.insert(t.end(), p->tfge.begin(), p->tfge.end());
        e = hipMalloc(&p->d_rows2, es * 2 * np);
        if (e == hipSuccess) {
            if (p->dtype == CRYO_F64) {
                e = hipMemcpy(p->d_rows2, t.data(), es * 2 * np, hipMemcpyHostToDevice);
            } else {
                std::vector<float> f(t.begin(), t.end());
                e = hipMemcpy(p->d_rows2, f.data(), es * 2 * np, hipMemcpyHostToDevice);
            }
        }
        if (e == hipSuccess) e = hipMalloc((void **)&p->d_info2, sizeof(uint32_t) * np);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_info2, p->tfinfo.data(), sizeof(uint32_t) * np,
                          hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && p->dtype == CRYO_F64) {
        const std::vector<double> gt = grad_param_table(p);
        e = hipMalloc((void **)&p->d_grad, sizeof(double) * gt.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d_grad, gt.data(), sizeof(double) * gt.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        if (p->d_rows) (void)hipFree(p->d_rows);
        if (info) (void)hipFree(info);
        if (p->d_pow) (void)hipFree(p->d_pow);
        if (p->d_rows2) (void)hipFree(p->d_rows2);
        if (p->d_info2) (void)hipFree(p->d_info2);
        if (p->d_grad) (void)hipFree(p->d_grad);
        p->d_rows = nullptr;
        p->d_pow = nullptr;
        p->d_rows2 = nullptr;
        p->d_info2 = nullptr;
        p->d_grad = nullptr;
        return fail(CRYO_ERR_DEVICE, std::string("device table upload: ") + hipGetErrorString(e));
    }
    p->d_info = info;
    return CRYO_OK;
}

// Lane-major per-row tables: row i = lg * rpl + reg of a line sits at
// reg * (64 wpl) + lg, lg the lane within the line.
// One line's rows: nodes 0..n-1 of the grid, row n-1 the outer wall
// (insulated when `terminal`, else as the problem says).  Writes the rows in
// the kernels' form (fgw, fge, finfo) at the lane-major positions; gw, ge and
// the slot laws are first formed as the equations write the rows.
static void fill_rows(cryo_plan *p, int n, bool terminal, double *fgwo, double *fgeo,
                      uint32_t *finfo) {
    const cryo_problem *prob = &p->prob;
    const int nr = p->nr, L = p->L, rpl = p->rpl;
    const int ZERO = law_zero(L), UNIT = law_unit(L);
    const double e2 = p->eta * p->eta;
    const int *bk = prob->bc.kind;
    for (int i = 0; i < n; ++i) {
        int idx = (i % rpl) * (WAVE * p->wpl) + i / rpl;
        uint32_t kind = (i == n - 1 && n < nr) ? (uint32_t)K_HI : (uint32_t)p->kind[i];
        uint32_t m = p->lay[i];
        uint32_t lawE = (i < n - 1) ? p->lay[i + 1] : ZERO;      // radial law of interval i+1
        uint32_t law2 = ZERO, law3 = ZERO, lawC = ZERO, heat = 0, held = 0, side = 0;
        double gw = 0.0, ge = 0.0;
        if (kind == K_CAP) {
            // eq. (13): A = -r_{i-1/2} lam_{i-1/2} / (r_i hbar_i h_i), C likewise
            double hb = 0.5 * (p->h[i] + p->h[i + 1]);
            gw = 0.5 * (p->r[i] + p->r[i - 1]) / (p->r[i] * hb * p->h[i]);
            ge = 0.5 * (p->r[i] + p->r[i + 1]) / (p->r[i] * hb * p->h[i + 1]);
            law2 = law3 = L + m;                                 // axial faces
            lawC = 2 * L + m;
            heat = (int)m == prob->pulse.layer ? 1u : 0u;
        } else if (kind == K_IFACE) {
            // eq. (18): lam*_m h_{i+1} (T_i - T_{i-1}) = lam*_{m+1} h_i (T_{i+1} - T_i)
            gw = p->h[i + 1];
            ge = p->h[i];
            law2 = p->lay[i];
            law3 = p->lay[i + 1];
        } else if (kind == K_LO) {
            // eq. (15)/(16): T_0 = T_1, or the held wall value
            if (bk[0] == CRYO_HELD) { lawC = UNIT; held = 1; }
            else { ge = 1.0; law3 = UNIT; }
        } else {  // K_HI: eq. (15)/(17): T_{N} = T_{N-1}, or the held wall value
            if (bk[1] == CRYO_HELD && !terminal) { lawC = UNIT; held = 1; side = 1; }
            else { gw = 1.0; law2 = UNIT; side = 1; }
        }
        // the stepping kernel's form: capacity rows times eta^2 (slot 2 then
        // takes the radial law), interface rows divided by the outer law
        // (slot 2 the ratio law, slot 3 one); boundary rows fold their unit or
        // zero slot laws into gw, ge
        double fgw = gw, fge = ge;
        uint32_t f2 = law2;
        if (kind == K_CAP) {
            fgw *= e2;
            fge *= e2;
            f2 = m;
        } else if (kind == K_IFACE) {
            f2 = L + p->lay[i];
        } else {
            fgw = law2 == (uint32_t)UNIT ? gw : 0.0;
            fge = law3 == (uint32_t)UNIT ? ge : 0.0;
            f2 = UNIT;
        }
        // polynomial laws: an interface row's quotient is formed in the
        // kernel from the inner (slot 2) and outer (slot 3) layer laws
        uint32_t f3 = ZERO;
        if (p->poly) {
            f3 = UNIT;
            if (kind == K_IFACE) {
                f2 = p->lay[i];
                f3 = p->lay[i + 1];
            }
        }
        fgwo[idx] = fgw;
        fgeo[idx] = fge;
        finfo[idx] = info_pack(kind, heat, held, side, lawE, f2, f3, lawC);
    }
}

static void build_row_tables(cryo_plan *p) {
    const int nr = p->nr, L = p->L, np = p->np;
    const int ZERO = law_zero(L), UNIT = law_unit(L);
    // padding rows: identity; polynomial laws divide slot 2 by slot 3 on
    // every row, so slot 3 is the unit law there
    const uint32_t pad = info_pack(K_PAD, 0, 0, 0, ZERO, ZERO, p->poly ? UNIT : ZERO, UNIT);
    p->fgw.assign(np, 0.0);
    p->fge.assign(np, 0.0);
    p->finfo.assign(np, pad);
    fill_rows(p, nr, false, p->fgw.data(), p->fge.data(), p->finfo.data());
    // stepped domain (eq. (9)): the terminal's lines, nodes 0..nr_top-1
    p->tfgw.assign(np, 0.0);
    p->tfge.assign(np, 0.0);
    p->tfinfo.assign(np, pad);
    if (p->stepped)
        fill_rows(p, p->nr_top, true, p->tfgw.data(), p->tfge.data(), p->tfinfo.data());
    p->surf_lane = (nr - 1) / p->rpl;
    p->surf_reg = (nr - 1) % p->rpl;
}

}  // namespace cryo

using namespace cryo;

extern "C" {

const char *cryo_last_error(void) { return g_err.c_str(); }

const char *cryo_version(void) { return "cryocell 0.7 (gfx950)"; }

cryo_status cryo_validate(const cryo_problem *prob) { return check_problem(prob); }

cryo_status cryo_stability_dt_max(const cryo_problem *prob, double T_min, double *dt_max) {
    cryo_status st = check_problem(prob);
    if (st != CRYO_OK) return st;
    if (!(T_min > 0) || !dt_max) return fail(CRYO_ERR_ARG, "T_min must be > 0");
    *dt_max = dt_bound(prob, T_min);
    return CRYO_OK;
}

cryo_status cryo_plan_create(const cryo_problem *prob, cryo_dtype dtype, cryo_plan **out) {
    if (!out) return fail(CRYO_ERR_ARG, "null output");
    *out = nullptr;
    cryo_status st = check_problem(prob);
    if (st != CRYO_OK) return st;
    if (dtype != CRYO_F64 && dtype != CRYO_F32) return fail(CRYO_ERR_ARG, "bad dtype");
    double Tm = prob->T_init;
    for (int s = 0; s < 4; ++s)
        if (prob->bc.kind[s] == CRYO_HELD) Tm = std::min(Tm, prob->bc.value[s]);
    double bound = dt_bound(prob, Tm);
    if (prob->dt > bound * (1 + 1e-12))
        return fail(CRYO_ERR_UNSTABLE, "dt = " + std::to_string(prob->dt) +
                                           " exceeds the explicit z bound " +
                                           std::to_string(bound) + " at T = " +
                                           std::to_string(Tm));

    cryo_plan *p = new cryo_plan();
    p->prob = *prob;
    p->layers.assign(prob->geom.layers, prob->geom.layers + prob->geom.n_layers);
    p->prob.geom.layers = p->layers.data();
    p->dtype = dtype;
    p->nr = prob->geom.nr;
    p->nz = prob->geom.nz;
    p->L = prob->geom.n_layers;
    pick_shape(p->nr, &p->rpl, &p->wpl);
    p->np = WAVE * p->wpl * p->rpl;
    p->lpw = pick_lpw(p->nz, p->wpl);
    p->eta = prob->geom.height / (p->nz - 1);
    const int nr = p->nr, L = p->L;

    // grid, eq. (9): r_{i+1} = r_i + h_{i+1}; equal intervals within a layer
    p->r.assign(nr, 0.0);
    p->h.assign(nr + 1, 0.0);
    p->lay.assign(nr + 1, 0);
    int i = 0;
    for (int m = 0; m < L; ++m)
        for (int k = 0; k < p->layers[m].intervals; ++k) {
            ++i;
            p->lay[i] = m;
            p->h[i] = p->layers[m].thickness / p->layers[m].intervals;
        }
    p->lay[0] = p->lay[1];
    p->r[0] = prob->geom.r_inner;
    for (i = 1; i < nr; ++i) p->r[i] = p->r[i - 1] + p->h[i];
    p->kind.assign(nr, K_CAP);
    p->kind[0] = K_LO;
    p->kind[nr - 1] = K_HI;
    for (i = 1; i < nr - 1; ++i)
        if (p->lay[i] != p->lay[i + 1]) p->kind[i] = K_IFACE;

    // laws (see Laws): radial, axial / eta^2, capacity, zero, unit
    Laws &lw = p->laws;
    memset(&lw, 0, sizeof(lw));
    lw.L = L;
    lw.cube = 1;
    for (int m = 0; m < L; ++m) {
        const cryo_material &mt = p->layers[m].mat;
        double kr = mt.k_scale * mt.k0 * pow(mt.tref, -mt.p);
        lw.K[m] = kr;
        lw.K[L + m] = kr / (p->eta * p->eta);
        lw.K[2 * L + m] = mt.rho * mt.c0 * pow(mt.tref, -mt.q) / prob->dt;
        lw.e[m] = lw.e[L + m] = mt.p;
        lw.e[2 * L + m] = mt.q;
        if (mt.q != 3.0) lw.cube = 0;
    }
    const int nlaw = 3 * L + 2, ZERO = law_zero(L), UNIT = law_unit(L);
    lw.K[ZERO] = 0.0;
    lw.K[UNIT] = 1.0;
    for (int id = 0; id < nlaw; ++id) lw.lk[id] = lw.K[id] > 0 ? log2(lw.K[id]) : -2000.0;

    // the stepping kernel's laws (see Laws): capacity rows scaled by eta^2,
    // interface rows by 1 / (outer law); FP32 takes log2 K - e, its laws being
    // evaluated from the sum of the two values they average
    Laws &fl = p->flaws;
    memset(&fl, 0, sizeof(fl));
    fl.L = L;
    fl.cube = lw.cube;
    const double e2 = p->eta * p->eta;
    for (int m = 0; m < L; ++m) {
        fl.K[m] = lw.K[m];
        fl.e[m] = lw.e[m];
        fl.K[2 * L + m] = lw.K[2 * L + m] * e2;
        fl.e[2 * L + m] = lw.e[2 * L + m];
        if (m + 1 < L) {
            fl.K[L + m] = lw.K[m] / lw.K[m + 1];
            fl.e[L + m] = lw.e[m] - lw.e[m + 1];
        }
    }
    fl.K[UNIT] = 1.0;
    for (int id = 0; id < nlaw; ++id)
        fl.lk[id] = fl.K[id] > 0 ? log2(fl.K[id]) - fl.e[id] : -2000.0;
    fill_pow_blob(fl, p->fpow_blob);

    if (step_lds(p) > MAX_STEP_LDS) {
        delete p;
        return fail(CRYO_ERR_UNSUPPORTED, "tables and line ring exceed a workgroup's LDS");
    }
    build_row_tables(p);
    p->pulse.b0 = snap(prob->pulse.t_on / prob->dt);
    p->pulse.W = snap(prob->pulse.width / prob->dt);
    p->pulse.P = snap(prob->pulse.period / prob->dt);
    p->pulse.amplitude = prob->pulse.amplitude;

    *out = p;
    return CRYO_OK;
}

void cryo_plan_destroy(cryo_plan *p) {
    if (!p) return;
    cryo_plan_destroy(p->sub);
    if (p->d_rows) (void)hipFree(p->d_rows);
    if (p->d_info) (void)hipFree(p->d_info);
    if (p->d_pow) (void)hipFree(p->d_pow);
    if (p->d_rows2) (void)hipFree(p->d_rows2);
    if (p->d_info2) (void)hipFree(p->d_info2);
    if (p->d_grad) (void)hipFree(p->d_grad);
    delete p;
}

cryo_status cryo_plan_shape(const cryo_plan *p, int32_t *rows_per_lane,
                            int32_t *waves_per_line, int32_t *lines_per_wave) {
    if (!p) return fail(CRYO_ERR_ARG, "null plan");
    if (rows_per_lane) *rows_per_lane = p->rpl;
    if (waves_per_line) *waves_per_line = p->wpl;
    if (lines_per_wave) *lines_per_wave = p->lpw;
    return CRYO_OK;
}

cryo_status cryo_plan_set_shape(cryo_plan *p, int32_t rows_per_lane, int32_t waves_per_line,
                                int32_t lines_per_wave) {
    if (!p) return fail(CRYO_ERR_ARG, "null plan");
    if (p->d_info) return fail(CRYO_ERR_ARG, "shape must be set before the plan's first run");
    if (!shape_built(rows_per_lane, waves_per_line))
        return fail(CRYO_ERR_UNSUPPORTED, "no kernel for this chunk shape");
    if ((int64_t)WAVE * waves_per_line * rows_per_lane < p->nr)
        return fail(CRYO_ERR_ARG, "chunk shape too short for the radial line");
    if (lines_per_wave < 1 || lines_per_wave > p->nz - 2)
        return fail(CRYO_ERR_ARG, "lines per wave must be 1..nz-2");
    p->lpw = lines_per_wave;
    if (rows_per_lane != p->rpl || waves_per_line != p->wpl) {
        const int rpl0 = p->rpl, wpl0 = p->wpl;
        p->rpl = rows_per_lane;
        p->wpl = waves_per_line;
        p->np = WAVE * p->wpl * p->rpl;
        if (step_lds(p) > MAX_STEP_LDS) {
            p->rpl = rpl0;
            p->wpl = wpl0;
            p->np = WAVE * p->wpl * p->rpl;
            return fail(CRYO_ERR_UNSUPPORTED, "chunk shape needs more LDS than a workgroup has");
        }
        build_row_tables(p);
    }
    if (p->sub) return cryo_plan_set_shape(p->sub, rows_per_lane, waves_per_line, lines_per_wave);
    return CRYO_OK;
}

// sum_k c_k T^k
static double poly_at(const double *c, int n, double T) {
    double s = 0.0;
    for (int k = n - 1; k >= 0; --k) s = s * T + c[k];
    return s;
}

cryo_status cryo_plan_set_poly_laws(cryo_plan *p, const double *a, const double *b,
                                    double joule_tref) {
    if (!p || !a || !b) return fail(CRYO_ERR_ARG, "null argument");
    if (p->d_info) return fail(CRYO_ERR_ARG, "laws must be set before the plan's first run");
    const int L = p->L;
    for (int i = 0; i < 4 * L; ++i)
        if (!std::isfinite(a[i])) return fail(CRYO_ERR_ARG, "capacity coefficient not finite");
    for (int i = 0; i < 5 * L; ++i)
        if (!std::isfinite(b[i])) return fail(CRYO_ERR_ARG, "conductivity coefficient not finite");
    if (!(joule_tref >= 0) || !std::isfinite(joule_tref))
        return fail(CRYO_ERR_ARG, "Joule reference temperature must be >= 0");
    // positive laws and eq. (21)'s bound at the coldest prescribed temperature
    const cryo_problem *pr = &p->prob;
    double Tm = pr->T_init;
    for (int s = 0; s < 4; ++s)
        if (pr->bc.kind[s] == CRYO_HELD) Tm = std::min(Tm, pr->bc.value[s]);
    double best = INFINITY;
    for (int m = 0; m < L; ++m) {
        const cryo_material &mt = p->layers[m].mat;
        const double c = poly_at(a + 4 * m, 4, Tm), lam = mt.k_scale * poly_at(b + 5 * m, 5, Tm);
        if (!(c > 0) || !(lam > 0))
            return fail(CRYO_ERR_ARG, "polynomial law not positive at T = " + std::to_string(Tm));
        best = std::min(best, mt.rho * c / lam);
    }
    const double bound = 0.5 * p->eta * p->eta * best;
    if (pr->dt > bound * (1 + 1e-12))
        return fail(CRYO_ERR_UNSTABLE, "dt exceeds the explicit z bound " + std::to_string(bound) +
                                           " of the polynomial laws at T = " + std::to_string(Tm));
    p->poly = true;
    p->poly_a.assign(a, a + 4 * L);
    p->poly_b.assign(b, b + 5 * L);
    p->joule_tref = joule_tref;
    p->flaws.cube = 0;
    // the stepping kernel's law blob: POLY_BLK coefficients per law id
    std::vector<double> &B = p->fpow_blob;
    B.assign(pow_blob_doubles(L), 0.0);
    const double e2 = p->eta * p->eta;
    for (int m = 0; m < L; ++m) {
        const cryo_material &mt = p->layers[m].mat;
        for (int k = 0; k < 5; ++k) B[(size_t)POLY_BLK * m + k] = mt.k_scale * b[5 * m + k];
        for (int k = 0; k < 4; ++k)
            B[(size_t)POLY_BLK * (2 * L + m) + k] = e2 * mt.rho * a[4 * m + k] / pr->dt;
    }
    B[(size_t)POLY_BLK * law_unit(L)] = 1.0;
    build_row_tables(p);
    if (p->sub) {
        // the turn-on model's sub-step tables take the same laws, or neither does
        const cryo_status st = cryo_plan_set_poly_laws(p->sub, a, b, joule_tref);
        if (st != CRYO_OK) {
            p->poly = false;
            p->flaws.cube = p->laws.cube;
            fill_pow_blob(p->flaws, p->fpow_blob);
            build_row_tables(p);
            return st;
        }
    }
    return CRYO_OK;
}

cryo_status cryo_plan_set_stepped(cryo_plan *p, int32_t z_full, int32_t nr_top) {
    if (!p) return fail(CRYO_ERR_ARG, "null plan");
    if (p->d_info) return fail(CRYO_ERR_ARG, "the domain must be set before the plan's first run");
    if (z_full < 1 || z_full > p->nz - 2) return fail(CRYO_ERR_ARG, "z_full must be 1..nz-2");
    if (nr_top < 3 || nr_top > p->nr) return fail(CRYO_ERR_ARG, "nr_top must be 3..nr");
    p->stepped = true;
    p->z_full = z_full;
    p->nr_top = nr_top;
    if (step_lds(p) > MAX_STEP_LDS) {
        p->stepped = false;
        return fail(CRYO_ERR_UNSUPPORTED, "the terminal's tables exceed a workgroup's LDS");
    }
    build_row_tables(p);
    if (p->sub) {
        // the turn-on model's sub-step tables take the same domain, or neither does
        const cryo_status st = cryo_plan_set_stepped(p->sub, z_full, nr_top);
        if (st != CRYO_OK) {
            p->stepped = false;
            build_row_tables(p);
            return st;
        }
    }
    return CRYO_OK;
}

cryo_status cryo_plan_set_turn_on(cryo_plan *p, int32_t on) {
    if (!p) return fail(CRYO_ERR_ARG, "null plan");
    if (!on) {
        cryo_plan_destroy(p->sub);
        p->sub = nullptr;
        return CRYO_OK;
    }
    if (p->sub) return CRYO_OK;
    if (p->pulse.W > 0 && !pulse_starts_on_steps(p->pulse))
        return fail(CRYO_ERR_UNSUPPORTED, "the turn-on model needs t_on and period to be "
                                          "whole multiples of dt");
    cryo_problem q = p->prob;
    q.dt = p->prob.dt / 100.0;
    cryo_plan *s = nullptr;
    cryo_status st = cryo_plan_create(&q, p->dtype, &s);
    if (st != CRYO_OK) return st;
    st = cryo_plan_set_shape(s, p->rpl, p->wpl, p->lpw);
    if (st == CRYO_OK && p->poly)
        st = cryo_plan_set_poly_laws(s, p->poly_a.data(), p->poly_b.data(), p->joule_tref);
    if (st == CRYO_OK && p->stepped) st = cryo_plan_set_stepped(s, p->z_full, p->nr_top);
    if (st != CRYO_OK) {
        cryo_plan_destroy(s);
        return st;
    }
    p->sub = s;
    return CRYO_OK;
}

cryo_status cryo_grid_radii(const cryo_plan *p, double *r) {
    if (!p || !r) return fail(CRYO_ERR_ARG, "null argument");
    memcpy(r, p->r.data(), sizeof(double) * p->nr);
    return CRYO_OK;
}

cryo_status cryo_source_fraction(const cryo_plan *p, int64_t k0, int64_t n, double *s) {
    if (!p || !s || n < 0 || k0 < 0) return fail(CRYO_ERR_ARG, "bad argument");
    for (int64_t k = 0; k < n; ++k) s[k] = source_fraction(p->pulse, k0 + k);
    return CRYO_OK;
}

// internal line-major field: one double, or one float pair, per node
static size_t field_bytes(const cryo_plan *p) {
    size_t b = 8 * (size_t)p->nz * p->np;
    return (b + 255) & ~(size_t)255;
}

cryo_status cryo_workspace_bytes(const cryo_plan *p, int64_t nsteps, size_t *bytes) {
    if (!p || !bytes || nsteps < 0) return fail(CRYO_ERR_ARG, "bad argument");
    size_t part = sizeof(double) * (size_t)SURF_CHUNK * step_grid(p);
    *bytes = 256 + 2 * field_bytes(p) + ((part + 255) & ~(size_t)255);
    return CRYO_OK;
}

cryo_status cryo_init(const cryo_plan *p, void *T, void *stream) {
    if (!p || !T) return fail(CRYO_ERR_ARG, "null argument");
    return launch_fill(p, T, (hipStream_t)stream);
}

}  // extern "C"

// Workspace (and resident state) layout: the error word, the two field
// buffers of the kernels' internal layout (ping-pong), then the per-workgroup
// surface partial sums of up to SURF_CHUNK steps.
static cryo_status check_ws(const cryo_plan *p, const void *ws, size_t ws_bytes) {
    size_t need = 0;
    cryo_workspace_bytes(p, 0, &need);
    if (!ws || ws_bytes < need)
        return fail(CRYO_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(CRYO_ERR_WORKSPACE, "workspace must be 256-aligned");
    return CRYO_OK;
}

static cryo_status plan_on_device(const cryo_plan *p) {
    cryo_status st = ensure_device(const_cast<cryo_plan *>(p));
    if (st == CRYO_OK && p->sub) st = ensure_device(p->sub);
    return st;
}

// nsteps steps from global step k0 on the internal fields of workspace w,
// starting from buffer *cur; *cur names the buffer holding the result.
static cryo_status run_steps(const cryo_plan *p, char *w, int *cur_io, int64_t k0,
                             int64_t nsteps, double *surf, hipStream_t s) {
    int *flag = (int *)w;
    void *buf[2] = {w + 256, w + 256 + field_bytes(p)};
    double *part = (double *)(w + 256 + 2 * field_bytes(p));
    cryo_status st = CRYO_OK;
    int G = step_grid(p);
    int64_t done_surf = 0;
    int cur = *cur_io;
    for (int64_t n = 0; n < nsteps; ++n) {
        double *pp = surf ? part + (size_t)(n % SURF_CHUNK) * G : nullptr;
        if (p->sub && pulse_start(p->pulse, k0 + n)) {
            // eq. (22): the pulse's first step as 100 sub-steps of dt / 100
            // (same layout and launch shape; the last one reports the surface)
            for (int i = 0; i < 100 && st == CRYO_OK; ++i) {
                double X = p->pulse.amplitude * turn_on_source(p->pulse, k0 + n, i);
                st = launch_step(p->sub, buf[cur], buf[cur ^ 1], X, i == 99 ? pp : nullptr, flag, s);
                cur ^= 1;
            }
        } else {
            double X = p->pulse.amplitude * source_fraction(p->pulse, k0 + n);
            st = launch_step(p, buf[cur], buf[cur ^ 1], X, pp, flag, s);
            cur ^= 1;
        }
        if (st != CRYO_OK) return st;
        *cur_io = cur;
        if (surf && ((n + 1) % SURF_CHUNK == 0 || n + 1 == nsteps)) {
            int cnt = (int)(n + 1 - done_surf);
            st = launch_surf_reduce(p, part, cnt, surf + done_surf, s);
            if (st != CRYO_OK) return st;
            done_surf = n + 1;
        }
    }
    return CRYO_OK;
}

namespace cryo {
// The forward of cryo_forward on a checked workspace `w` (error word, two
// internal fields, surface partials) of a plan whose device tables exist.
cryo_status forward_in(const cryo_plan *p, void *T, int64_t k0, int64_t nsteps, char *w,
                       double *surf, hipStream_t s) {
    int *flag = (int *)w;
    int cur = 0;
    // the conversion kernel also clears the non-finite flag
    cryo_status st = launch_to_internal(p, T, w + 256, flag, s);
    if (st == CRYO_OK) st = run_steps(p, w, &cur, k0, nsteps, surf, s);
    if (st != CRYO_OK) return st;
    return launch_from_internal(p, w + 256 + cur * field_bytes(p), T, flag, s);
}

bool plan_tables_on_device(const cryo_plan *p) {
    return p->d_info != nullptr && (!p->sub || p->sub->d_info != nullptr);
}
}  // namespace cryo

// Resident state: the caller's workspace holding the field in the internal
// layout between calls, and which of its two buffers is current.  Calls on
// one state are ordered by the stream, so the host knows the current buffer.
struct cryo_state {
    const cryo_plan *plan;
    char *mem;
    int cur;
};

extern "C" {

cryo_status cryo_forward(const cryo_plan *p, void *T, int64_t k0, int64_t nsteps, void *ws,
                         size_t ws_bytes, double *surf, void *stream) {
    if (!p || !T || nsteps < 0 || k0 < 0) return fail(CRYO_ERR_ARG, "bad argument");
    cryo_status st = check_ws(p, ws, ws_bytes);
    if (st == CRYO_OK) st = plan_on_device(p);
    if (st != CRYO_OK) return st;
    return cryo::forward_in(p, T, k0, nsteps, (char *)ws, surf, (hipStream_t)stream);
}

cryo_status cryo_state_create(const cryo_plan *p, void *mem, size_t bytes, cryo_state **out) {
    if (!p || !out) return fail(CRYO_ERR_ARG, "null argument");
    *out = nullptr;
    cryo_status st = check_ws(p, mem, bytes);
    if (st == CRYO_OK) st = plan_on_device(p);
    if (st != CRYO_OK) return st;
    cryo_state *z = new cryo_state();
    z->plan = p;
    z->mem = (char *)mem;
    z->cur = 0;
    *out = z;
    return CRYO_OK;
}

void cryo_state_destroy(cryo_state *z) { delete z; }

cryo_status cryo_state_load(cryo_state *z, const void *T, void *stream) {
    if (!z || !T) return fail(CRYO_ERR_ARG, "null argument");
    z->cur = 0;
    return launch_to_internal(z->plan, T, z->mem + 256, (int *)z->mem, (hipStream_t)stream);
}

cryo_status cryo_state_forward(cryo_state *z, int64_t k0, int64_t nsteps, double *surf,
                               void *stream) {
    if (!z || nsteps < 0 || k0 < 0) return fail(CRYO_ERR_ARG, "bad argument");
    return run_steps(z->plan, z->mem, &z->cur, k0, nsteps, surf, (hipStream_t)stream);
}

cryo_status cryo_state_store(const cryo_state *z, void *T, void *stream) {
    if (!z || !T) return fail(CRYO_ERR_ARG, "null argument");
    const cryo_plan *p = z->plan;
    return launch_from_internal(p, z->mem + 256 + z->cur * field_bytes(p), T, (int *)z->mem,
                                (hipStream_t)stream);
}

cryo_status cryo_poll(const cryo_plan *p, const void *ws, void *stream) {
    if (!p || !ws) return fail(CRYO_ERR_ARG, "null argument");
    int flag = 0;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&flag, ws, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(CRYO_ERR_DEVICE, "poll copy failed");
    if (flag) return fail(CRYO_ERR_NONFINITE, "non-finite temperature, or one outside the "
                                              "supported range [1/16 K, 2^20 K), produced");
    return CRYO_OK;
}

}  // extern "C"
