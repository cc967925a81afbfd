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

// Average of the rectangular gate of eq. (4) over step k, all times in step
// units: pulses occupy [b0 + n P, b0 + n P + W), n >= 0.
double source_fraction(const Pulse &p, int64_t k) {
    if (!(p.W > 0)) return 0.0;
    double lo = (double)k, hi = lo + 1.0, s = 0.0;
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
    const cryo_pulse &pu = pr->pulse;
    if (pu.layer < 0 || pu.layer >= g.n_layers)
        return fail(CRYO_ERR_ARG, "heater layer index out of range");
    if (!(pu.period > 0) || !(pu.width >= 0) || pu.width > pu.period || !(pu.t_on >= 0) ||
        !std::isfinite(pu.amplitude))
        return fail(CRYO_ERR_ARG, "pulse needs period > 0, 0 <= width <= period, t_on >= 0");
    for (int s = 0; s < 4; ++s) {
        if (pr->bc.kind[s] != CRYO_INSULATED && pr->bc.kind[s] != CRYO_HELD)
            return fail(CRYO_ERR_ARG, "boundary kind must be 0 or 1");
        if (pr->bc.kind[s] == CRYO_HELD && !(pr->bc.value[s] > 0))
            return fail(CRYO_ERR_ARG, "held boundary temperature must be > 0");
    }
    if (g.r_inner == 0 && pr->bc.kind[0] != CRYO_INSULATED)
        return fail(CRYO_ERR_ARG, "r_inner = 0 (the axis) must be insulated");
    if (!(pr->dt > 0) || !std::isfinite(pr->dt)) return fail(CRYO_ERR_ARG, "dt must be > 0");
    if (!(pr->T_init > 0)) return fail(CRYO_ERR_ARG, "T_init must be > 0");
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

static int pick_rpl(int nr) {
    int r = 2;
    while (WAVE * r < nr) r *= 2;
    return r;
}

// Device copies of the per-row tables, made once on the first call that
// needs the device (on the device current at that time).
cryo_status ensure_device(cryo_plan *p) {
    if (p->d_info) return CRYO_OK;
    (void)hipGetDevice(&p->device);
    const int np = p->np;
    size_t es = p->dtype == CRYO_F64 ? sizeof(double) : sizeof(float);
    hipError_t e = hipMalloc(&p->d_gw, es * np);
    if (e == hipSuccess) e = hipMalloc(&p->d_ge, es * np);
    uint32_t *info = nullptr;
    if (e == hipSuccess) e = hipMalloc((void **)&info, sizeof(uint32_t) * np);
    if (e == hipSuccess) {
        if (p->dtype == CRYO_F64) {
            e = hipMemcpy(p->d_gw, p->gw.data(), es * np, hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(p->d_ge, p->ge.data(), es * np, hipMemcpyHostToDevice);
        } else {
            std::vector<float> a(p->gw.begin(), p->gw.end()), b(p->ge.begin(), p->ge.end());
            e = hipMemcpy(p->d_gw, a.data(), es * np, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(p->d_ge, b.data(), es * np, hipMemcpyHostToDevice);
        }
    }
    if (e == hipSuccess)
        e = hipMemcpy(info, p->info.data(), sizeof(uint32_t) * np, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (p->d_gw) (void)hipFree(p->d_gw);
        if (p->d_ge) (void)hipFree(p->d_ge);
        if (info) (void)hipFree(info);
        p->d_gw = p->d_ge = nullptr;
        return fail(CRYO_ERR_DEVICE, std::string("device table upload: ") + hipGetErrorString(e));
    }
    p->d_info = info;
    return CRYO_OK;
}

}  // namespace cryo

using namespace cryo;

extern "C" {

const char *cryo_last_error(void) { return g_err.c_str(); }

const char *cryo_version(void) { return "cryocell 0.1 (gfx950)"; }

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
    p->rpl = pick_rpl(p->nr);
    p->np = WAVE * p->rpl;
    p->eta = prob->geom.height / (p->nz - 1);
    const int nr = p->nr, L = p->L, np = p->np, rpl = p->rpl;

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

    // laws: radial 0..L-1, axial (divided by eta^2) L..2L-1, capacity
    Laws &lw = p->laws;
    memset(&lw, 0, sizeof(lw));
    lw.L = L;
    lw.n = 2 * L;
    for (int m = 0; m < L; ++m) {
        const cryo_material &mt = p->layers[m].mat;
        double lk = log2(mt.k_scale * mt.k0) - mt.p * log2(mt.tref);
        lw.p[m] = mt.p;
        lw.lk[m] = lk;
        lw.p[L + m] = mt.p;
        lw.lk[L + m] = lk - log2(p->eta * p->eta);
        lw.q[m] = mt.q;
        lw.lrc[m] = log2(mt.rho * mt.c0 / prob->dt) - mt.q * log2(mt.tref);
    }

    // lane-major per-row tables: row i = lane * rpl + reg sits at reg * 64 + lane
    p->gw.assign(np, 0.0);
    p->ge.assign(np, 0.0);
    p->info.assign(np, info_pack(K_PAD, 0, 0, 0, 0, 0));
    for (i = 0; i < nr; ++i) {
        int idx = (i % rpl) * WAVE + i / rpl;
        uint32_t kind = p->kind[i];
        uint32_t lawE = (i < nr - 1) ? p->lay[i + 1] : 0;
        uint32_t m = p->lay[i];
        uint32_t law2 = 0, law3 = 0, heat = 0;
        if (kind == K_CAP) {
            // eq. (13): A = -r_{i-1/2} lam_{i-1/2} / (r_i hbar_i h_i), C likewise
            double hb = 0.5 * (p->h[i] + p->h[i + 1]);
            p->gw[idx] = 0.5 * (p->r[i] + p->r[i - 1]) / (p->r[i] * hb * p->h[i]);
            p->ge[idx] = 0.5 * (p->r[i] + p->r[i + 1]) / (p->r[i] * hb * p->h[i + 1]);
            law2 = law3 = L + m;
            heat = (int)m == prob->pulse.layer ? 1u : 0u;
        } else if (kind == K_IFACE) {
            // eq. (18): lam*_m h_{i+1} (T_i - T_{i-1}) = lam*_{m+1} h_i (T_{i+1} - T_i)
            p->gw[idx] = p->h[i + 1];
            p->ge[idx] = p->h[i];
            law2 = p->lay[i];
            law3 = p->lay[i + 1];
        }
        p->info[idx] = info_pack(kind, heat, lawE, law2, law3, m);
    }
    p->surf_lane = (nr - 1) / rpl;
    p->surf_reg = (nr - 1) % rpl;
    p->pulse.b0 = snap(prob->pulse.t_on / prob->dt);
    p->pulse.W = snap(prob->pulse.width / prob->dt);
    p->pulse.P = snap(prob->pulse.period / prob->dt);
    p->pulse.amplitude = prob->pulse.amplitude;

    *out = p;
    return CRYO_OK;
}

void cryo_plan_destroy(cryo_plan *p) {
    if (!p) return;
    if (p->d_gw) (void)hipFree(p->d_gw);
    if (p->d_ge) (void)hipFree(p->d_ge);
    if (p->d_info) (void)hipFree(p->d_info);
    delete p;
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

cryo_status cryo_forward(const cryo_plan *p, void *T, int64_t k0, int64_t nsteps, void *ws,
                         size_t ws_bytes, double *surf, void *stream) {
    if (!p || !T || nsteps < 0 || k0 < 0) return fail(CRYO_ERR_ARG, "bad argument");
    size_t need = 0;
    cryo_workspace_bytes(p, nsteps, &need);
    if (!ws || ws_bytes < need)
        return fail(CRYO_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(CRYO_ERR_WORKSPACE, "workspace must be 256-aligned");
    cryo_status st0 = ensure_device(const_cast<cryo_plan *>(p));
    if (st0 != CRYO_OK) return st0;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    int *flag = (int *)w;
    void *buf[2] = {w + 256, w + 256 + field_bytes(p)};
    double *part = (double *)(w + 256 + 2 * field_bytes(p));
    // the conversion kernel also clears the non-finite flag
    cryo_status st = launch_to_internal(p, T, buf[0], flag, s);
    if (st != CRYO_OK) return st;
    int G = step_grid(p);
    int64_t done_surf = 0;
    for (int64_t n = 0; n < nsteps; ++n) {
        double X = p->pulse.amplitude * source_fraction(p->pulse, k0 + n);
        double *pp = surf ? part + (size_t)(n % SURF_CHUNK) * G : nullptr;
        st = launch_step(p, buf[n & 1], buf[(n + 1) & 1], X, pp, s);
        if (st != CRYO_OK) return st;
        if (surf && ((n + 1) % SURF_CHUNK == 0 || n + 1 == nsteps)) {
            int cnt = (int)(n + 1 - done_surf);
            st = launch_surf_reduce(p, part, cnt, surf + done_surf, s);
            if (st != CRYO_OK) return st;
            done_surf = n + 1;
        }
    }
    return launch_from_internal(p, buf[nsteps & 1], T, flag, s);
}

cryo_status cryo_poll(const cryo_plan *p, const void *ws, void *stream) {
    if (!p || !ws) return fail(CRYO_ERR_ARG, "null argument");
    int flag = 0;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&flag, ws, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(CRYO_ERR_DEVICE, "poll copy failed");
    if (flag) return fail(CRYO_ERR_NONFINITE, "non-finite temperature produced");
    return CRYO_OK;
}

}  // extern "C"
