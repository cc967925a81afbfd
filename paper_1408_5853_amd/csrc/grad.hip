// Gradient driver: J = sum_{n=1..N} (S_n - target_n)^2 of the surface mean S
// and dJ/d[amplitude, width, thickness_m, k_scale_m] by the discrete
// adjoint, with checkpoints every K steps and recompute of each segment.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

namespace cryo {

cryo_status launch_adj(const cryo_plan *p, int pass, const AdjArgs &d, int *flag, hipStream_t s,
                       const AdjArgs *d1 = nullptr);
cryo_status launch_adj_init(const cryo_plan *p, double *lam, double cS, hipStream_t s);
cryo_status launch_zero(double *ptr, size_t n, hipStream_t s);
int adj_slots(const cryo_plan *p);
size_t adj_lds(const cryo_plan *p);

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// d/d(width) of the pulse average of step k (step units in, 1/s out): a pulse
// end inside the step counts fully, one on a step boundary half on each side
static double source_fraction_dwidth(const Pulse &p, double dt, int64_t k) {
    if (!(p.W > 0)) return 0.0;
    double lo = (double)k, hi = lo + 1.0, d = 0.0;
    int64_t n = (int64_t)floor((lo - p.b0 - p.W) / p.P);
    if (n < 0) n = 0;
    for (;; ++n) {
        double b = p.b0 + (double)n * p.P;
        if (b >= hi) break;
        double e = b + p.W;
        if (e > lo && e < hi) d += 1.0;
        else if (e == lo || e == hi) d += 0.5;
    }
    return d / dt;
}

// The kernel steps (launches) of a run of N steps: one per step, or, with
// the turn-on model (eq. (22)), the 100 sub-steps of dt/100 of each
// pulse-start step.  Each carries its source factor, that factor's width
// derivative [1/s], and the step whose surface it completes (1..N, 0 none).
struct Launch {
    bool sub;
    double s, ds;
    int64_t obs;
};

// d/d(width) of sub-step i's factor: the gate average's derivative over the
// sub-step (a pulse end inside counts fully, on its boundary half) times p^2
static double turn_on_source_dwidth(const Pulse &p, double dt, int64_t k, int i) {
    if (!(p.W > 0)) return 0.0;
    const double lo = (double)k + (double)i / 100.0, hi = (double)k + (double)(i + 1) / 100.0;
    double d = 0.0;
    int64_t n = (int64_t)floor((lo - p.b0 - p.W) / p.P);
    if (n < 0) n = 0;
    for (;; ++n) {
        const double b = p.b0 + (double)n * p.P;
        if (b >= hi) break;
        const double e = b + p.W;
        if (e > lo && e < hi) d += 1.0;
        else if (e == lo || e == hi) d += 0.5;
    }
    return d / ((hi - lo) * dt) * (1.0 - exp(-(double)i / 7.0));
}

static std::vector<Launch> launch_list(const cryo_plan *p, int64_t N) {
    std::vector<Launch> v;
    v.reserve((size_t)std::max<int64_t>(N, 0));
    for (int64_t k = 0; k < N; ++k) {
        if (p->sub && pulse_start(p->pulse, k)) {
            for (int i = 0; i < 100; ++i)
                v.push_back({true, turn_on_source(p->pulse, k, i),
                             turn_on_source_dwidth(p->pulse, p->prob.dt, k, i), i == 99 ? k + 1 : 0});
        } else {
            v.push_back({false, source_fraction(p->pulse, k),
                         source_fraction_dwidth(p->pulse, p->prob.dt, k), k + 1});
        }
    }
    return v;
}

static int64_t launch_count(const cryo_plan *p, int64_t N) {
    int64_t m = N;
    if (p->sub)
        for (int64_t k = 0; k < N; ++k) m += pulse_start(p->pulse, k) ? 99 : 0;
    return m;
}

struct GradLayout {
    size_t flag, fwd_buf[2], part, ck, seg, lam[2], Y[2], lpart[2], acc, accg, surf, total;
    int64_t nck, K;
};

// checkpoints every K kernel steps (sub-steps of the turn-on model count)
static GradLayout grad_layout(const cryo_plan *p, int64_t N, int64_t ckpt) {
    GradLayout g;
    const size_t F = al256(8 * (size_t)p->nz * p->np);
    const int64_t M = launch_count(p, N);
    int64_t K = ckpt > 0 ? ckpt : (int64_t)ceil(sqrt((double)std::max<int64_t>(M, 1)));
    K = std::max<int64_t>(1, std::min<int64_t>(K, std::max<int64_t>(M, 1)));
    g.K = K;
    g.nck = (M + K - 1) / K;
    size_t o = 0;
    g.flag = o; o += 256;
    g.fwd_buf[0] = o; o += F;
    g.fwd_buf[1] = o; o += F;
    g.part = o; o += al256(sizeof(double) * (size_t)SURF_CHUNK * step_grid(p));
    g.ck = o; o += F * (size_t)std::max<int64_t>(g.nck, 1);
    g.seg = o; o += F * (size_t)(K + 1);
    g.lam[0] = o; o += F;
    g.lam[1] = o; o += F;
    // y and the radial part of lam, by step parity (the fused passes read
    // step k's while writing step k-1's)
    g.Y[0] = o; o += F;
    g.Y[1] = o; o += F;
    g.lpart[0] = o; o += F;
    g.lpart[1] = o; o += F;
    g.acc = o; o += al256(sizeof(double) * 3 * (size_t)p->np * adj_slots(p));
    g.accg = o; o += al256(sizeof(double) * 2 * (size_t)adj_slots(p));
    g.surf = o; o += al256(sizeof(double) * (size_t)std::max<int64_t>(N, 1));
    g.total = o;
    return g;
}

}  // namespace cryo

namespace cryo {

// One gradient in phases, so that many can be in flight on several streams:
// enqueue the forward with checkpoints, read the surface trace (J and the
// adjoint seeds), enqueue the backward sweep, reduce the sums on the host.
struct GradRun {
    cryo_plan *p;
    const void *T0;
    int64_t N;
    const double *target;
    char *w;
    GradLayout g;
    hipStream_t s;
    std::vector<double> S, cS;
    double J;
    std::vector<Launch> L;    // the run's kernel steps
};

static cryo_status grad_check(const cryo_plan *p, int64_t N, const double *target, int64_t ckpt,
                              const void *T0, void *ws, size_t ws_bytes) {
    if (!p || !T0 || N < 1 || !target || ckpt < 0) return fail(CRYO_ERR_ARG, "bad argument");
    if (p->dtype != CRYO_F64) return fail(CRYO_ERR_UNSUPPORTED, "the adjoint needs an FP64 plan");
    if (p->poly) return fail(CRYO_ERR_UNSUPPORTED, "no adjoint of the polynomial laws");
    if (adj_lds(p) > MAX_STEP_LDS)
        return fail(CRYO_ERR_UNSUPPORTED, "the adjoint's tables exceed a workgroup's LDS for this "
                                          "shape; choose fewer rows per line");
    const int key = p->rpl * 10 + p->wpl;
    if (!(key == 21 || key == 41 || key == 81 || key == 42 || key == 82 || key == 44 || key == 84))
        return fail(CRYO_ERR_UNSUPPORTED, "the adjoint kernels take 2, 4 or 8 rows per lane; set "
                                          "such a shape before the plan's first run");
    const GradLayout g = grad_layout(p, N, ckpt);
    if (!ws || ws_bytes < g.total)
        return fail(CRYO_ERR_WORKSPACE, "gradient workspace needs " + std::to_string(g.total) +
                                            " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(CRYO_ERR_WORKSPACE, "workspace must be 256-aligned");
    return CRYO_OK;
}

static size_t field_f64(const cryo_plan *p) { return al256(8 * (size_t)p->nz * p->np); }

// forward with checkpoints and the surface trace (enqueued on r.s)
static cryo_status grad_forward(GradRun &r) {
    cryo_plan *p = r.p;
    cryo_status st = ensure_device(p);
    if (st == CRYO_OK && p->sub) st = ensure_device(p->sub);
    if (st != CRYO_OK) return st;
    r.L = launch_list(p, r.N);
    const GradLayout &g = r.g;
    char *w = r.w;
    hipStream_t s = r.s;
    int *flag = (int *)(w + g.flag);
    const size_t F = field_f64(p);
    double *surf = (double *)(w + g.surf);
    double *part = (double *)(w + g.part);
    const int G = step_grid(p);
    st = launch_to_internal(p, r.T0, w + g.fwd_buf[0], flag, s);
    if (st != CRYO_OK) return st;
    int64_t done = 0;
    const int64_t M = (int64_t)r.L.size();
    for (int64_t l = 0; l < M; ++l) {
        const Launch &ln = r.L[l];
        void *cur = w + g.fwd_buf[l & 1], *nxt = w + g.fwd_buf[(l + 1) & 1];
        if (l % g.K == 0 && hipMemcpyAsync(w + g.ck + F * (l / g.K), cur, F,
                                           hipMemcpyDeviceToDevice, s) != hipSuccess)
            return fail(CRYO_ERR_DEVICE, "checkpoint copy");
        const double X = p->pulse.amplitude * ln.s;
        double *pp = ln.obs > 0 ? part + (size_t)((ln.obs - 1) % SURF_CHUNK) * G : nullptr;
        st = launch_step(ln.sub ? p->sub : p, cur, nxt, X, pp, flag, s);
        if (st != CRYO_OK) return st;
        if (ln.obs > 0 && (ln.obs % SURF_CHUNK == 0 || ln.obs == r.N)) {
            st = launch_surf_reduce(p, part, (int)(ln.obs - done), surf + done, s);
            if (st != CRYO_OK) return st;
            done = ln.obs;
        }
    }
    // the final state sits in fwd_buf[M & 1]: the surface trace is all the
    // backward sweep needs from it
    return CRYO_OK;
}

// wait for the forward, read the trace: J and the seeds dJ/dS_n
static cryo_status grad_objective(GradRun &r) {
    r.S.assign(r.N, 0.0);
    if (hipMemcpyAsync(r.S.data(), r.w + r.g.surf, sizeof(double) * r.N, hipMemcpyDeviceToHost,
                       r.s) != hipSuccess ||
        hipStreamSynchronize(r.s) != hipSuccess)
        return fail(CRYO_ERR_DEVICE, "surface trace copy");
    r.J = 0.0;
    r.cS.assign(r.N + 1, 0.0);
    for (int64_t n = 1; n <= r.N; ++n) {
        const double dv = r.S[n - 1] - r.target[n - 1];
        r.J += dv * dv;
        r.cS[n] = 2.0 * dv;
    }
    return CRYO_OK;
}

// segments backwards: restore the checkpoint, recompute, adjoint steps
static cryo_status grad_backward(GradRun &r) {
    cryo_plan *p = r.p;
    const GradLayout &g = r.g;
    char *w = r.w;
    hipStream_t s = r.s;
    int *flag = (int *)(w + g.flag);
    const size_t F = field_f64(p);
    auto ckp = [&](int64_t i) { return (double *)(w + g.ck + F * i); };
    auto segp = [&](int64_t i) { return (double *)(w + g.seg + F * i); };
    const int ngrp = adj_slots(p);
    double *acc = (double *)(w + g.acc), *accg = (double *)(w + g.accg);
    cryo_status st = launch_zero(acc, 3 * (size_t)p->np * ngrp, s);
    if (st == CRYO_OK) st = launch_zero(accg, 2 * (size_t)ngrp, s);
    double *lam[2] = {(double *)(w + g.lam[0]), (double *)(w + g.lam[1])};
    if (st == CRYO_OK) st = launch_adj_init(p, lam[0], r.cS[r.N], s);
    if (st != CRYO_OK) return st;
    int cur = 0;
    const int64_t M = (int64_t)r.L.size();
    // the plan whose tables step launch k (the turn-on sub-steps: dt / 100)
    auto plan_of = [&](int64_t k) { return r.L[k].sub ? p->sub : p; };
    for (int64_t sg = g.nck - 1; sg >= 0; --sg) {
        const int64_t a = sg * g.K, b = std::min<int64_t>(M, a + g.K);
        if (hipMemcpyAsync(segp(0), ckp(sg), F, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return fail(CRYO_ERR_DEVICE, "checkpoint restore");
        for (int64_t k = a; k < b; ++k) {
            const double X = p->pulse.amplitude * r.L[k].s;
            st = launch_step(plan_of(k), segp(k - a), segp(k - a + 1), X, nullptr, flag, s);
            if (st != CRYO_OK) return st;
        }
        // adjoint step k: pass 1 reads lam^{k+1} (lam[cur]) and writes y^k,
        // pass 2 writes lam^k (lam[cur ^ 1]); pass 2 of step k and pass 1 of
        // step k-1 run as one launch inside the segment
        auto args = [&](int64_t k, int c) {
            AdjArgs d;
            d.T = segp(k - a);
            d.X = segp(k - a + 1);
            d.lam_in = lam[c];
            d.Y = (double *)(w + g.Y[k & 1]);
            d.lpart = (double *)(w + g.lpart[k & 1]);
            d.lam_out = lam[c ^ 1];
            d.acc = acc;
            d.accg = accg;
            d.s = r.L[k].s;
            d.ds = r.L[k].ds;
            // the state before launch k is observed when launch k-1 ends a step
            d.cS = k >= 1 && r.L[k - 1].obs > 0 ? r.cS[r.L[k - 1].obs] : 0.0;
            d.xs = p->eta * p->eta;
            return d;
        };
        // pass 1 (the line solves, with the capacity term) runs on the tables
        // of its own launch; pass 2 (axial faces) needs no capacity law, so
        // the fused launch takes those of its pass 1
        st = launch_adj(plan_of(b - 1), 1, args(b - 1, cur), flag, s);
        for (int64_t k = b - 1; k > a && st == CRYO_OK; --k) {
            const AdjArgs d2 = args(k, cur), d1 = args(k - 1, cur ^ 1);
            st = launch_adj(plan_of(k - 1), 21, d2, flag, s, &d1);
            cur ^= 1;
        }
        if (st == CRYO_OK) st = launch_adj(plan_of(a), 2, args(a, cur), flag, s);
        if (st != CRYO_OK) return st;
        cur ^= 1;
    }
    return CRYO_OK;
}

// wait for the backward; row sums over workgroup slots (fixed order), then the
// parameter gradient
static cryo_status grad_finish(GradRun &run, double *grad) {
    cryo_plan *p = run.p;
    const GradLayout &g = run.g;
    char *w = run.w;
    hipStream_t s = run.s;
    const int ngrp = adj_slots(p);
    const double *acc = (const double *)(w + g.acc), *accg = (const double *)(w + g.accg);
    std::vector<double> hacc(3 * (size_t)p->np * ngrp), hg(2 * (size_t)ngrp);
    int hflag = 0;
    if (hipMemcpyAsync(hacc.data(), acc, sizeof(double) * hacc.size(), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(hg.data(), accg, sizeof(double) * hg.size(), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(&hflag, w + g.flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(CRYO_ERR_DEVICE, "gradient sums copy");
    if (hflag) return fail(CRYO_ERR_NONFINITE, "non-finite or out-of-range temperature produced");
    const int nr = p->nr, L = p->L, np = p->np, rpl = p->rpl, NL = np / rpl;
    std::vector<double> SW(nr, 0.0), SE(nr, 0.0), SZ(nr, 0.0);
    for (int i = 0; i < nr; ++i) {
        const int q = (i % rpl) * NL + i / rpl;
        for (int gi = 0; gi < ngrp; ++gi) {
            const double *A = hacc.data() + (size_t)gi * 3 * np;
            SW[i] += A[q];
            SE[i] += A[np + q];
            SZ[i] += A[2 * np + q];
        }
    }
    double gQ = 0.0, gW = 0.0;
    for (int gi = 0; gi < ngrp; ++gi) {
        gQ += hg[2 * gi];
        gW += hg[2 * gi + 1];
    }
    // geometry derivatives: h_i = thick_m / n_m for intervals of layer m,
    // r_i = r_inner + sum of h up to i
    std::vector<double> dr((size_t)nr * L, 0.0), dh((size_t)(nr + 1) * L, 0.0);
    for (int i = 1; i < nr; ++i) {
        const int m = p->lay[i];
        dh[(size_t)i * L + m] = 1.0 / p->layers[m].intervals;
        for (int l = 0; l < L; ++l) dr[(size_t)i * L + l] = dr[(size_t)(i - 1) * L + l] + dh[(size_t)i * L + l];
    }
    std::vector<double> gd(L, 0.0), gs(L, 0.0);
    const std::vector<double> &r = p->r, &h = p->h;
    for (int i = 1; i < nr - 1; ++i) {
        if (p->kind[i] == K_CAP) {
            const int m = p->lay[i];
            gs[m] -= (SW[i] + SE[i] - SZ[i]) / p->layers[m].mat.k_scale;
            const double rw = 0.5 * (r[i] + r[i - 1]), re = 0.5 * (r[i] + r[i + 1]);
            const double hb = 0.5 * (h[i] + h[i + 1]);
            for (int l = 0; l < L; ++l) {
                const double dri = dr[(size_t)i * L + l];
                const double drw = 0.5 * (dri + dr[(size_t)(i - 1) * L + l]);
                const double dre = 0.5 * (dri + dr[(size_t)(i + 1) * L + l]);
                const double dhi = dh[(size_t)i * L + l], dhe = dh[(size_t)(i + 1) * L + l];
                const double dhb = 0.5 * (dhi + dhe);
                const double wW = drw / rw - dri / r[i] - dhb / hb - dhi / h[i];
                const double wE = dre / re - dri / r[i] - dhb / hb - dhe / h[i + 1];
                gd[l] -= SW[i] * wW + SE[i] * wE;
            }
        } else if (p->kind[i] == K_IFACE) {
            const int a = p->lay[i], b = p->lay[i + 1];
            gs[a] -= SW[i] / p->layers[a].mat.k_scale;
            gs[b] -= SE[i] / p->layers[b].mat.k_scale;
            for (int l = 0; l < L; ++l)
                gd[l] -= SW[i] * dh[(size_t)(i + 1) * L + l] / h[i + 1] +
                         SE[i] * dh[(size_t)i * L + l] / h[i];
        }
    }
    grad[0] = gQ;
    grad[1] = gW;
    for (int l = 0; l < L; ++l) {
        grad[2 + l] = gd[l];
        grad[2 + L + l] = gs[l];
    }
    return CRYO_OK;
}

}  // namespace cryo

using namespace cryo;

extern "C" {

cryo_status cryo_gradient_workspace_bytes(const cryo_plan *p, int64_t nsteps, int64_t ckpt,
                                          size_t *bytes) {
    if (!p || !bytes || nsteps < 1 || ckpt < 0) return fail(CRYO_ERR_ARG, "bad argument");
    *bytes = grad_layout(p, nsteps, ckpt).total;
    return CRYO_OK;
}

cryo_status cryo_gradient(const cryo_plan *pc, const void *T0, int64_t N, const double *target,
                          int64_t ckpt, void *ws, size_t ws_bytes, double *J, double *grad,
                          double *surf_out, void *stream) {
    if (!J || !grad) return fail(CRYO_ERR_ARG, "bad argument");
    cryo_status st = grad_check(pc, N, target, ckpt, T0, ws, ws_bytes);
    if (st != CRYO_OK) return st;
    GradRun r;
    r.p = const_cast<cryo_plan *>(pc);
    r.T0 = T0;
    r.N = N;
    r.target = target;
    r.w = (char *)ws;
    r.g = grad_layout(pc, N, ckpt);
    r.s = (hipStream_t)stream;
    st = grad_forward(r);
    if (st == CRYO_OK) st = grad_objective(r);
    if (st == CRYO_OK) st = grad_backward(r);
    if (st == CRYO_OK) st = grad_finish(r, grad);
    if (st != CRYO_OK) return st;
    *J = r.J;
    if (surf_out) memcpy(surf_out, r.S.data(), sizeof(double) * N);
    return CRYO_OK;
}

cryo_status cryo_gradient_many(int32_t n, cryo_plan *const *plans, const void *const *T0,
                               int64_t N, const double *const *targets, int64_t ckpt,
                               void *const *ws, const size_t *ws_bytes, int32_t n_streams,
                               double *J, double *const *grad, double *const *surf_out) {
    if (n < 1 || !plans || !T0 || !targets || !ws || !ws_bytes || !J || !grad || n_streams < 1)
        return fail(CRYO_ERR_ARG, "bad argument");
    for (int i = 0; i < n; ++i) {
        cryo_status st = grad_check(plans[i], N, targets[i], ckpt, T0[i], ws[i], ws_bytes[i]);
        if (st != CRYO_OK) return fail(st, "design " + std::to_string(i) + ": " + cryo_last_error());
        if (!grad[i]) return fail(CRYO_ERR_ARG, "design " + std::to_string(i) + ": null grad");
    }
    const int ns = std::min<int>(n_streams, n);
    std::vector<hipStream_t> streams(ns, nullptr);
    cryo_status st = CRYO_OK;
    for (int k = 0; k < ns && st == CRYO_OK; ++k)
        if (hipStreamCreateWithFlags(&streams[k], hipStreamNonBlocking) != hipSuccess)
            st = fail(CRYO_ERR_DEVICE, "stream creation");
    std::vector<GradRun> runs(n);
    for (int i = 0; i < n && st == CRYO_OK; ++i) {
        GradRun &r = runs[i];
        r.p = plans[i];
        r.T0 = T0[i];
        r.N = N;
        r.target = targets[i];
        r.w = (char *)ws[i];
        r.g = grad_layout(plans[i], N, ckpt);
        r.s = streams[i % ns];
    }
    // all forwards in flight, then each trace as it completes, then all
    // backward sweeps, then the reductions
    for (int i = 0; i < n && st == CRYO_OK; ++i) st = grad_forward(runs[i]);
    for (int i = 0; i < n && st == CRYO_OK; ++i) st = grad_objective(runs[i]);
    for (int i = 0; i < n && st == CRYO_OK; ++i) st = grad_backward(runs[i]);
    for (int i = 0; i < n && st == CRYO_OK; ++i) {
        st = grad_finish(runs[i], grad[i]);
        if (st == CRYO_OK) {
            J[i] = runs[i].J;
            if (surf_out && surf_out[i]) memcpy(surf_out[i], runs[i].S.data(), sizeof(double) * N);
        } else {
            st = fail(st, "design " + std::to_string(i) + ": " + cryo_last_error());
        }
    }
    for (hipStream_t x : streams)
        if (x) {
            (void)hipStreamSynchronize(x);
            (void)hipStreamDestroy(x);
        }
    return st;
}

}  // extern "C"
