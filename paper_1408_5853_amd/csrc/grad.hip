// Gradient driver: J = sum_{n=1..N} (S_n - target_n)^2 of the surface mean S
// and dJ/d[amplitude, width, thickness_m, k_scale_m] by the discrete
// adjoint: the states of the last steps kept from the forward as far as the
// plan's store reaches, checkpoints every K steps before them and recompute
// of each segment.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "internal.h"

namespace cryo {

cryo_status launch_adj(const cryo_plan *p, int pass, const AdjArgs &d, int *flag, hipStream_t s,
                       const AdjArgs *d1 = nullptr);
cryo_status launch_adj_init(const cryo_plan *p, double *lam, const double *cS, hipStream_t s);
cryo_status launch_zero(double *ptr, size_t n, hipStream_t s);
int adj_slots(const cryo_plan *p);
int adj_grid(const cryo_plan *p);
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
    size_t flag, fwd_buf[2], part, ck, seg, store, lam[2], Y[2], lpart[2], acc, accg, surf, tgt,
        seed, rs, out, total;
    int64_t nck, K;
    int64_t H, D;    // head kernel steps (checkpointed, recomputed), stored tail steps
};

// The last D kernel steps (the plan's gradient store, at most all of them)
// keep their states from the forward: T^H .. T^M in D + 1 fields.  The H
// steps before them are checkpointed every K steps and each segment is
// recomputed into a buffer of K fields.
static GradLayout grad_layout_store(const cryo_plan *p, int64_t N, int64_t ckpt, int64_t store,
                                    int64_t M) {
    GradLayout g;
    const size_t F = al256(8 * (size_t)p->nz * p->np);
    g.D = std::min<int64_t>(std::max<int64_t>(store, 0), M);
    g.H = M - g.D;
    int64_t K = ckpt > 0 ? ckpt : (int64_t)ceil(sqrt((double)std::max<int64_t>(g.H, 1)));
    K = std::max<int64_t>(1, std::min<int64_t>(K, std::max<int64_t>(g.H, 1)));
    g.K = K;
    g.nck = (g.H + K - 1) / K;
    size_t o = 0;
    g.flag = o; o += 256;
    g.fwd_buf[0] = o; o += F;
    g.fwd_buf[1] = o; o += F;
    g.part = o; o += al256(sizeof(double) * (size_t)SURF_CHUNK * step_grid(p));
    g.ck = o; o += F * (size_t)g.nck;
    // segment states a+1 .. b (state a is read from its checkpoint)
    g.seg = o; o += g.H > 0 ? F * (size_t)K : 0;
    g.store = o; o += g.D > 0 ? F * (size_t)(g.D + 1) : 0;
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
    // a host target's copy, the seeds dJ/dS_n (n = 0..N), the per-row face
    // sums, and J and grad for a host caller
    g.tgt = o; o += al256(sizeof(double) * (size_t)std::max<int64_t>(N, 1));
    g.seed = o; o += al256(sizeof(double) * (size_t)(N + 1));
    g.rs = o; o += al256(sizeof(double) * 3 * (size_t)p->nr);
    g.out = o; o += al256(sizeof(double) * (3 + 2 * (size_t)p->L));
    g.total = o;
    return g;
}

static GradLayout grad_layout(const cryo_plan *p, int64_t N, int64_t ckpt) {
    return grad_layout_store(p, N, ckpt, p->grad_store, launch_count(p, N));
}

// The largest store (at most all M kernel steps) whose workspace fits in
// `budget`.  Every store d costs at least the fields of d + 9 states (the
// stored ones and the final one, two forward buffers, six adjoint fields)
// beyond the parts that do not depend on it, and at most 2 sqrt(M - d) + 2
// more (checkpoints and segment), so the scan down from that bound is short.
static int64_t store_for_budget(const cryo_plan *p, int64_t N, int64_t ckpt, size_t budget) {
    const int64_t M = launch_count(p, N);
    const size_t F = al256(8 * (size_t)p->nz * p->np);
    const GradLayout all = grad_layout_store(p, N, ckpt, M, M);
    const size_t fixed = all.total - F * (size_t)(M + 9);
    if (budget < fixed + 9 * F) return 0;
    int64_t d = std::min<int64_t>(M, (int64_t)((budget - fixed) / F) - 9);
    for (; d > 0; --d)
        if (grad_layout_store(p, N, ckpt, d, M).total <= budget) return d;
    return 0;
}

// The weights of the parameter gradient, from the geometry: h_i = thick_m /
// n_m on the intervals of layer m and r_i = r_inner + the h up to i, so each
// capacity row's faces (eq. (13)) and each interface row's two one-sided
// fluxes (eq. (18)) move with every thickness, and every face law is
// k_scale_m times the layer's law.  Layout (doubles): W[nr][L] and E[nr][L],
// the thickness weights of a row's west and east face sums; per row {class
// (0 none, 1 capacity, 2 interface), inner layer, outer layer}; k_scale[L].
std::vector<double> grad_param_table(const cryo_plan *p) {
    const int nr = p->nr, L = p->L;
    std::vector<double> t(grad_param_doubles(nr, L), 0.0);
    double *W = t.data(), *E = W + (size_t)nr * L, *rowc = E + (size_t)nr * L;
    double *ks = rowc + 3 * (size_t)nr;
    std::vector<double> dr((size_t)nr * L, 0.0), dh((size_t)(nr + 1) * L, 0.0);
    for (int i = 1; i < nr; ++i) {
        const int m = p->lay[i];
        dh[(size_t)i * L + m] = 1.0 / p->layers[m].intervals;
        for (int l = 0; l < L; ++l) dr[(size_t)i * L + l] = dr[(size_t)(i - 1) * L + l] + dh[(size_t)i * L + l];
    }
    const std::vector<double> &r = p->r, &h = p->h;
    for (int i = 1; i < nr - 1; ++i) {
        if (p->kind[i] == K_CAP) {
            const int m = p->lay[i];
            rowc[3 * i] = 1.0;
            rowc[3 * i + 1] = rowc[3 * i + 2] = m;
            const double rw = 0.5 * (r[i] + r[i - 1]), re = 0.5 * (r[i] + r[i + 1]);
            const double hb = 0.5 * (h[i] + h[i + 1]);
            for (int l = 0; l < L; ++l) {
                const double dri = dr[(size_t)i * L + l];
                const double drw = 0.5 * (dri + dr[(size_t)(i - 1) * L + l]);
                const double dre = 0.5 * (dri + dr[(size_t)(i + 1) * L + l]);
                const double dhi = dh[(size_t)i * L + l], dhe = dh[(size_t)(i + 1) * L + l];
                const double dhb = 0.5 * (dhi + dhe);
                W[(size_t)i * L + l] = drw / rw - dri / r[i] - dhb / hb - dhi / h[i];
                E[(size_t)i * L + l] = dre / re - dri / r[i] - dhb / hb - dhe / h[i + 1];
            }
        } else if (p->kind[i] == K_IFACE) {
            rowc[3 * i] = 2.0;
            rowc[3 * i + 1] = p->lay[i];
            rowc[3 * i + 2] = p->lay[i + 1];
            for (int l = 0; l < L; ++l) {
                W[(size_t)i * L + l] = dh[(size_t)(i + 1) * L + l] / h[i + 1];
                E[(size_t)i * L + l] = dh[(size_t)i * L + l] / h[i];
            }
        }
    }
    for (int m = 0; m < L; ++m) ks[m] = p->layers[m].mat.k_scale;
    return t;
}

// J = sum_n (S_n - target_n)^2 and the seeds seed[n] = dJ/dS_n = 2 (S_n -
// target_n), seed[0] = 0 (the initial state is not observed).  One
// workgroup: each thread sums its strided terms in order, then a fixed tree.
constexpr int OBJ_THREADS = 1024;
__global__ __launch_bounds__(OBJ_THREADS) void k_objective(const double *S, const double *tgt,
                                                           int64_t N, double *seed, double *J) {
    __shared__ double part[OBJ_THREADS];
    const int t = threadIdx.x;
    double a = 0.0;
    for (int64_t n = t; n < N; n += OBJ_THREADS) {
        const double dv = S[n] - tgt[n];
        seed[n + 1] = 2.0 * dv;
        a += dv * dv;
    }
    if (t == 0) seed[0] = 0.0;
    part[t] = a;
    __syncthreads();
    for (int w = OBJ_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0) *J = part[0];
}

// The adjoint's per-row face sums over its workgroup slots, in slot order:
// rs[c * nr + i] for c = west, east, axial and row i (lane-major position q).
__global__ void k_grad_rows(const double *acc, int ngrp, int nr, int np, int rpl, double *rs) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 3 * nr) return;
    const int c = idx / nr, i = idx % nr;
    const int q = (i % rpl) * (np / rpl) + i / rpl;
    double v = 0.0;
    for (int gi = 0; gi < ngrp; ++gi) v += acc[(size_t)gi * 3 * np + (size_t)c * np + q];
    rs[idx] = v;
}

// grad = [amplitude, width, thickness_0..L-1, k_scale_0..L-1], one
// workgroup per parameter: each thread sums its strided terms (the slots'
// source sums, or the rows' face sums times their weights) in order, then a
// fixed tree
constexpr int PAR_THREADS = 256;
__global__ __launch_bounds__(PAR_THREADS) void k_grad_params(const double *rs, const double *accg,
                                                             int ngrp, int nr, int L,
                                                             const double *tab, double *grad) {
    __shared__ double part[PAR_THREADS];
    const double *W = tab, *E = tab + (size_t)nr * L, *rowc = tab + 2 * (size_t)nr * L;
    const double *ks = rowc + 3 * (size_t)nr;
    const double *SW = rs, *SE = rs + nr, *SZ = rs + 2 * (size_t)nr;
    const int t = threadIdx.x, par = blockIdx.x;
    double g = 0.0;
    if (par < 2) {
        for (int gi = t; gi < ngrp; gi += PAR_THREADS) g += accg[2 * gi + par];
    } else if (par < 2 + L) {
        const int l = par - 2;
        for (int i = 1 + t; i < nr - 1; i += PAR_THREADS)
            g -= SW[i] * W[(size_t)i * L + l] + SE[i] * E[(size_t)i * L + l];
    } else {
        const int m = par - 2 - L;
        for (int i = 1 + t; i < nr - 1; i += PAR_THREADS) {
            const double cls = rowc[3 * i];
            const int a = (int)rowc[3 * i + 1], b = (int)rowc[3 * i + 2];
            if (cls == 1.0) {
                if (a == m) g -= (SW[i] + SE[i] - SZ[i]) / ks[m];
            } else if (cls == 2.0) {
                if (a == m) g -= SW[i] / ks[a];
                if (b == m) g -= SE[i] / ks[b];
            }
        }
    }
    part[t] = g;
    __syncthreads();
    for (int w = PAR_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0) grad[par] = part[0];
}

static cryo_status launched(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CRYO_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return CRYO_OK;
}

}  // namespace cryo

namespace cryo {

// One gradient, every phase on one stream with no host wait: the forward
// with checkpoints, J and the seeds, the backward sweep, the parameter sums.
struct GradRun {
    cryo_plan *p;
    const void *T0;
    int64_t N;
    const double *target;     // device, N values
    double *J, *grad;         // device results
    char *w;
    GradLayout g;
    hipStream_t s;
    std::vector<Launch> L;    // the run's kernel steps
};

static cryo_status grad_check(const cryo_plan *p, int64_t N, const double *target, int64_t ckpt,
                              const void *T0, void *ws, size_t ws_bytes) {
    if (!p || !T0 || N < 1 || !target || ckpt < 0) return fail(CRYO_ERR_ARG, "bad argument");
    if (p->dtype != CRYO_F64) return fail(CRYO_ERR_UNSUPPORTED, "the adjoint needs an FP64 plan");
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

static GradRun grad_run(const cryo_plan *p, const void *T0, int64_t N, int64_t ckpt, void *ws,
                        hipStream_t s) {
    GradRun r;
    r.p = const_cast<cryo_plan *>(p);
    r.T0 = T0;
    r.N = N;
    r.w = (char *)ws;
    r.g = grad_layout(p, N, ckpt);
    r.s = s;
    r.target = nullptr;
    r.J = r.grad = nullptr;
    return r;
}

// forward with checkpoints (head) or kept states (tail) and the surface trace
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
    // state k: in the stored tail, or one of two buffers (the checkpoints
    // are copies)
    auto state = [&](int64_t k) -> void * {
        return g.D > 0 && k >= g.H ? w + g.store + F * (size_t)(k - g.H) : w + g.fwd_buf[k & 1];
    };
    st = launch_to_internal(p, r.T0, state(0), flag, s);
    if (st != CRYO_OK) return st;
    int64_t done = 0;
    const int64_t M = (int64_t)r.L.size();
    for (int64_t l = 0; l < M; ++l) {
        const Launch &ln = r.L[l];
        void *cur = state(l), *nxt = state(l + 1);
        if (l < g.H && l % g.K == 0 &&
            hipMemcpyAsync(w + g.ck + F * (l / g.K), cur, F, hipMemcpyDeviceToDevice, s) !=
                hipSuccess)
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
    // the backward sweep needs the final state only when the tail is stored
    // (the last segment's recompute makes it otherwise)
    return CRYO_OK;
}

// J and the seeds dJ/dS_n, from the trace on the device
static cryo_status grad_objective(GradRun &r) {
    hipLaunchKernelGGL(k_objective, dim3(1), dim3(OBJ_THREADS), 0, r.s,
                       (const double *)(r.w + r.g.surf), r.target, r.N,
                       (double *)(r.w + r.g.seed), r.J);
    return launched("objective");
}

// the adjoint steps backwards: the stored tail first, then each head
// segment (recompute from its checkpoint, adjoint steps)
static cryo_status grad_backward(GradRun &r) {
    cryo_plan *p = r.p;
    const GradLayout &g = r.g;
    char *w = r.w;
    hipStream_t s = r.s;
    int *flag = (int *)(w + g.flag);
    const size_t F = field_f64(p);
    auto ckp = [&](int64_t i) { return (double *)(w + g.ck + F * i); };
    auto segp = [&](int64_t i) { return (double *)(w + g.seg + F * i); };
    const double *seed = (const double *)(w + g.seed);
    const int ngrp = adj_slots(p);
    double *acc = (double *)(w + g.acc), *accg = (double *)(w + g.accg);
    cryo_status st = launch_zero(acc, 3 * (size_t)p->np * ngrp, s);
    if (st == CRYO_OK) st = launch_zero(accg, 2 * (size_t)ngrp, s);
    double *lam[2] = {(double *)(w + g.lam[0]), (double *)(w + g.lam[1])};
    if (st == CRYO_OK) st = launch_adj_init(p, lam[0], seed + r.N, s);
    if (st != CRYO_OK) return st;
    int cur = 0;
    const int64_t M = (int64_t)r.L.size();
    // the plan whose tables step launch k (the turn-on sub-steps: dt / 100)
    auto plan_of = [&](int64_t k) { return r.L[k].sub ? p->sub : p; };
    // adjoint steps b-1 down to a, with state k at T(k): pass 1 reads
    // lam^{k+1} (lam[cur]) and writes y^k, pass 2 writes lam^k (lam[cur ^ 1]);
    // pass 2 of step k and pass 1 of step k-1 run as one launch
    auto sweep = [&](int64_t a, int64_t b, auto T) -> cryo_status {
        auto args = [&](int64_t k, int c) {
            AdjArgs d;
            d.T = T(k);
            d.X = T(k + 1);
            d.lam_in = lam[c];
            d.Y = (double *)(w + g.Y[k & 1]);
            d.lpart = (double *)(w + g.lpart[k & 1]);
            d.lam_out = lam[c ^ 1];
            d.acc = acc;
            d.accg = accg;
            d.s = r.L[k].s;
            d.ds = r.L[k].ds;
            // the state before launch k is observed when launch k-1 ends a step
            d.cS = k >= 1 && r.L[k - 1].obs > 0 ? seed + r.L[k - 1].obs : nullptr;
            d.xs = p->eta * p->eta;
            return d;
        };
        // pass 1 (the line solves, with the capacity term) runs on the tables
        // of its own launch; pass 2 (axial faces) needs no capacity law, so
        // the fused launch takes those of its pass 1
        cryo_status e = launch_adj(plan_of(b - 1), 1, args(b - 1, cur), flag, s);
        for (int64_t k = b - 1; k > a && e == CRYO_OK; --k) {
            const AdjArgs d2 = args(k, cur), d1 = args(k - 1, cur ^ 1);
            e = launch_adj(plan_of(k - 1), 21, d2, flag, s, &d1);
            cur ^= 1;
        }
        if (e == CRYO_OK) e = launch_adj(plan_of(a), 2, args(a, cur), flag, s);
        cur ^= 1;
        return e;
    };
    // the stored tail: its states are where the forward left them
    if (g.D > 0) {
        st = sweep(g.H, M, [&](int64_t k) { return (double *)(w + g.store) + (F / 8) * (k - g.H); });
        if (st != CRYO_OK) return st;
    }
    // then the head's segments backwards: recompute states a+1 .. b from the
    // checkpoint of state a, then the adjoint steps
    for (int64_t sg = g.nck - 1; sg >= 0; --sg) {
        const int64_t a = sg * g.K, b = std::min<int64_t>(g.H, a + g.K);
        auto T = [&](int64_t k) { return k == a ? ckp(sg) : segp(k - a - 1); };
        for (int64_t k = a; k < b; ++k) {
            const double X = p->pulse.amplitude * r.L[k].s;
            st = launch_step(plan_of(k), T(k), T(k + 1), X, nullptr, flag, s);
            if (st != CRYO_OK) return st;
        }
        st = sweep(a, b, T);
        if (st != CRYO_OK) return st;
    }
    return CRYO_OK;
}

// row sums over the workgroup slots (fixed order), then the parameters
static cryo_status grad_finish(GradRun &r) {
    cryo_plan *p = r.p;
    const GradLayout &g = r.g;
    double *rs = (double *)(r.w + g.rs);
    const int ngrp = adj_slots(p);
    hipLaunchKernelGGL(k_grad_rows, dim3((3 * p->nr + 255) / 256), dim3(256), 0, r.s,
                       (const double *)(r.w + g.acc), ngrp, p->nr, p->np, p->rpl, rs);
    cryo_status st = launched("gradient row sums");
    if (st != CRYO_OK) return st;
    if (!p->d_grad) return fail(CRYO_ERR_ARG, "the plan has no gradient tables");
    hipLaunchKernelGGL(k_grad_params, dim3(2 + 2 * p->L), dim3(PAR_THREADS), 0, r.s,
                       (const double *)rs, (const double *)(r.w + g.accg), ngrp, p->nr, p->L,
                       (const double *)p->d_grad, r.grad);
    return launched("gradient parameters");
}

static cryo_status grad_enqueue(GradRun &r) {
    cryo_status st = grad_forward(r);
    if (st == CRYO_OK) st = grad_objective(r);
    if (st == CRYO_OK) st = grad_backward(r);
    if (st == CRYO_OK) st = grad_finish(r);
    return st;
}

// a host caller's target goes to the workspace, J and grad come from it
static cryo_status grad_stage_host(GradRun &r, const double *target) {
    double *t = (double *)(r.w + r.g.tgt);
    if (hipMemcpyAsync(t, target, sizeof(double) * r.N, hipMemcpyHostToDevice, r.s) != hipSuccess)
        return fail(CRYO_ERR_DEVICE, "target copy");
    r.target = t;
    r.J = (double *)(r.w + r.g.out);
    r.grad = r.J + 1;
    return CRYO_OK;
}

// wait for a host caller's run; results and the error word to the host
static cryo_status grad_collect(GradRun &r, double *J, double *grad, double *surf_out) {
    const int ng = 2 + 2 * r.p->L;
    std::vector<double> out(1 + ng);
    int hflag = 0;
    if (hipMemcpyAsync(out.data(), r.J, sizeof(double) * out.size(), hipMemcpyDeviceToHost,
                       r.s) != hipSuccess ||
        (surf_out && hipMemcpyAsync(surf_out, r.w + r.g.surf, sizeof(double) * r.N,
                                    hipMemcpyDeviceToHost, r.s) != hipSuccess) ||
        hipMemcpyAsync(&hflag, r.w + r.g.flag, sizeof(int), hipMemcpyDeviceToHost, r.s) !=
            hipSuccess ||
        hipStreamSynchronize(r.s) != hipSuccess)
        return fail(CRYO_ERR_DEVICE, "gradient results copy");
    if (hflag) return fail(CRYO_ERR_NONFINITE, "non-finite or out-of-range temperature produced");
    *J = out[0];
    memcpy(grad, out.data() + 1, sizeof(double) * ng);
    return CRYO_OK;
}

// streams of cryo_gradient_many: made once per device, kept until the
// process ends (default priority, not synchronising with the null stream)
static std::mutex g_pool_mu;
static std::vector<hipStream_t> g_pool[64];

static cryo_status pool_streams(int n, std::vector<hipStream_t> &out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(CRYO_ERR_DEVICE, "current device");
    std::lock_guard<std::mutex> lk(g_pool_mu);
    std::vector<hipStream_t> &v = g_pool[dev];
    while ((int)v.size() < n) {
        hipStream_t x = nullptr;
        if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess)
            return fail(CRYO_ERR_DEVICE, "stream creation");
        v.push_back(x);
    }
    out.assign(v.begin(), v.begin() + n);
    return CRYO_OK;
}

// Designs side by side: as many as it takes for their launches to cover the
// compute units (a launch of the gradient's kernels has adj_grid workgroups
// of 8 waves, which at the adjoint's register use fill one unit each), at
// most 4 (the hardware queues a process gets by default: streams beyond
// them share queues and run one after another).
static int auto_streams(int n, cryo_plan *const *plans) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int grid = 1;
    for (int i = 0; i < n; ++i) grid = std::max(grid, adj_grid(plans[i]));
    return std::max(1, std::min(4, (cus + grid - 1) / grid));
}

}  // namespace cryo

using namespace cryo;

extern "C" {

cryo_status cryo_plan_set_gradient_store(cryo_plan *p, int64_t steps) {
    if (!p || steps < 0) return fail(CRYO_ERR_ARG, "bad argument");
    p->grad_store = steps;
    return CRYO_OK;
}

cryo_status cryo_gradient_store_steps(const cryo_plan *p, int64_t nsteps, int64_t ckpt,
                                     size_t budget_bytes, int64_t *steps) {
    if (!p || !steps || nsteps < 1 || ckpt < 0) return fail(CRYO_ERR_ARG, "bad argument");
    *steps = store_for_budget(p, nsteps, ckpt, budget_bytes);
    return CRYO_OK;
}

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
    GradRun r = grad_run(pc, T0, N, ckpt, ws, (hipStream_t)stream);
    st = grad_stage_host(r, target);
    if (st == CRYO_OK) st = grad_enqueue(r);
    if (st == CRYO_OK) st = grad_collect(r, J, grad, surf_out);
    return st;
}

cryo_status cryo_gradient_async(const cryo_plan *pc, const void *T0, int64_t N,
                                const double *target, int64_t ckpt, void *ws, size_t ws_bytes,
                                double *J, double *grad, double *surf_out, void *stream) {
    if (!J || !grad) return fail(CRYO_ERR_ARG, "bad argument");
    cryo_status st = grad_check(pc, N, target, ckpt, T0, ws, ws_bytes);
    if (st != CRYO_OK) return st;
    GradRun r = grad_run(pc, T0, N, ckpt, ws, (hipStream_t)stream);
    r.target = target;
    r.J = J;
    r.grad = grad;
    st = grad_enqueue(r);
    if (st == CRYO_OK && surf_out &&
        hipMemcpyAsync(surf_out, r.w + r.g.surf, sizeof(double) * N, hipMemcpyDeviceToDevice,
                       r.s) != hipSuccess)
        st = fail(CRYO_ERR_DEVICE, "surface trace copy");
    return st;
}

cryo_status cryo_gradient_many(int32_t n, cryo_plan *const *plans, const void *const *T0,
                               int64_t N, const double *const *targets, int64_t ckpt,
                               void *const *ws, const size_t *ws_bytes, int32_t n_streams,
                               double *J, double *const *grad, double *const *surf_out) {
    if (n < 1 || !plans || !T0 || !targets || !ws || !ws_bytes || !J || !grad || n_streams < 0)
        return fail(CRYO_ERR_ARG, "bad argument");
    for (int i = 0; i < n; ++i) {
        cryo_status st = grad_check(plans[i], N, targets[i], ckpt, T0[i], ws[i], ws_bytes[i]);
        if (st != CRYO_OK) return fail(st, "design " + std::to_string(i) + ": " + cryo_last_error());
        if (!grad[i]) return fail(CRYO_ERR_ARG, "design " + std::to_string(i) + ": null grad");
    }
    // designs that share a workspace run one after another on one stream:
    // workspace groups in order of first use, group q on stream q mod ns
    std::vector<int> grp(n);
    std::vector<void *> wsg;
    for (int i = 0; i < n; ++i) {
        int q = 0;
        while (q < (int)wsg.size() && wsg[q] != ws[i]) ++q;
        if (q == (int)wsg.size()) wsg.push_back(ws[i]);
        grp[i] = q;
    }
    if (n_streams == 0) n_streams = auto_streams(n, plans);
    std::vector<hipStream_t> streams;
    cryo_status st = pool_streams(std::min<int>(n_streams, (int)wsg.size()), streams);
    if (st != CRYO_OK) return st;
    const int ns = (int)streams.size();
    int dev = 0;
    (void)hipGetDevice(&dev);
    // device tables first, here: the enqueuing threads then only read plans
    // (a plan may serve several designs)
    for (int i = 0; i < n && st == CRYO_OK; ++i) {
        st = ensure_device(plans[i]);
        if (st == CRYO_OK && plans[i]->sub) st = ensure_device(plans[i]->sub);
    }
    if (st != CRYO_OK) return st;
    // Per design, outside the (possibly shared) workspaces: its target, then
    // J, grad, the surface trace and the error word, which each design's
    // work on its stream copies there before the next design may reuse its
    // workspace.  One device block (allocated here, freed on return), filled
    // from the host at once and read back at once.
    std::vector<size_t> ro(n + 1, 0);
    for (int i = 0; i < n; ++i) ro[i + 1] = ro[i] + (size_t)(2 * N + 4 + 2 * plans[i]->L);
    std::vector<double> hres(ro[n], 0.0);
    for (int i = 0; i < n; ++i) memcpy(hres.data() + ro[i], targets[i], sizeof(double) * N);
    double *dres = nullptr;
    if (hipMalloc((void **)&dres, sizeof(double) * ro[n]) != hipSuccess)
        return fail(CRYO_ERR_DEVICE, "gradient results block");
    struct Free {
        double *p;
        ~Free() { (void)hipFree(p); }
    } free_res{dres};
    if (hipMemcpy(dres, hres.data(), sizeof(double) * ro[n], hipMemcpyHostToDevice) != hipSuccess)
        return fail(CRYO_ERR_DEVICE, "target copy");
    auto rJ = [&](int i) { return dres + ro[i] + N; };
    auto rS = [&](int i) { return dres + ro[i] + N + 1 + 2 + 2 * plans[i]->L; };
    auto rF = [&](int i) { return rS(i) + N; };
    std::vector<GradRun> runs;
    runs.reserve(n);
    for (int i = 0; i < n; ++i) {
        runs.push_back(grad_run(plans[i], T0[i], N, ckpt, ws[i], streams[grp[i] % ns]));
        runs[i].target = dres + ro[i];
        runs[i].J = rJ(i);
        runs[i].grad = rJ(i) + 1;
    }
    // each stream's designs enqueued in order by a host thread of its own
    // (a single thread would wait on one stream's full queue while the
    // others ran dry), then the results
    std::vector<cryo_status> tst(ns, CRYO_OK);
    std::vector<int> tbad(ns, -1);
    std::vector<std::string> terr(ns);
    auto work = [&](int k) {
        if (hipSetDevice(dev) != hipSuccess) {
            tst[k] = CRYO_ERR_DEVICE;
            tbad[k] = k;
            terr[k] = "device selection in an enqueuing thread";
            return;
        }
        for (int i = 0; i < n; ++i) {
            if (grp[i] % ns != k) continue;
            GradRun &r = runs[i];
            cryo_status e = grad_enqueue(r);
            // the trace and the error word leave the workspace with the design
            if (e == CRYO_OK &&
                (hipMemcpyAsync(rS(i), r.w + r.g.surf, sizeof(double) * N,
                                hipMemcpyDeviceToDevice, r.s) != hipSuccess ||
                 hipMemcpyAsync(rF(i), r.w + r.g.flag, sizeof(int), hipMemcpyDeviceToDevice,
                                r.s) != hipSuccess))
                e = fail(CRYO_ERR_DEVICE, "gradient results copy");
            if (e != CRYO_OK) {
                tst[k] = e;
                tbad[k] = i;
                terr[k] = cryo_last_error();
                return;
            }
        }
    };
    std::vector<std::thread> pool;
    std::vector<int> inline_work;
    for (int k = 1; k < ns; ++k) {
        try {
            pool.emplace_back(work, k);
        } catch (...) {            // no thread: this thread enqueues those designs too
            inline_work.push_back(k);
        }
    }
    work(0);
    for (int k : inline_work) work(k);
    for (std::thread &x : pool) x.join();
    for (hipStream_t x : streams) (void)hipStreamSynchronize(x);
    int first = -1;
    for (int k = 0; k < ns; ++k)
        if (tst[k] != CRYO_OK && (first < 0 || tbad[k] < tbad[first])) first = k;
    if (first >= 0)
        return fail(tst[first], "design " + std::to_string(tbad[first]) + ": " + terr[first]);
    if (hipMemcpy(hres.data(), dres, sizeof(double) * ro[n], hipMemcpyDeviceToHost) != hipSuccess)
        return fail(CRYO_ERR_DEVICE, "gradient results copy");
    for (int i = 0; i < n; ++i) {
        int flag = 0;
        memcpy(&flag, hres.data() + (rF(i) - dres), sizeof(int));
        if (flag)
            return fail(CRYO_ERR_NONFINITE, "design " + std::to_string(i) +
                                                ": non-finite or out-of-range temperature produced");
        J[i] = hres[ro[i] + N];
        memcpy(grad[i], hres.data() + ro[i] + N + 1, sizeof(double) * (2 + 2 * plans[i]->L));
        if (surf_out && surf_out[i])
            memcpy(surf_out[i], hres.data() + (rS(i) - dres), sizeof(double) * N);
    }
    return CRYO_OK;
}

}  // extern "C"
