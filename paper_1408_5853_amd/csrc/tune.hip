// Autotuners: cryo_autotune times every built kernel shape (rows per lane,
// waves per line) and lines-per-wave on one problem and returns the fastest;
// cryo_batch_autotune does the same per shape group of a batch, timing
// batches of the group's instances, then refines each group's lines per
// wave on the whole batch.  The tuners own their trial fields and
// workspaces (device allocations of their own, outside any stepping call).
// An optional text cache records results across runs: keyed by dtype,
// radial and axial node counts, layer count and law family (cube or general
// capacity exponents) for one problem, and by dtype, default shape, law
// family, domain and largest radial size for a batch group, and by a hash of
// the whole batch for the refinement.  Batch instances may carry plan
// options (polynomial laws, stepped domain); they are grouped and timed as
// cryo_batch_create_with groups and steps them.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

using namespace cryo;

namespace {

// every capacity exponent 3 selects the kernels' cube path
bool all_cube(const cryo_problem *p) {
    for (int m = 0; m < p->geom.n_layers; ++m)
        if (p->geom.layers[m].mat.q != 3.0) return false;
    return true;
}

// an instance's options: polynomial laws, stepped domain
bool opt_poly(const cryo_instance_options *o, int i) { return o && o[i].poly_a; }
bool opt_stepped(const cryo_instance_options *o, int i) {
    return o && (o[i].z_full != 0 || o[i].nr_top != 0);
}

std::string cache_key(const cryo_problem *p, cryo_dtype dt) {
    char b[160];
    snprintf(b, sizeof b, "%s %d %d %d %s", dt == CRYO_F64 ? "f64" : "f32", p->geom.nr,
             p->geom.nz, p->geom.n_layers, all_cube(p) ? "cube" : "power");
    return b;
}

bool cache_lookup(const char *path, const std::string &key, int32_t *shape) {
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char k[128];
        int a, b, c, n;
        if (sscanf(line, "%127[^|]| %d %d %d%n", k, &a, &b, &c, &n) == 4) {
            std::string ks(k);
            while (!ks.empty() && ks.back() == ' ') ks.pop_back();
            if (ks == key) {
                shape[0] = a;
                shape[1] = b;
                shape[2] = c;
                found = true;
            }
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const int32_t *shape, double us) {
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s | %d %d %d | %.3f us/step\n", key.c_str(), shape[0], shape[1], shape[2], us);
    fclose(f);
}

// An instance group of a batch (instances with one default shape, law
// family and domain), as cryo_batch_create_with forms them.
struct Group {
    int rpl, wpl;
    bool cube, poly, stepped;
    int nr_max = 0, nz_min = 1 << 30;
    std::vector<int> inst;
};

// Time per step of the whole batch with the given shapes (the best of three
// timed runs of `run_steps` after the capture block).
cryo_status time_batch(int32_t n, const cryo_problem *probs, const cryo_instance_options *opts,
                       cryo_dtype dtype, const std::vector<int32_t> &shp, int run_steps,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1, double *us) {
    cryo_batch *b = nullptr;
    cryo_status st = cryo_batch_create_with(n, probs, dtype, shp.data(), opts, &b);
    if (st != CRYO_OK) return st;
    std::vector<int64_t> off((size_t)n + 1);
    cryo_batch_offsets(b, off.data());
    size_t wsb = 0;
    cryo_batch_workspace_bytes(b, &wsb);
    void *T = nullptr, *ws = nullptr;
    if (hipMalloc(&T, (size_t)off.back() * (dtype == CRYO_F64 ? 8 : 4)) != hipSuccess ||
        hipMalloc(&ws, wsb) != hipSuccess) {
        if (T) (void)hipFree(T);
        cryo_batch_destroy(b);
        return fail(CRYO_ERR_DEVICE, "batch tuner buffers");
    }
    st = cryo_batch_init(b, T, s);
    if (st == CRYO_OK) st = cryo_batch_forward(b, T, 0, 32, ws, wsb, s);
    double best = 1e300;
    for (int rep = 0; rep < 3 && st == CRYO_OK; ++rep) {
        (void)hipEventRecord(e0, s);
        st = cryo_batch_forward(b, T, 32 + (int64_t)rep * run_steps, run_steps, ws, wsb, s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        best = std::min(best, 1e3 * ms / run_steps);
    }
    if (st == CRYO_OK) st = cryo_batch_poll(b, ws, s, nullptr);
    (void)hipFree(ws);
    (void)hipFree(T);
    cryo_batch_destroy(b);
    *us = best;
    return st;
}

// FNV-1a over what decides a batch's grouping and work: per instance its
// grid, layer count, law family and domain.
uint64_t batch_hash(int32_t n, const cryo_problem *probs, const cryo_instance_options *opts,
                    cryo_dtype dtype) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)dtype);
    mix((uint64_t)n);
    for (int i = 0; i < n; ++i) {
        mix((uint64_t)probs[i].geom.nr);
        mix((uint64_t)probs[i].geom.nz);
        mix((uint64_t)probs[i].geom.n_layers);
        mix(all_cube(&probs[i]) ? 1 : 0);
        // options change the hash only where they are set, so a batch
        // without any keeps its key
        if (opt_poly(opts, i)) mix(0x706f6c79);
        if (opt_stepped(opts, i)) {
            mix(0x73746570);
            mix((uint64_t)opts[i].z_full);
            mix((uint64_t)opts[i].nr_top);
        }
    }
    return h;
}

// Second pass on the whole batch.  The groups' launches share the chip (one
// graph branch per group), so the lines per wave that suit a group alone
// need not suit it beside the others: each group in turn, most nodes first,
// tries lines per wave 1, 2 and 4 with every other group as picked, and
// keeps a value that makes the whole batch at least 1 % faster; a second
// sweep over the groups follows when the first changed any (the groups'
// best values depend on each other).  Cached per batch (a hash of the
// instances' grids, layer counts and law families).
cryo_status refine_lines_per_wave(int32_t n, const cryo_problem *probs,
                                  const cryo_instance_options *opts, cryo_dtype dtype,
                                  int run_steps, const char *cache_path, hipStream_t s,
                                  hipEvent_t e0, hipEvent_t e1,
                                  const std::vector<Group> &groups, int32_t *shapes) {
    char hb[64];
    snprintf(hb, sizeof hb, "batchset %016llx",
             (unsigned long long)batch_hash(n, probs, opts, dtype));
    auto gkey = [&](size_t gi) { return std::string(hb) + " g" + std::to_string(gi); };
    auto apply = [&](const Group &g, int lpw, std::vector<int32_t> &shp) {
        for (int i : g.inst) shp[3 * i + 2] = std::max(1, std::min(lpw, probs[i].geom.nz - 2));
    };
    std::vector<int32_t> shp(shapes, shapes + 3 * (size_t)n);
    bool cached = cache_path != nullptr;
    std::vector<int> lp(groups.size());
    for (size_t gi = 0; gi < groups.size() && cached; ++gi) {
        int32_t c[3];
        if (!cache_lookup(cache_path, gkey(gi), c) || c[0] != groups[gi].rpl) cached = false;
        else lp[gi] = c[2];
    }
    if (cached) {
        for (size_t gi = 0; gi < groups.size(); ++gi) apply(groups[gi], lp[gi], shp);
        std::copy(shp.begin(), shp.end(), shapes);
        return CRYO_OK;
    }
    std::vector<size_t> order(groups.size());
    std::vector<double> work(groups.size(), 0.0);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        order[gi] = gi;
        for (int i : groups[gi].inst) work[gi] += (double)probs[i].geom.nr * probs[i].geom.nz;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return work[a] > work[b]; });
    double best = 0.0;
    cryo_status st = time_batch(n, probs, opts, dtype, shp, run_steps, s, e0, e1, &best);
    if (st != CRYO_OK) return st;
    for (int sweep = 0; sweep < 2; ++sweep) {
        bool changed = false;
        for (size_t gi : order) {
            const Group &g = groups[gi];
            const int cur = shp[3 * g.inst[0] + 2];
            int keep = cur;
            for (int lpw : {1, 2, 4}) {
                if (lpw == cur) continue;
                std::vector<int32_t> trial(shp);
                apply(g, lpw, trial);
                if (trial == shp) continue;
                double t = 0.0;
                st = time_batch(n, probs, opts, dtype, trial, run_steps, s, e0, e1, &t);
                if (st != CRYO_OK) return st;
                if (t < 0.99 * best) {
                    best = t;
                    keep = lpw;
                }
            }
            if (keep != cur) changed = true;
            apply(g, keep, shp);
        }
        if (!changed) break;
    }
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        int32_t c[3] = {shp[3 * groups[gi].inst[0]], shp[3 * groups[gi].inst[0] + 1], 0};
        // the group's value before the cap at nz - 2
        c[2] = 0;
        for (int i : groups[gi].inst) c[2] = std::max<int32_t>(c[2], shp[3 * i + 2]);
        cache_store(cache_path, gkey(gi), c, best);
    }
    std::copy(shp.begin(), shp.end(), shapes);
    return CRYO_OK;
}

}  // namespace

extern "C" {

cryo_status cryo_autotune(const cryo_problem *prob, cryo_dtype dtype, int32_t steps,
                          const char *cache_path, void *stream, int32_t *shape,
                          double *us_per_step) {
    if (!prob || !shape || steps < 1) return fail(CRYO_ERR_ARG, "bad argument");
    const std::string key = cache_key(prob, dtype);
    if (cache_lookup(cache_path, key, shape)) {
        if (us_per_step) *us_per_step = -1.0;
        return CRYO_OK;
    }
    hipStream_t s = (hipStream_t)stream;
#define TUNE_SHAPE(RP, GW) {RP, GW},
    const int shapes[][2] = {CRYO_FOR_SHAPES(TUNE_SHAPE)};
#undef TUNE_SHAPE
    const int lpws[] = {1, 2, 4, 8};
    double best = 1e300;
    int32_t bs[3] = {0, 0, 0};
    size_t es = dtype == CRYO_F64 ? 8 : 4;
    size_t fbytes = es * (size_t)prob->geom.nr * prob->geom.nz * (dtype == CRYO_F32 ? 2 : 1);
    void *T = nullptr;
    if (hipMalloc(&T, fbytes) != hipSuccess) return fail(CRYO_ERR_DEVICE, "tuner field");
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    cryo_status result = CRYO_OK;
    for (const auto &sh : shapes) {
        if (64 * sh[0] * sh[1] < prob->geom.nr) continue;
        if (64 * sh[0] * sh[1] >= 4 * prob->geom.nr && sh[0] * sh[1] > 2) continue;   // mostly padding
        for (int lpw : lpws) {
            if (lpw > prob->geom.nz - 2) continue;
            cryo_plan *p = nullptr;
            if (cryo_plan_create(prob, dtype, &p) != CRYO_OK) {
                result = CRYO_ERR_ARG;
                break;
            }
            if (cryo_plan_set_shape(p, sh[0], sh[1], lpw) != CRYO_OK) {
                cryo_plan_destroy(p);
                continue;
            }
            size_t wsb = 0;
            cryo_workspace_bytes(p, steps, &wsb);
            void *ws = nullptr;
            if (hipMalloc(&ws, wsb) != hipSuccess) {
                cryo_plan_destroy(p);
                result = fail(CRYO_ERR_DEVICE, "tuner workspace");
                break;
            }
            cryo_status st = cryo_init(p, T, s);
            if (st == CRYO_OK) st = cryo_forward(p, T, 0, 4, ws, wsb, nullptr, s);
            (void)hipEventRecord(e0, s);
            if (st == CRYO_OK) st = cryo_forward(p, T, 4, steps, ws, wsb, nullptr, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (st == CRYO_OK && cryo_poll(p, ws, s) == CRYO_OK) {
                const double us = 1e3 * ms / steps;
                if (us < best) {
                    best = us;
                    bs[0] = sh[0];
                    bs[1] = sh[1];
                    bs[2] = lpw;
                }
            }
            (void)hipFree(ws);
            cryo_plan_destroy(p);
        }
        if (result != CRYO_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(T);
    if (result != CRYO_OK) return result;
    if (bs[0] == 0) return fail(CRYO_ERR_UNSUPPORTED, "no kernel shape ran");
    memcpy(shape, bs, sizeof bs);
    if (us_per_step) *us_per_step = best;
    cache_store(cache_path, key, bs, best);
    return CRYO_OK;
}

cryo_status cryo_batch_autotune_with(int32_t n, const cryo_problem *probs, cryo_dtype dtype,
                                     const cryo_instance_options *opts, int32_t steps,
                                     const char *cache_path, void *stream, int32_t *shapes) {
    if (n < 1 || !probs || !shapes || steps < 1) return fail(CRYO_ERR_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    // the turn-on model's rare sub-steps run on the instance's own shape and
    // are not timed: trial batches step without it
    std::vector<cryo_instance_options> plain;
    if (opts) {
        plain.assign(opts, opts + n);
        for (cryo_instance_options &o : plain) o.turn_on = 0;
        opts = plain.data();
    }
    // the groups cryo_batch_create forms with default shapes
    std::vector<Group> groups;
    for (int i = 0; i < n; ++i) {
        cryo_plan *p = nullptr;
        cryo_status st = cryo_plan_create(&probs[i], dtype, &p);
        if (st != CRYO_OK)
            return fail(st, "instance " + std::to_string(i) + ": " + cryo_last_error());
        int rpl = 0, wpl = 0, lpw = 0;
        cryo_plan_shape(p, &rpl, &wpl, &lpw);
        cryo_plan_destroy(p);
        // the grouping of cryo_batch_create_with: shape, law family, domain
        const bool poly = opt_poly(opts, i), stepped = opt_stepped(opts, i);
        const bool cube = !poly && all_cube(&probs[i]);
        Group *g = nullptr;
        for (Group &q : groups)
            if (q.rpl == rpl && q.wpl == wpl && q.cube == cube && q.poly == poly &&
                q.stepped == stepped)
                g = &q;
        if (!g) {
            groups.push_back(Group());
            g = &groups.back();
            g->rpl = rpl;
            g->wpl = wpl;
            g->cube = cube;
            g->poly = poly;
            g->stepped = stepped;
        }
        g->inst.push_back(i);
        g->nr_max = std::max(g->nr_max, probs[i].geom.nr);
        g->nz_min = std::min(g->nz_min, probs[i].geom.nz);
    }
#define TUNE_SHAPE(RP, GW) {RP, GW},
    const int built[][2] = {CRYO_FOR_SHAPES(TUNE_SHAPE)};
#undef TUNE_SHAPE
    const int lpws[] = {1, 2, 4, 8};
    const int run_steps = ((steps + 31) / 32) * 32;         // whole captured blocks
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    cryo_status result = CRYO_OK;
    for (const Group &g : groups) {
        char kb[160];
        // (rectangular power-law groups keep the key they had before the
        // options existed)
        snprintf(kb, sizeof kb, "batch %s %d %d %s%s %d", dtype == CRYO_F64 ? "f64" : "f32", g.rpl,
                 g.wpl, g.poly ? "poly" : g.cube ? "cube" : "power",
                 g.stepped ? " stepped" : "", g.nr_max);
        int32_t best_shape[3] = {g.rpl, g.wpl, 4};
        if (!cache_lookup(cache_path, kb, best_shape)) {
            // up to 8 of the group's instances, spread over its sizes
            std::vector<int> order(g.inst);
            std::sort(order.begin(), order.end(), [&](int a, int b) {
                return (int64_t)probs[a].geom.nr * probs[a].geom.nz <
                       (int64_t)probs[b].geom.nr * probs[b].geom.nz;
            });
            std::vector<int> sub;
            const int k = std::min<int>(8, (int)order.size());
            for (int q = 0; q < k; ++q) sub.push_back(order[(size_t)q * order.size() / k]);
            std::vector<cryo_problem> sp;
            std::vector<cryo_instance_options> so;
            double nodes = 0;
            for (int i : sub) {
                sp.push_back(probs[i]);
                if (opts) so.push_back(opts[i]);
                nodes += (double)probs[i].geom.nr * probs[i].geom.nz;
            }
            double best = 1e300;
            for (const auto &sh : built) {
                const int rows = 64 * sh[0] * sh[1];
                if (rows < g.nr_max || (rows >= 2 * g.nr_max && sh[0] * sh[1] > 2)) continue;
                for (int lpw : lpws) {
                    std::vector<int32_t> shp;
                    for (int i : sub) {
                        shp.push_back(sh[0]);
                        shp.push_back(sh[1]);
                        shp.push_back(std::min(lpw, probs[i].geom.nz - 2));
                    }
                    cryo_batch *b = nullptr;
                    if (cryo_batch_create_with((int32_t)sub.size(), sp.data(), dtype, shp.data(),
                                               opts ? so.data() : nullptr, &b) != CRYO_OK)
                        continue;
                    int64_t nel = 0;
                    std::vector<int64_t> off(sub.size() + 1);
                    cryo_batch_offsets(b, off.data());
                    nel = off.back();
                    size_t wsb = 0;
                    cryo_batch_workspace_bytes(b, &wsb);
                    void *T = nullptr, *ws = nullptr;
                    if (hipMalloc(&T, nel * (dtype == CRYO_F64 ? 8 : 4)) != hipSuccess ||
                        hipMalloc(&ws, wsb) != hipSuccess) {
                        if (T) (void)hipFree(T);
                        cryo_batch_destroy(b);
                        result = fail(CRYO_ERR_DEVICE, "batch tuner buffers");
                        break;
                    }
                    cryo_status st = cryo_batch_init(b, T, s);
                    // the first block captures the graph; the timed run replays it
                    if (st == CRYO_OK) st = cryo_batch_forward(b, T, 0, 32, ws, wsb, s);
                    (void)hipEventRecord(e0, s);
                    if (st == CRYO_OK) st = cryo_batch_forward(b, T, 32, run_steps, ws, wsb, s);
                    (void)hipEventRecord(e1, s);
                    (void)hipEventSynchronize(e1);
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (st == CRYO_OK && cryo_batch_poll(b, ws, s, nullptr) == CRYO_OK) {
                        const double t = 1e-3 * ms / (nodes * run_steps);
                        if (t < best) {
                            best = t;
                            best_shape[0] = sh[0];
                            best_shape[1] = sh[1];
                            best_shape[2] = lpw;
                        }
                    }
                    (void)hipFree(ws);
                    (void)hipFree(T);
                    cryo_batch_destroy(b);
                }
                if (result != CRYO_OK) break;
            }
            if (result != CRYO_OK) break;
            if (best == 1e300) {
                result = fail(CRYO_ERR_UNSUPPORTED, "no kernel shape ran for a batch group");
                break;
            }
            cache_store(cache_path, kb, best_shape, 1e6 * best * nodes);
        }
        for (int i : g.inst) {
            shapes[3 * i] = best_shape[0];
            shapes[3 * i + 1] = best_shape[1];
            shapes[3 * i + 2] = std::max(1, std::min(best_shape[2], probs[i].geom.nz - 2));
        }
    }
    if (result == CRYO_OK && groups.size() > 1)
        result = refine_lines_per_wave(n, probs, opts, dtype, run_steps, cache_path, s, e0, e1,
                                       groups, shapes);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return result;
}

cryo_status cryo_batch_autotune(int32_t n, const cryo_problem *probs, cryo_dtype dtype,
                                int32_t steps, const char *cache_path, void *stream,
                                int32_t *shapes) {
    return cryo_batch_autotune_with(n, probs, dtype, nullptr, steps, cache_path, stream, shapes);
}

}  // extern "C"
