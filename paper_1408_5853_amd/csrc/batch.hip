// Batched stepping of many independent cells (design sweeps): instances
// are grouped by kernel shape; each step is one launch per shape group over
// all of its instances, and blocks of steps are captured once in a HIP graph
// (one branch per shape group) and replayed.  The global step index lives
// in device memory so a captured block can be replayed for any step range.
// Steps where an instance with the turn-on model starts a pulse run eagerly,
// instance by instance.
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

namespace cryo {

constexpr int GRAPH_STEPS = 32;      // steps per captured graph block (even)

struct Bucket {
    int rpl, wpl;
    bool cube;                       // every capacity exponent is 3
    bool poly;                       // polynomial laws (eqs. (23)-(25))
    bool stepped;                    // stepped domain (eq. (9))
    std::vector<int> inst;           // instance indices
    std::vector<int2> map;           // workgroup -> (instance, workgroup of instance)
    size_t desc_off = 0, map_off = 0;  // byte offsets in the device block
};

}  // namespace cryo

struct cryo_batch {
    std::vector<cryo_plan *> plans;
    cryo_dtype dtype;
    std::vector<int64_t> off;        // element offsets of the instances' fields
    std::vector<cryo::Bucket> buckets;
    void *d_block = nullptr;         // descriptors and workgroup maps
    size_t block_bytes = 0;
    std::vector<unsigned char> h_block;
    // workspace layout
    std::vector<size_t> ws_field;    // per instance: offset of its two internal buffers
    size_t ws_bytes = 0;
    // graph cache (tied to one workspace)
    void *graph_ws = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

namespace cryo {

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t field_bytes_internal(const cryo_plan *p) { return align256(8 * (size_t)p->nz * p->np); }

static int64_t abi_elems(const cryo_plan *p) {
    return (int64_t)p->nz * p->nr * (p->dtype == CRYO_F32 ? 2 : 1);
}

// descriptor builders live with the kernels (forward.hip)
size_t step_desc_bytes(cryo_dtype dt);
void step_desc_fill(const cryo_plan *p, void *out, void *buf0, void *buf1, int *flag);
cryo_status launch_step_batch(cryo_dtype dt, int rpl, int wpl, bool cube, bool poly,
                              bool stepped, const void *desc, const int2 *map, int nwg,
                              size_t lds, int64_t n, const int64_t *k0, hipStream_t s);
cryo_status launch_set_i64(int64_t *ptr, int64_t v, hipStream_t s);
cryo_status launch_add_i64(int64_t *ptr, int64_t v, hipStream_t s);

static void batch_free_graph(cryo_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_ws = nullptr;
}

// Lay out the workspace: flags (one int per instance), the step counter,
// then each instance's two internal field buffers.
static void batch_layout(cryo_batch *b) {
    size_t o = align256(sizeof(int) * b->plans.size()) + 256;
    b->ws_field.resize(b->plans.size());
    for (size_t i = 0; i < b->plans.size(); ++i) {
        b->ws_field[i] = o;
        o += 2 * field_bytes_internal(b->plans[i]);
    }
    b->ws_bytes = o;
}

static size_t counter_off(const cryo_batch *b) { return align256(sizeof(int) * b->plans.size()); }

static cryo_status batch_build_buckets(cryo_batch *b) {
    b->buckets.clear();
    std::map<int, int> idx;
    for (size_t i = 0; i < b->plans.size(); ++i) {
        const cryo_plan *p = b->plans[i];
        // shape, law family (cube, power, polynomial) and domain
        const bool cube = !p->poly && p->flaws.cube != 0;
        int key = p->rpl * 10 + p->wpl + (cube ? 1000 : 0) + (p->poly ? 2000 : 0) +
                  (p->stepped ? 4000 : 0);
        if (!idx.count(key)) {
            idx[key] = (int)b->buckets.size();
            Bucket bk;
            bk.rpl = p->rpl;
            bk.wpl = p->wpl;
            bk.cube = cube;
            bk.poly = p->poly;
            bk.stepped = p->stepped;
            b->buckets.push_back(bk);
        }
        Bucket &bk = b->buckets[idx[key]];
        const int g = step_grid(p);
        for (int w = 0; w < g; ++w) bk.map.push_back(make_int2((int)bk.inst.size(), w));
        bk.inst.push_back((int)i);
    }
    // heaviest groups first: their branches are captured (and start) first,
    // so the longest chains are not queued behind the short ones
    auto work = [&](const Bucket &bk) {
        double w = 0;
        for (int i : bk.inst) w += (double)b->plans[i]->nr * b->plans[i]->nz;
        return w;
    };
    std::stable_sort(b->buckets.begin(), b->buckets.end(),
                     [&](const Bucket &x, const Bucket &y) { return work(x) > work(y); });
    const size_t ds = step_desc_bytes(b->dtype);
    size_t o = 0;
    for (Bucket &bk : b->buckets) {
        bk.desc_off = o;
        o = align256(o + ds * bk.inst.size());
        bk.map_off = o;
        o = align256(o + sizeof(int2) * bk.map.size());
    }
    b->block_bytes = o;
    b->h_block.assign(o, 0);
    for (Bucket &bk : b->buckets)
        memcpy(b->h_block.data() + bk.map_off, bk.map.data(), sizeof(int2) * bk.map.size());
    return CRYO_OK;
}

}  // namespace cryo

using namespace cryo;

extern "C" {

cryo_status cryo_batch_create(int32_t n, const cryo_problem *probs, cryo_dtype dtype,
                              const int32_t *shapes, cryo_batch **out) {
    return cryo_batch_create_with(n, probs, dtype, shapes, nullptr, out);
}

cryo_status cryo_batch_create_with(int32_t n, const cryo_problem *probs, cryo_dtype dtype,
                                   const int32_t *shapes, const cryo_instance_options *opts,
                                   cryo_batch **out) {
    if (!out || n < 1 || !probs) return fail(CRYO_ERR_ARG, "bad batch arguments");
    *out = nullptr;
    cryo_batch *b = new cryo_batch();
    b->dtype = dtype;
    for (int i = 0; i < n; ++i) {
        cryo_plan *p = nullptr;
        cryo_status st = cryo_plan_create(&probs[i], dtype, &p);
        // the instance's plan options, as cryo_plan_set_poly_laws and
        // cryo_plan_set_stepped set them on a single plan
        if (st == CRYO_OK && opts) {
            const cryo_instance_options &o = opts[i];
            if ((o.poly_a != nullptr) != (o.poly_b != nullptr))
                st = fail(CRYO_ERR_ARG, "polynomial laws need both poly_a and poly_b");
            else if (!o.poly_a && o.joule_tref != 0.0)
                st = fail(CRYO_ERR_ARG, "the Joule source needs the polynomial laws");
            else if (o.poly_a)
                st = cryo_plan_set_poly_laws(p, o.poly_a, o.poly_b, o.joule_tref);
            if (st == CRYO_OK && (o.z_full != 0 || o.nr_top != 0))
                st = cryo_plan_set_stepped(p, o.z_full, o.nr_top);
            // the sub-step tables take the laws and domain set above, and
            // the shape set below
            if (st == CRYO_OK && o.turn_on) st = cryo_plan_set_turn_on(p, 1);
        }
        if (st == CRYO_OK && shapes)
            st = cryo_plan_set_shape(p, shapes[3 * i], shapes[3 * i + 1], shapes[3 * i + 2]);
        else if (st == CRYO_OK)
            // the instances fill the device together: longer line blocks
            // amortise each block's start-up line
            st = cryo_plan_set_shape(p, p->rpl, p->wpl, std::min(BATCH_LPW, p->nz - 2));
        if (st != CRYO_OK) {
            std::string m = "instance " + std::to_string(i) + ": " + cryo_last_error();
            if (p) cryo_plan_destroy(p);
            cryo_batch_destroy(b);
            return fail(st, m);
        }
        b->plans.push_back(p);
    }
    b->off.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) b->off[i + 1] = b->off[i] + abi_elems(b->plans[i]);
    batch_build_buckets(b);
    batch_layout(b);
    *out = b;
    return CRYO_OK;
}

void cryo_batch_destroy(cryo_batch *b) {
    if (!b) return;
    batch_free_graph(b);
    if (b->d_block) (void)hipFree(b->d_block);
    for (cryo_plan *p : b->plans) cryo_plan_destroy(p);
    delete b;
}

cryo_status cryo_batch_offsets(const cryo_batch *b, int64_t *off) {
    if (!b || !off) return fail(CRYO_ERR_ARG, "null argument");
    memcpy(off, b->off.data(), sizeof(int64_t) * b->off.size());
    return CRYO_OK;
}

cryo_status cryo_batch_workspace_bytes(const cryo_batch *b, size_t *bytes) {
    if (!b || !bytes) return fail(CRYO_ERR_ARG, "null argument");
    *bytes = b->ws_bytes;
    return CRYO_OK;
}

cryo_status cryo_batch_init(const cryo_batch *b, void *T, void *stream) {
    if (!b || !T) return fail(CRYO_ERR_ARG, "null argument");
    const size_t es = b->dtype == CRYO_F64 ? 8 : 4;
    for (size_t i = 0; i < b->plans.size(); ++i) {
        cryo_status st = cryo_init(b->plans[i], (char *)T + es * b->off[i], stream);
        if (st != CRYO_OK) return st;
    }
    return CRYO_OK;
}

cryo_status cryo_batch_forward(cryo_batch *b, void *T, int64_t k0, int64_t nsteps, void *ws,
                               size_t ws_bytes, void *stream) {
    if (!b || !T || k0 < 0 || nsteps < 0) return fail(CRYO_ERR_ARG, "bad argument");
    if (!ws || ws_bytes < b->ws_bytes)
        return fail(CRYO_ERR_WORKSPACE, "batch workspace needs " + std::to_string(b->ws_bytes) +
                                            " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(CRYO_ERR_WORKSPACE, "workspace must be 256-aligned");
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    const size_t es = b->dtype == CRYO_F64 ? 8 : 4;
    const int n = (int)b->plans.size();
    for (cryo_plan *p : b->plans) {
        cryo_status st = ensure_device(p);
        if (st == CRYO_OK && p->sub) st = ensure_device(p->sub);
        if (st != CRYO_OK) return st;
    }
    if (!b->d_block) {
        hipError_t e = hipMalloc(&b->d_block, b->block_bytes);
        if (e != hipSuccess) return fail(CRYO_ERR_DEVICE, "batch descriptor block");
    }
    // descriptors point into this workspace: refresh them (and the graph)
    // when the workspace moves
    if (b->graph_ws != ws) {
        batch_free_graph(b);
        const size_t ds = step_desc_bytes(b->dtype);
        for (Bucket &bk : b->buckets)
            for (size_t q = 0; q < bk.inst.size(); ++q) {
                const int i = bk.inst[q];
                char *f = w + b->ws_field[i];
                step_desc_fill(b->plans[i], b->h_block.data() + bk.desc_off + ds * q, f,
                               f + field_bytes_internal(b->plans[i]), (int *)w + i);
            }
        hipError_t e = hipMemcpy(b->d_block, b->h_block.data(), b->block_bytes,
                                 hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(CRYO_ERR_DEVICE, "batch descriptor upload");
    }
    int64_t *k0p = (int64_t *)(w + counter_off(b));
    for (int i = 0; i < n; ++i) {
        cryo_status st = launch_to_internal(b->plans[i], (char *)T + es * b->off[i],
                                            w + b->ws_field[i], (int *)w + i, s);
        if (st != CRYO_OK) return st;
    }
    cryo_status st = CRYO_OK;
    // the steps of one bucket (its instances only) on stream strm: step
    // offsets first .. first + count - 1 from the device step counter
    auto launch_bucket = [&](const Bucket &bk, int64_t first, int64_t count,
                             hipStream_t strm) -> cryo_status {
        size_t lds = 0;
        for (int i : bk.inst) lds = std::max(lds, step_lds(b->plans[i]));
        for (int64_t m = first; m < first + count; ++m) {
            cryo_status r = launch_step_batch(
                b->dtype, bk.rpl, bk.wpl, bk.cube, bk.poly, bk.stepped,
                (const char *)b->d_block + bk.desc_off,
                (const int2 *)((const char *)b->d_block + bk.map_off), (int)bk.map.size(), lds,
                m, k0p, strm);
            if (r != CRYO_OK) return r;
        }
        return CRYO_OK;
    };
    auto ensure_graph = [&]() -> cryo_status {
        if (b->exec) return CRYO_OK;
        // One graph per block of GRAPH_STEPS steps: the buckets hold
        // disjoint instances, so each bucket's chain of steps is a branch
        // of its own (forked from and joined to the capture stream), and
        // the branches may run side by side; the step counter advances
        // after the join.
        const size_t nb = b->buckets.size();
        hipStream_t cs;
        std::vector<hipStream_t> bs(nb, nullptr);
        std::vector<hipEvent_t> ev(nb + 1, nullptr);
        bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
        for (size_t q = 0; ok && q < nb; ++q)
            ok = hipStreamCreateWithFlags(&bs[q], hipStreamNonBlocking) == hipSuccess;
        for (size_t q = 0; ok && q <= nb; ++q)
            ok = hipEventCreateWithFlags(&ev[q], hipEventDisableTiming) == hipSuccess;
        cryo_status r = ok ? CRYO_OK : CRYO_ERR_DEVICE;
        hipGraph_t g = nullptr;
        hipError_t e2 = hipErrorUnknown;
        if (ok) {
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) r = CRYO_ERR_DEVICE;
            if (r == CRYO_OK && hipEventRecord(ev[nb], cs) != hipSuccess) r = CRYO_ERR_DEVICE;
            for (size_t q = 0; r == CRYO_OK && q < nb; ++q) {
                if (hipStreamWaitEvent(bs[q], ev[nb], 0) != hipSuccess) r = CRYO_ERR_DEVICE;
                if (r == CRYO_OK) r = launch_bucket(b->buckets[q], 0, GRAPH_STEPS, bs[q]);
                if (r == CRYO_OK && (hipEventRecord(ev[q], bs[q]) != hipSuccess ||
                                     hipStreamWaitEvent(cs, ev[q], 0) != hipSuccess))
                    r = CRYO_ERR_DEVICE;
            }
            if (r == CRYO_OK) r = launch_add_i64(k0p, GRAPH_STEPS, cs);
            e2 = hipStreamEndCapture(cs, &g);
        }
        for (size_t q = 0; q < nb; ++q)
            if (bs[q]) (void)hipStreamDestroy(bs[q]);
        for (size_t q = 0; q <= nb; ++q)
            if (ev[q]) (void)hipEventDestroy(ev[q]);
        if (ok) (void)hipStreamDestroy(cs);
        if (r != CRYO_OK || e2 != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return fail(CRYO_ERR_DEVICE, "graph capture of the step block failed");
        }
        if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(CRYO_ERR_DEVICE, "graph instantiation failed");
        }
        b->graph = g;
        b->graph_ws = ws;
        return CRYO_OK;
    };
    // The fields of all instances sit in buffer `par` before global step k.
    int64_t k = k0;
    int par = 0;
    // regular steps k .. k + count - 1 of every instance: captured blocks of
    // GRAPH_STEPS steps (they start from buffer 0) and single launches
    auto regular = [&](int64_t count) -> cryo_status {
        cryo_status r = CRYO_OK;
        if (count > 0 && par == 1) {
            // one step from buffer 1: step offset 1 from counter k - 1
            r = launch_set_i64(k0p, k - 1, s);
            for (const Bucket &bk : b->buckets)
                if (r == CRYO_OK) r = launch_bucket(bk, 1, 1, s);
            if (r != CRYO_OK) return r;
            ++k;
            --count;
            par = 0;
        }
        if (count == 0) return CRYO_OK;
        r = launch_set_i64(k0p, k, s);
        const int64_t blocks = count / GRAPH_STEPS, rem = count % GRAPH_STEPS;
        if (r == CRYO_OK && blocks > 0) r = ensure_graph();
        for (int64_t q = 0; q < blocks && r == CRYO_OK; ++q)
            if (hipGraphLaunch(b->exec, s) != hipSuccess) r = fail(CRYO_ERR_DEVICE, "graph launch failed");
        // (each block advanced the counter by GRAPH_STEPS)
        for (const Bucket &bk : b->buckets)
            if (r == CRYO_OK) r = launch_bucket(bk, 0, rem, s);
        k += count;
        par = (int)(rem & 1);
        return r;
    };
    // Step kk, where an instance of the turn-on model starts a pulse: single-
    // plan launches of the same kernels, that instance's step as the 100
    // sub-steps of dt / 100 of eq. (22) (an even number of buffer swaps, so
    // its field is then copied to the buffer the other instances' steps write).
    auto special = [&](int64_t kk) -> cryo_status {
        for (int i = 0; i < n; ++i) {
            const cryo_plan *p = b->plans[i];
            char *f = w + b->ws_field[i];
            void *buf[2] = {f, f + field_bytes_internal(p)};
            int *flag = (int *)w + i;
            cryo_status r = CRYO_OK;
            if (p->sub && pulse_start(p->pulse, kk)) {
                int c = par;
                for (int q = 0; q < 100 && r == CRYO_OK; ++q) {
                    const double X = p->pulse.amplitude * turn_on_source(p->pulse, kk, q);
                    r = launch_step(p->sub, buf[c], buf[c ^ 1], X, nullptr, flag, s);
                    c ^= 1;
                }
                if (r == CRYO_OK && hipMemcpyAsync(buf[par ^ 1], buf[par], field_bytes_internal(p),
                                                   hipMemcpyDeviceToDevice, s) != hipSuccess)
                    r = fail(CRYO_ERR_DEVICE, "sub-step field copy");
            } else {
                const double X = p->pulse.amplitude * source_fraction(p->pulse, kk);
                r = launch_step(p, buf[par], buf[par ^ 1], X, nullptr, flag, s);
            }
            if (r != CRYO_OK) return r;
        }
        ++k;
        par ^= 1;
        return CRYO_OK;
    };
    // the steps of the range where a turn-on instance starts a pulse
    std::vector<int64_t> starts;
    for (const cryo_plan *p : b->plans) {
        if (!p->sub || !(p->pulse.W > 0) || !pulse_starts_on_steps(p->pulse)) continue;
        const int64_t kb = (int64_t)p->pulse.b0, kp = (int64_t)p->pulse.P;
        int64_t kk = kb;
        if (k0 > kb) kk = kb + (k0 - kb + kp - 1) / kp * kp;
        for (; kk < k0 + nsteps; kk += kp)
            if (pulse_start(p->pulse, kk)) starts.push_back(kk);
    }
    std::sort(starts.begin(), starts.end());
    starts.erase(std::unique(starts.begin(), starts.end()), starts.end());
    for (int64_t ks : starts) {
        st = regular(ks - k);
        if (st == CRYO_OK) st = special(ks);
        if (st != CRYO_OK) return st;
    }
    st = regular(k0 + nsteps - k);
    if (st != CRYO_OK) return st;
    b->graph_ws = ws;
    for (int i = 0; i < n; ++i) {
        const cryo_plan *p = b->plans[i];
        char *f = w + b->ws_field[i];
        st = launch_from_internal(p, f + par * field_bytes_internal(p),
                                  (char *)T + es * b->off[i], (int *)w + i, s);
        if (st != CRYO_OK) return st;
    }
    return CRYO_OK;
}

cryo_status cryo_batch_poll(const cryo_batch *b, const void *ws, void *stream, int32_t *bad) {
    if (!b || !ws) return fail(CRYO_ERR_ARG, "null argument");
    std::vector<int> flags(b->plans.size());
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(flags.data(), ws, sizeof(int) * flags.size(), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(CRYO_ERR_DEVICE, "poll copy failed");
    int32_t first = -1;
    for (size_t i = 0; i < flags.size(); ++i)
        if (flags[i] && first < 0) first = (int32_t)i;
    if (bad) *bad = first;
    if (first >= 0)
        return fail(CRYO_ERR_NONFINITE, "instance " + std::to_string(first) +
                                            " produced a non-finite or out-of-range temperature");
    return CRYO_OK;
}

cryo_status cryo_batch_shape(const cryo_batch *b, int32_t i, int32_t *shape) {
    if (!b || !shape || i < 0 || i >= (int32_t)b->plans.size())
        return fail(CRYO_ERR_ARG, "bad argument");
    return cryo_plan_shape(b->plans[i], shape, shape + 1, shape + 2);
}

}  // extern "C"
