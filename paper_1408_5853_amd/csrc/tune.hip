// Autotuner: times every built kernel shape (rows per lane, waves per line)
// and lines-per-wave on a problem and returns the fastest.  The tuner owns
// its trial field and workspace (device allocations of its own, outside any
// stepping call).  An optional text cache keyed by (dtype, nr, nz, layers)
// records results across runs.
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "internal.h"

using namespace cryo;

namespace {

std::string cache_key(const cryo_problem *p, cryo_dtype dt) {
    char b[128];
    snprintf(b, sizeof b, "%s %d %d %d", dt == CRYO_F64 ? "f64" : "f32", p->geom.nr, p->geom.nz,
             p->geom.n_layers);
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

}  // extern "C"
