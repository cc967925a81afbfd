// Internal declarations shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "cryocell.h"

namespace cryo {

constexpr int WAVE = 64;
constexpr int MAX_LAYERS = 16;
constexpr int MAX_NR = 2048;
constexpr int SURF_CHUNK = 1024;    // steps per surface reduction round

// Row classes of one radial line (eq. (13), eq. (18), eq. (15), padding).
enum RowKind : uint32_t { K_PAD = 0, K_LO = 1, K_HI = 2, K_CAP = 3, K_IFACE = 4 };

// Per-row packed info word:
//   bits 0-2  kind, bit 3 heater capacity node,
//   bits 4-8  law of the east r-face (radial law table),
//   bits 9-13 law of slot 2, bits 14-18 law of slot 3 (combined table:
//             0..L-1 radial laws, L..2L-1 axial laws already divided by eta^2),
//   bits 19-23 capacity law (layer of the node).
__host__ __device__ inline uint32_t info_pack(uint32_t kind, uint32_t heat, uint32_t lawE,
                                              uint32_t law2, uint32_t law3, uint32_t lawC) {
    return kind | (heat << 3) | (lawE << 4) | (law2 << 9) | (law3 << 14) | (lawC << 19);
}

// lambda = exp2(p * log2(T) + lk); rho c / dt = exp2(q * log2(T) + lrc)
struct Laws {
    double p[2 * MAX_LAYERS], lk[2 * MAX_LAYERS];
    double q[MAX_LAYERS], lrc[MAX_LAYERS];
    int n;          // number of entries in p/lk (2L)
    int L;
};

struct Pulse {      // in step units, snapped
    double b0, W, P;
    double amplitude;
};

}  // namespace cryo

// Opaque plan.
struct cryo_plan {
    cryo_problem prob;
    std::vector<cryo_layer> layers;
    cryo_dtype dtype;
    int nr, nz, L;
    int rpl;                 // radial rows per lane (chunk length)
    int np;                  // padded line length = 64 * rpl
    double eta;
    std::vector<double> r, h;         // node radii, interval widths (h[0] unused)
    std::vector<int> lay;             // layer of interval i
    std::vector<int> kind;            // row class per node
    // host copies of the lane-major tables
    std::vector<double> gw, ge;
    std::vector<uint32_t> info;
    cryo::Laws laws;
    cryo::Pulse pulse;
    int surf_lane, surf_reg;          // owner of row nr-1
    // device tables (read-only, made at create time)
    void *d_gw = nullptr, *d_ge = nullptr;
    uint32_t *d_info = nullptr;
    int device = 0;
};

namespace cryo {
void set_error(const std::string &msg);
cryo_status fail(cryo_status st, const std::string &msg);
double source_fraction(const Pulse &p, int64_t k);

// launchers (forward.hip)
cryo_status launch_to_internal(const cryo_plan *p, const void *T, void *Ti, int *flag,
                               hipStream_t s);
cryo_status launch_from_internal(const cryo_plan *p, const void *Ti, void *T, int *flag,
                                 hipStream_t s);
cryo_status launch_fill(const cryo_plan *p, void *T, hipStream_t s);
cryo_status launch_step(const cryo_plan *p, const void *Tin, void *Tout, double X,
                        double *partial, hipStream_t s);
cryo_status launch_surf_reduce(const cryo_plan *p, const double *partial, int nsteps,
                               double *out, hipStream_t s);
int step_grid(const cryo_plan *p);
cryo_status ensure_device(cryo_plan *p);
}  // namespace cryo
