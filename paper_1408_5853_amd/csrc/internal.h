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
constexpr int STEP_WAVES_HOST = 8;  // waves per stepping workgroup
constexpr int BATCH_LPW = 4;        // default lines per wave of batch instances

// Built chunk shapes (rows per lane, waves per line) of the stepping kernel:
// one wave per line with 2..16 rows per lane (so that padding stays small
// for any nr up to 1024), then 4 or 8 rows per lane over 2 or 4 waves.
#define CRYO_FOR_SHAPES(X) \
    X(2, 1) X(3, 1) X(4, 1) X(5, 1) X(6, 1) X(7, 1) X(8, 1) X(10, 1) X(12, 1) X(16, 1) \
    X(4, 2) X(8, 2) X(4, 4) X(8, 4)
constexpr int ONE_WAVE_RPL[] = {2, 3, 4, 5, 6, 7, 8, 10, 12, 16};
inline bool shape_built(int rpl, int wpl) {
#define CRYO_SHAPE_EQ(RP, GW) if (rpl == RP && wpl == GW) return true;
    CRYO_FOR_SHAPES(CRYO_SHAPE_EQ)
#undef CRYO_SHAPE_EQ
    return false;
}

// Row classes of one radial line (eq. (13), eq. (18), eq. (15), padding).
enum RowKind : uint32_t { K_PAD = 0, K_LO = 1, K_HI = 2, K_CAP = 3, K_IFACE = 4 };

// Material laws.  A law id selects a multiplier K and an exponent row:
//   ids 0..L-1    radial conductivity of layer m:  K = k_scale k0 tref^-p, e = p
//   ids L..2L-1   axial conductivity / eta^2:      K = (that) / eta^2,     e = p
//   ids 2L..3L-1  rho c / dt of layer m:           K = rho c0 tref^-q / dt, e = q
//   id  3L        zero law (value 0),  id 3L+1  unit law (value 1)
// value = K * T^e.  Exponent rows: 0..L-1 hold p_m, L..2L-1 hold q_m, 2L is 0.
// The stepping kernel has a second law set (`flaws`) in which every capacity
// row is multiplied by eta^2 (so its axial faces use the radial law) and
// every interface row is divided by the outer layer's law:
//   ids 0..L-1    radial conductivity of layer m (as above)
//   ids L..2L-2   lambda_m / lambda_{m+1}: K = K_m / K_{m+1}, e = p_m - p_{m+1}
//   ids 2L..3L-1  eta^2 rho c / dt of layer m
//   zero and unit laws as above.
constexpr int MAX_LAWS = 3 * MAX_LAYERS + 2;
__host__ __device__ inline int law_zero(int L) { return 3 * L; }
__host__ __device__ inline int law_unit(int L) { return 3 * L + 1; }

// Per-row packed info word:
//   bits 0-2 kind, bit 3 heater capacity node, bit 4 held boundary row,
//   bit 5 its side (0 inner, 1 outer), bits 6-11 law of the east r-face,
//   bits 12-17 law of slot 2, bits 18-23 law of slot 3, bits 24-29 capacity law.
// Slot 2 is the north axial face of a capacity row (eq. (11)), slot 3 is not
// used by capacity rows (their south face is the previous line's north
// face); an interface row (eq. (18)) evaluates its inner and outer layer laws
// at the node in slots 2 and 3; boundary and padding rows use the zero and
// unit laws so that one formula serves every row.  The stepping kernel's
// words (`finfo`, law ids of `flaws`): slot 2 of a capacity row is the
// radial law of its layer, slot 2 of an interface row the ratio law, slot 3
// is unused, and held walls are found by position (rows 0 and nr - 1).
__host__ __device__ inline uint32_t info_pack(uint32_t kind, uint32_t heat, uint32_t held,
                                              uint32_t side, uint32_t lawE, uint32_t law2,
                                              uint32_t law3, uint32_t lawC) {
    return kind | (heat << 3) | (held << 4) | (side << 5) | (lawE << 6) | (law2 << 12) |
           (law3 << 18) | (lawC << 24);
}

struct Laws {
    int L;
    int cube;                       // every capacity exponent q is 3
    double K[MAX_LAWS];             // multiplier per law id
    double lk[MAX_LAWS];            // log2 K (-2000 for the zero law)
    double e[MAX_LAWS];             // exponent per law id
};

// FP64 powers T^e from tables: T = 2^x m, m in [1,2); m0 = 1 + (j + 1/2)/NM
// for the top POW_MBITS mantissa bits j; u = m / m0 - 1 (|u| <= 1/(2 NM));
// K T^e = [K 2^(x e)] m0^e (1 + u)^e, with (1 + u)^e summed as its binomial
// series to degree 7.  The first dropped term bounds the truncation:
// |binom(e, 8)| u^8 <= |binom(e, 8)| 2^-56 relative, which is 0 for e = 0..7,
// 1.4e-17 for e = -1, 2.3e-15 for e = -4 and 9e-14 for e = -8; the host
// refuses exponents whose bound exceeds POW_TRUNC_MAX (about -5.3 <= e <= 12.5).
// One block of doubles per law id:
//   [0, 2 NM)            {m0^e, 2/m0} for j = 0..NM-1
//   [2 NM, 2 NM + NE)    K 2^(x e) for binades x = EMIN..EMIN+NE-1
//   2 NM + NE            e; the next slot is unused
//   2 NM + NE + 2 ..     binomial(e, k), k = 2..7
//   then 2 pad doubles: a 1296-byte block shifts successive laws by 4 LDS
//   banks, so lanes reading different laws do not collide
constexpr int POW_MBITS = 6, POW_NM = 1 << POW_MBITS, POW_NE = 24, POW_EMIN = -4;
constexpr int POW_DEG = 7;
constexpr double POW_TRUNC_MAX = 1e-14;
constexpr double POW_TLO = 0.0625, POW_THI = 1048576.0;   // 2^EMIN, 2^(EMIN+NE)
constexpr int POW_BX = 2 * POW_NM;                 // binade multipliers
constexpr int POW_BE = POW_BX + POW_NE;            // exponent, then binomials from +2
constexpr int POW_BLK = POW_BE + 2 + (POW_DEG - 1) + 2;
// Polynomial laws (eqs. (23), (24)) use the same blob size with POLY_BLK
// doubles per law id in the stepping kernel's id scheme: ids 0..L-1 hold
// k_scale b_k of layer m, ids 2L..3L-1 eta^2 rho a_k / dt, the zero and unit
// laws 0 and 1; the ratio ids are unused (an interface row divides its
// inner layer's law, slot 2, by its outer layer's, slot 3).
constexpr int POLY_BLK = 6;
// blob: (3L+2) law blocks, then {cube multiplier, addend} pairs per law id
__host__ __device__ inline size_t pow_blob_doubles(int L) {
    return (size_t)(3 * L + 2) * (POW_BLK + 2);
}

// Arguments of the adjoint kernels of one step (FP64, internal layout).
struct AdjArgs {
    const double *T;        // T^n (internal layout)
    const double *X;        // T^{n+1}
    const double *lam_in;   // lam^{n+1}
    double *Y;              // pass 1 out: y
    double *lpart;          // pass 1 out: radial part of lam^n
    double *lam_out;        // pass 2 out: lam^n
    double *acc;            // per workgroup: [workgroups][3][np] row sums
    double *accg;           // per workgroup: [workgroups][2]  (y s, y Q ds/dw)
    double s, ds;           // pulse average of step n and its width derivative
    const double *cS;       // dJ_n / dS_n in device memory (null: 0, as for n = 0)
    double xs;              // scale of the capacity rows (eta^2): the source's too
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
    int wpl;                 // waves per line
    int np;                  // padded line length = 64 * wpl * rpl
    int lpw;                 // interior lines marched by one wave per step
    double eta;
    std::vector<double> r, h;         // node radii, interval widths (h[0] unused)
    std::vector<int> lay;             // layer of interval i
    std::vector<int> kind;            // row class per node
    // the laws as the equations write them (per layer: radial, axial,
    // capacity; from these the kernels' laws are formed), and host copies of
    // the lane-major row tables in the kernels' form of the rows of eqs.
    // (13), (15), (18) (capacity rows times eta^2, interface rows divided by
    // the outer law), which the stepping and the adjoint kernels share
    cryo::Laws laws;
    std::vector<double> fgw, fge;
    std::vector<uint32_t> finfo;
    cryo::Laws flaws;
    std::vector<double> fpow_blob;
    cryo::Pulse pulse;
    int surf_lane, surf_reg;          // owner of row nr-1
    // device tables (read-only, made at create time)
    void *d_rows = nullptr;           // [2][np]: fgw, fge
    uint32_t *d_info = nullptr;       // [np]: finfo
    double *d_pow = nullptr;          // fpow_blob
    int device = 0;
    // transient turn-on model (eq. (22)): the same cell at dt / 100, whose
    // tables step the sub-steps of each pulse-start step (null when off)
    cryo_plan *sub = nullptr;
    // polynomial laws (eqs. (23), (24)) and the Joule source (eq. (25)):
    // when set, fpow_blob holds the polynomial coefficients (see POLY_BLK)
    // and finfo's slot 3 the denominator law of each row (the outer layer's
    // law on interface rows, the unit law elsewhere)
    bool poly = false;
    std::vector<double> poly_a, poly_b;   // [L][4], [L][5] as given
    double joule_tref = 0.0;
    // stepped domain (eq. (9)): lines above z_full span nodes 0..nr_top-1
    // (the terminal); its lines' tables in the stepping kernel's form
    bool stepped = false;
    int z_full = 0, nr_top = 0;
    std::vector<double> tfgw, tfge;
    std::vector<uint32_t> tfinfo;
    void *d_rows2 = nullptr;          // [2][np]: tfgw, tfge
    uint32_t *d_info2 = nullptr;      // [np]: tfinfo
    // FP64 plans: the parameter weights of the gradient (grad_param_table)
    double *d_grad = nullptr;
    // kernel steps at the end of a gradient's run whose states its forward
    // keeps (no recompute for their adjoint steps); 0: none
    int64_t grad_store = 0;
};

namespace cryo {
void set_error(const std::string &msg);
cryo_status fail(cryo_status st, const std::string &msg);
double source_fraction(const Pulse &p, int64_t k);
bool pulse_starts_on_steps(const Pulse &p);
bool pulse_start(const Pulse &p, int64_t k);
double turn_on_source(const Pulse &p, int64_t k, int i);

// launchers (forward.hip)
cryo_status launch_to_internal(const cryo_plan *p, const void *T, void *Ti, int *flag,
                               hipStream_t s);
cryo_status launch_from_internal(const cryo_plan *p, const void *Ti, void *T, int *flag,
                                 hipStream_t s);
cryo_status launch_fill(const cryo_plan *p, void *T, hipStream_t s);
cryo_status launch_step(const cryo_plan *p, const void *Tin, void *Tout, double X,
                        double *partial, int *flag, hipStream_t s);
cryo_status launch_surf_reduce(const cryo_plan *p, const double *partial, int nsteps,
                               double *out, hipStream_t s);
int step_grid(const cryo_plan *p);
size_t step_lds(const cryo_plan *p);            // dynamic LDS of the stepping kernel
constexpr size_t MAX_STEP_LDS = 160 * 1024 - 4096;   // leaves room for static LDS
cryo_status ensure_device(cryo_plan *p);
// host.hip: cryo_forward's device work on a checked workspace, and whether
// a plan (and its turn-on sub-plan) has made its device tables
cryo_status forward_in(const cryo_plan *p, void *T, int64_t k0, int64_t nsteps, char *w,
                       double *surf, hipStream_t s);
bool plan_tables_on_device(const cryo_plan *p);
// grad.hip: the weights that turn the adjoint's per-row face sums into the
// thickness and conductivity-scale derivatives (size grad_param_doubles)
std::vector<double> grad_param_table(const cryo_plan *p);
inline size_t grad_param_doubles(int nr, int L) { return 2 * (size_t)nr * L + 3 * (size_t)nr + L; }
}  // namespace cryo
