// Device code shared by the stepping and adjoint kernels: law evaluation
// from LDS tables, compensated FP32 pairs, wave shuffles and the partitioned
// tridiagonal solve.
#pragma once

#include <math.h>
#include <string.h>

#include "internal.h"

namespace cryo {

// reciprocal: hardware estimate (relative error below 5e-8 on gfx950)
// refined by one Newton step (below 3e-15).  The step's solves work in delta
// form, so a pivot off by that much perturbs only the increment, by a
// relative 3e-15; the adjoint's uses (transposed solves, derivative factors)
// carry it into the gradient at the same relative size.
__device__ inline double rcp(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(fma(-x, r, 1.0), r, r);
}
__device__ inline float rcp(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(fmaf(-x, r, 1.0f), r, r);
}

// Law evaluation K[id] * T^e[id] from tables staged in LDS.
template <typename R>
struct LawLds;

template <>
struct LawLds<double> {
    const double *blk;      // law blocks (POW_BLK doubles per law id)
    const double *cka;      // cube path: K T^3 + A, pairs {K, A} per law id
    // T on the table range [2^POW_EMIN, 2^(POW_EMIN+POW_NE)) K
    static __device__ inline bool in_range(double x) {
        return x >= POW_TLO && x < POW_THI;
    }
    __device__ inline double expo(int id) const { return blk[id * POW_BLK + POW_BE]; }
    // K[id] T^e[id]; T off the table range (or not finite) is clamped to its
    // edge binade, so callers check the range themselves (in_range)
    __device__ inline double lawc(int id, double x) const { return pw<1>(id, x); }
    // K[id] (s/2)^e[id]: the law at the mean of two values given their sum s
    // (halving only moves the binade: same tables, index one binade lower)
    __device__ inline double lawm(int id, double s) const { return pw<2>(id, s); }
    template <int SH>
    __device__ inline double pw(int id, double x) const {
        const double mh = __builtin_amdgcn_frexp_mant(x);          // x = mh 2^xe, mh in [1/2, 1)
        const int xe = __builtin_amdgcn_frexp_exp(x);
        const int xc = min(max(xe, POW_EMIN + SH), POW_EMIN + POW_NE + SH - 1) - (POW_EMIN + SH);
        const unsigned hi = (unsigned)(__double_as_longlong(x) >> 32);
        const int jm = (int)__builtin_amdgcn_ubfe(hi, 20 - POW_MBITS, POW_MBITS);
        const double *B = blk + id * POW_BLK;
        const double2 ee = *(const double2 *)(B + POW_BE);      // e
        const double2 c23 = *(const double2 *)(B + POW_BE + 2);
        const double2 c45 = *(const double2 *)(B + POW_BE + 4);
        const double2 c67 = *(const double2 *)(B + POW_BE + 6);
        const double2 mm = *(const double2 *)(B + 2 * jm);
        const double u = fma(mh, mm.y, -1.0);                   // m / m0 - 1
        // (1 + u)^e, |u| <= 2^-(POW_MBITS+1), by Estrin's scheme (depth 4,
        // against 7 dependent steps for Horner's)
        const double u2 = u * u, u4 = u2 * u2;
        const double p01 = fma(ee.x, u, 1.0), p23 = fma(c23.y, u, c23.x);
        const double p45 = fma(c45.y, u, c45.x), p67 = fma(c67.y, u, c67.x);
        const double s = fma(fma(p67, u2, p45), u4, fma(p23, u2, p01));
        return (B[POW_BX + xc] * mm.x) * s;
    }
    // as lawc, and flags an argument off the table range
    __device__ inline double law(int id, double x, int &bad) const {
        bad |= !in_range(x);
        return lawc(id, x);
    }
    __device__ inline double cube(int id, double x) const {
        const double2 k = *(const double2 *)(cka + 2 * id);
        return fma(k.x, x * x * x, k.y);
    }
};

// Polynomial laws (eqs. (23), (24)): sum_k c_k x^k, k <= 4, by Horner's
// rule, from POLY_BLK doubles per law id staged in LDS in place of the power
// tables (c_0 .. c_4, one pad).  Interface rows need a quotient of two laws,
// which callers form.
template <typename R>
struct LawPoly;
template <>
struct LawPoly<double> {
    const double *c;
    static __device__ inline bool in_range(double x) { return LawLds<double>::in_range(x); }
    __device__ inline double lawc(int id, double x) const {
        const double2 k01 = *(const double2 *)(c + POLY_BLK * id);
        const double2 k23 = *(const double2 *)(c + POLY_BLK * id + 2);
        const double k4 = c[POLY_BLK * id + 4];
        return fma(fma(fma(fma(k4, x, k23.y), x, k23.x), x, k01.y), x, k01.x);
    }
    // the law at the mean of two values given their sum
    __device__ inline double lawm(int id, double s) const { return lawc(id, 0.5 * s); }
};
// FP32 pairs: the same coefficients rounded to float, Horner's rule in float
template <>
struct LawPoly<float> {
    const float *c;
    __device__ inline float lawc(int id, float x) const {
        const float2 k01 = *(const float2 *)(c + POLY_BLK * id);
        const float2 k23 = *(const float2 *)(c + POLY_BLK * id + 2);
        const float k4 = c[POLY_BLK * id + 4];
        return fmaf(fmaf(fmaf(fmaf(k4, x, k23.y), x, k23.x), x, k01.y), x, k01.x);
    }
    __device__ inline float lawm(int id, float s) const { return lawc(id, 0.5f * s); }
};

// FP32: 2^(e log2 s + lk); the stepping kernel's tables hold lk = log2 K - e,
// so that s is the sum of the two values whose mean the law is taken at.
// The hardware log2 and exp2 instructions serve directly: s is a sum of two
// temperatures (a normal float), and the zero law's exponent (lk = -2000)
// gives 0; only law values below 1e-38, which no law here reaches, could
// differ from the library functions, which add a rescaling for subnormal
// arguments and results around the same instructions (six more instructions
// per law).
template <>
struct LawLds<float> {
    const float *lk, *ex, *cka;
    static __device__ inline bool in_range(float) { return true; }
    __device__ inline float lawm(int id, float s) const {
        return __builtin_amdgcn_exp2f(fmaf(ex[id], __builtin_amdgcn_logf(s), lk[id]));
    }
    __device__ inline float cube(int id, float x) const {
        const float2 k = *(const float2 *)(cka + 2 * id);
        return fmaf(k.x, x * x * x, k.y);
    }
};

template <typename R>
struct StepArgs {
    const R *Tin;             // single plan: this step's input and output
    R *Tout;
    R *buf[2];                // batch: ping-pong buffers (step n reads buf[n & 1])
    const R *gw, *ge;         // per-row tables: west/east geometry factors
    const uint32_t *info;
    const double *pow_blob;   // FP64 power tables (device)
    Laws laws;
    int nz, np;
    int lpw;                  // lines per wave (a contiguous block)
    R X;                      // amplitude * pulse average of this step
    int held[4];              // r_inner, r_outer, z_low, z_high
    R val[4];
    double *partial;          // nullable: per-workgroup surface partial sums
    int *flag;                // error word: bit 1 = temperature off the law tables
    double wz_end, wz_mid;    // trapezoid weights of the surface mean
    int surf_lane, surf_reg;
    int groups;               // workgroups of one step of this instance
    Pulse pulse;              // batch: schedule evaluated on the device
    int joule;                // heater source times X / sqrt(T) (eq. (25)), X holding sqrt(T_J)
    // stepped domain (eq. (9)): lines above z_full take the terminal's row
    // tables (nz - 1 when there is none)
    int z_full;
    const R *gw2, *ge2;
    const uint32_t *info2;
    double jsq;               // sqrt(T_J) with the Joule source, else 1 (batch
                              // and adjoint kernels form their source with it)
};

constexpr int STEP_WAVES = STEP_WAVES_HOST;

// v of lane (idx4 / 4) mod 64: the permute takes address bits 7:2 as the
// source lane, so idx4 = 4 lane + (256 - 4 s) reads lane - s around the wave
// and the constant folds into the instruction's offset field
__device__ inline float lane_read(float v, int idx4) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(idx4, __builtin_bit_cast(int, v)));
}
__device__ inline double lane_read(double v, int idx4) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_ds_bpermute(idx4, (int)b);
    const int hi = __builtin_amdgcn_ds_bpermute(idx4, (int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <typename R>
__device__ inline R shfl_up1(R v, int s, int lane) {
    R u = __shfl_up(v, s, WAVE);
    return lane >= s ? u : (R)0;
}
template <typename R>
__device__ inline R shfl_dn1(R v, int s, int lane) {
    R u = __shfl_down(v, s, WAVE);
    return lane + s < WAVE ? u : (R)0;
}

// Forward elimination of one row r >= 1 of a lane's chunk, with a fill-in
// column on the chunk's first row x_0:  al_r x_0 + x_r + ga_r x_{r+1} = de_r
template <typename R, int RPL>
__device__ inline void elim_row(int r, R aa, R bb, R cc, R dd, R (&al)[RPL], R (&ga)[RPL],
                                R (&de)[RPL]) {
    if (r == 1) {
        const R inv = rcp(bb);
        al[1] = aa * inv;
        ga[1] = cc * inv;
        de[1] = dd * inv;
    } else {
        const R inv = rcp(bb - aa * ga[r - 1]);
        al[r] = -aa * al[r - 1] * inv;
        ga[r] = cc * inv;
        de[r] = (dd - aa * de[r - 1]) * inv;
    }
}

// Rest of the partitioned solve, after every lane has eliminated rows 1..RPL-1
// of its chunk (elim_row).  A line is spread over G waves (64 G lanes, lane
// lg = wig * 64 + lane owns rows lg*RPL .. lg*RPL+RPL-1):
//  1. back-eliminate each chunk onto its ends x_0, x_e;
//  2. eliminate x_0 with the first row, leaving one unknown x_e per lane and a
//     tridiagonal reduced system across the 64 G lanes;
//  3. each wave solves its 64 unknowns by parallel cyclic reduction, with the
//     couplings to the neighbouring waves' unknowns as two extra right-hand
//     sides (spikes);
//  4. the 2 G wave-end unknowns satisfy a small system, exchanged in LDS and
//     solved by every lane;
//  5. back-substitution.
// (a0, b0, c0, d0) is the chunk's first row.  On exit x[r] holds the solution
// of row lg * RPL + r.  xch: LDS exchange area of this line's waves (9 G
// values); all waves of the workgroup must call this together when G > 1.
template <typename R, int RPL, int G>
__device__ inline void solve_tail(R a0, R b0, R c0, R d0, R (&al)[RPL], R (&ga)[RPL],
                                  R (&de)[RPL], R (&x)[RPL], int lane, int wig, R *xch) {
    static_assert(RPL >= 2, "chunks of at least two rows");
#pragma unroll
    for (int r = RPL - 3; r >= 1; --r) {
        de[r] = de[r] - ga[r] * de[r + 1];
        al[r] = al[r] - ga[r] * al[r + 1];
        ga[r] = -ga[r] * ga[r + 1];
    }
    // first row: a0 x_e(k-1) + sb x_0 + sc x_e(k) = sd
    R sb, sc, sd;
    if (RPL == 2) {
        sb = b0;
        sc = c0;
        sd = d0;
    } else {
        sb = b0 - c0 * al[1];
        sc = -c0 * ga[1];
        sd = d0 - c0 * de[1];
    }
    const R isb = rcp(sb);
    const R sig = a0 * isb, tau = sc * isb, rho = sd * isb;   // x_0 = rho - sig x_e(k-1) - tau x_e(k)
    // Lane reads wrap around the wave: a value from past either end only meets
    // a coefficient that is exactly zero there (the line's first row has no
    // west coupling, its last no east coupling, the spikes zero the wave
    // ends, and cyclic reduction keeps couplings beyond the ends zero), and
    // every lane's values are finite, so no select is needed.
    // (l4 is opaque to the optimiser: the twelve addresses are formed here,
    // not hoisted out of the caller's loop into registers held throughout)
    int l4 = lane << 2;
    asm volatile("" : "+v"(l4));
    const int up1 = l4 + 4 * (WAVE - 1), dn1 = l4 + 4;
    R sigN = lane_read(sig, dn1), tauN = lane_read(tau, dn1);
    R rhoN = lane_read(rho, dn1);
    if constexpr (G > 1) {
        if (lane == 0) {
            xch[3 * wig + 0] = sig;
            xch[3 * wig + 1] = tau;
            xch[3 * wig + 2] = rho;
        }
        __syncthreads();
        if (lane == WAVE - 1 && wig < G - 1) {
            sigN = xch[3 * (wig + 1) + 0];
            tauN = xch[3 * (wig + 1) + 1];
            rhoN = xch[3 * (wig + 1) + 2];
        }
    }
    const int e = RPL - 1;
    // reduced row of x_e(k):  A x_e(k-1) + B x_e(k) + C x_e(k+1) = D
    R A = -al[e] * sig;
    R B = (R)1 - al[e] * tau - ga[e] * sigN;
    R C = -ga[e] * tauN;
    R D = de[e] - al[e] * rho - ga[e] * rhoN;
    {
        const R ib = rcp(B);
        A *= ib;
        C *= ib;
        D *= ib;
    }
    // spikes: couplings across the wave ends moved to extra right-hand sides
    R PL = (R)0, PR = (R)0, Afirst = (R)0, Clast = (R)0;
    if constexpr (G > 1) {
        Afirst = __shfl(A, 0, WAVE);
        Clast = __shfl(C, WAVE - 1, WAVE);
        if (lane == 0) {
            A = (R)0;
            PL = (R)1;
        }
        if (lane == WAVE - 1) {
            C = (R)0;
            PR = (R)1;
        }
    }
#pragma unroll
    for (int s = 1; s < WAVE; s <<= 1) {
        const int iu = l4 + 4 * (WAVE - s), id = l4 + 4 * s;
        const R Am = lane_read(A, iu), Cm = lane_read(C, iu), Dm = lane_read(D, iu);
        const R Ap = lane_read(A, id), Cp = lane_read(C, id), Dp = lane_read(D, id);
        const R ib = rcp((R)1 - A * Cm - C * Ap);
        const R nA = -A * Am * ib;
        const R nC = -C * Cp * ib;
        const R nD = (D - A * Dm - C * Dp) * ib;
        if constexpr (G > 1) {
            const R PLm = lane_read(PL, iu), PLp = lane_read(PL, id);
            const R PRm = lane_read(PR, iu), PRp = lane_read(PR, id);
            PL = (PL - A * PLm - C * PLp) * ib;
            PR = (PR - A * PRm - C * PRp) * ib;
        }
        A = nA;
        C = nC;
        D = nD;
    }
    R xe = D, uL = (R)0;
    if constexpr (G > 1) {
        // x_e = y + vL uL + vR uR with uL, uR the neighbouring waves' end unknowns
        const R vL = -Afirst * PL, vR = -Clast * PR;
        R *xi = xch + 3 * G;     // per wave: y, vL, vR at its first and last lane
        if (lane == 0) {
            xi[6 * wig + 0] = D;
            xi[6 * wig + 1] = vL;
            xi[6 * wig + 2] = vR;
        }
        if (lane == WAVE - 1) {
            xi[6 * wig + 3] = D;
            xi[6 * wig + 4] = vL;
            xi[6 * wig + 5] = vR;
        }
        __syncthreads();
        // f_w = y0 + vL0 l_{w-1} + vR0 f_{w+1};  l_w = y63 + vL63 l_{w-1} + vR63 f_{w+1}
        // eliminate upwards: f_w = g_w + h_w f_{w+1}, l_w = p_w + q_w f_{w+1}
        R gq[G], hq[G], pq[G], qq[G];
        R pPrev = (R)0, qPrev = (R)0;
#pragma unroll
        for (int w = 0; w < G; ++w) {
            const R y0 = xi[6 * w + 0], vL0 = xi[6 * w + 1], vR0 = xi[6 * w + 2];
            const R y63 = xi[6 * w + 3], vL63 = xi[6 * w + 4], vR63 = xi[6 * w + 5];
            const R den = rcp((R)1 - vL0 * qPrev);
            gq[w] = (y0 + vL0 * pPrev) * den;
            hq[w] = vR0 * den;
            pq[w] = y63 + vL63 * (pPrev + qPrev * gq[w]);
            qq[w] = vR63 + vL63 * qPrev * hq[w];
            pPrev = pq[w];
            qPrev = qq[w];
        }
        R fNext = (R)0, fw[G], lw[G];
#pragma unroll
        for (int w = G - 1; w >= 0; --w) {
            fw[w] = gq[w] + hq[w] * fNext;
            lw[w] = pq[w] + qq[w] * fNext;
            fNext = fw[w];
        }
        R uR = (R)0;
#pragma unroll
        for (int w = 0; w < G; ++w) {
            if (w == wig - 1) uL = lw[w];
            if (w == wig + 1) uR = fw[w];
        }
        xe = D + vL * uL + vR * uR;
    }
    R xeP = lane_read(xe, up1);
    if (G > 1 && lane == 0) xeP = uL;
    const R x0 = rho - sig * xeP - tau * xe;
#pragma unroll
    for (int r = 1; r < RPL - 1; ++r) x[r] = de[r] - al[r] * x0 - ga[r] * xe;
    x[0] = x0;
    x[e] = xe;
}

// FP32 fields carry a compensated pair per node (hi + lo, |lo| <= ulp(hi)/2):
// a single float cannot hold per-step increments far below its ulp, so the
// low part keeps them; arithmetic stays in FP32.
template <typename R>
struct Pair {
    static constexpr bool on = false;
};
template <>
struct Pair<float> {
    static constexpr bool on = true;
};

// (a_hi + a_lo) - (b_hi + b_lo) for nearby values: the hi difference is exact
template <typename R>
__device__ inline R dif(R ah, R al, R bh, R bl) {
    if constexpr (Pair<R>::on)
        return (ah - bh) + (al - bl);
    else
        return ah - bh;
}

// LDS bytes of the staged tables: laws, then per-row gw, ge, info
template <typename R>
__host__ __device__ inline size_t law_lds_bytes(int L) {
    const int nlaw = 3 * L + 2;
    if constexpr (sizeof(R) == 8)
        return sizeof(double) * pow_blob_doubles(L);
    else    // room for POLY_BLK floats per law id (polynomial laws)
        return sizeof(float) * POLY_BLK * nlaw;
}
// The stepping kernel also keeps a two-slot ring of line buffers per wave
// (the lines after the current one, loaded straight into LDS): a slot is
// RPL rows x planes x 64 lanes.
template <typename R>
__host__ __device__ inline size_t ring_lds_offset(int L, int np) {
    size_t b = (law_lds_bytes<R>(L) + 15) & ~(size_t)15;
    return (b + (2 * sizeof(R) + sizeof(uint32_t)) * (size_t)np + 15) & ~(size_t)15;
}
// one set of per-row tables (gw, ge, info) of an np-row line, 16-aligned
template <typename R>
__host__ __device__ inline size_t step_tables_bytes(int np) {
    return ((2 * sizeof(R) + sizeof(uint32_t)) * (size_t)np + 15) & ~(size_t)15;
}
template <typename R>
__host__ __device__ inline size_t ring_slot_elems(int rpl) {
    return (size_t)rpl * (Pair<R>::on ? 2 : 1) * WAVE;
}
// The ring serves FP32 pairs while a slot stays within 4 KiB; FP64 spends
// that LDS on its law tables instead (its prefetch gained nothing measurable).
template <typename R>
__host__ __device__ constexpr bool ring_used(int rpl) {
    // a slot of rpl rows x 2 planes x 64 lanes, filled in 16-byte pieces
    return sizeof(R) == 4 && rpl * 2 * WAVE * sizeof(R) <= 4096 && (rpl * 2) % 4 == 0;
}
// FP64 with 10 or more rows per lane keeps the carried axial fluxes in LDS
// (registers)
template <typename R>
__host__ __device__ constexpr bool fs_in_lds(int rpl) {
    return sizeof(R) == 8 && rpl >= 10;
}
// the ring, or the FP64 carried fluxes, after the tables
template <typename R>
__host__ __device__ inline size_t step_lds_bytes(int L, int np, int rpl = 0) {
    size_t extra = 0;
    if (ring_used<R>(rpl))
        extra = 2 * (size_t)STEP_WAVES * ring_slot_elems<R>(rpl);
    else if (fs_in_lds<R>(rpl))
        extra = (size_t)STEP_WAVES * rpl * WAVE;
    return ring_lds_offset<R>(L, np) + extra * sizeof(R);
}

// Stage the law tables in LDS (dynamic shared memory); all threads call it.
template <typename R>
__device__ inline LawLds<R> stage_laws(const StepArgs<R> &a, unsigned char *smem) {
    const int t = threadIdx.x, nt = blockDim.x, L = a.laws.L, nlaw = 3 * L + 2;
    LawLds<R> v;
    if constexpr (sizeof(R) == 8) {
        double *d = (double *)smem;
        const int nb = (int)pow_blob_doubles(L);
        for (int i = t; i < nb; i += nt) d[i] = a.pow_blob[i];
        v.blk = d;
        v.cka = d + (size_t)nlaw * POW_BLK;
    } else {
        float *f = (float *)smem;
        for (int i = t; i < nlaw; i += nt) {
            f[i] = (float)a.laws.lk[i];
            f[nlaw + i] = (float)a.laws.e[i];
            const bool capl = i >= 2 * L && i < 3 * L;
            f[2 * nlaw + 2 * i] = capl ? (float)a.laws.K[i] : 0.0f;
            f[2 * nlaw + 2 * i + 1] = i == law_unit(L) ? 1.0f : 0.0f;
        }
        v.lk = f;
        v.ex = f + nlaw;
        v.cka = f + 2 * nlaw;
    }
    __syncthreads();
    return v;
}

// Polynomial laws: the stepping kernel's coefficient blob (POLY_BLK doubles
// per law id) staged in LDS in the field's type; all threads call it.
template <typename R>
__device__ inline LawPoly<R> stage_poly(const StepArgs<R> &a, unsigned char *smem) {
    const int n = POLY_BLK * (3 * a.laws.L + 2);
    R *d = (R *)smem;
    for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = (R)a.pow_blob[i];
    __syncthreads();
    return LawPoly<R>{d};
}

}  // namespace cryo
