// gfx950 kernels of the discrete adjoint of one step of eq. (8) (FP64).
//
// A step maps T^n -> T^{n+1}: per interior line j the residual
//   r = A(T^n) T^{n+1} - F(T^n) = 0,
// (rows of eq. (13), (18), (15)), plus the copied or held z-boundary lines.
// With lam^{n+1} = dJ/dT^{n+1} the adjoint step is
//   mu_j   = lam^{n+1}_j (+ the copied boundary line's entries),
//   y_j    = A_j^{-T} mu_j                     (transposed line solve),
//   lam^n  = dJ_n/dT^n - sum over rows of y * (d r / d T^n),
//   dJ/dth -= sum over rows of y * (d r / d theta).
// Pass 1 (k_adj1) does the line solves and the radial part of lam^n; pass 2
// (k_adj2) adds the axial-face part, which couples neighbouring lines: the
// face between lines j and j+1 with flux F = lam_f (T_{j+1} - T_j) adds
// dF/dT_j (y_j - y_{j+1}) to line j and dF/dT_{j+1} (y_j - y_{j+1}) to j+1.
//
// Parameter sensitivities are accumulated per row (radial flux terms y fw Dw
// and y fe De, axial term y (F_N - F_S)) and per heater (y s, y Q ds/dw);
// the host turns the row sums into d/d thickness and d/d k_scale.
//
// The rows are those the stepping kernel solves: each line's rows multiplied
// by row constants (capacity rows by eta^2, interface rows by 1 / lambda of
// the outer layer at the node).  With r' = S r and S independent of T^{n+1},
// y' = S^{-1} y and y' dr'/dT^n = y dr/dT^n wherever r = 0 (the step's
// solution), so lam^n and the row sums (y' fw' = y fw, y' fe' = y fe) are
// those of the rows as written; only the source's derivative carries S.
#include <math.h>
#include <string.h>

#include <type_traits>

#include "device_common.h"

namespace cryo {

constexpr int ADJ_WAVES = 8;

// pass 1 keeps per-row sums in LDS after the law and row tables
__host__ __device__ inline size_t adj_acc_offset(int L, int np) {
    return ring_lds_offset<double>(L, np);
}
__host__ __device__ inline size_t adj_lds_bytes(int L, int np, int rpl) {
    return adj_acc_offset(L, np) + 2 * (size_t)ADJ_WAVES * rpl * WAVE * sizeof(double);
}

// exchange of one value per lane with the neighbouring lanes of the line
// (shuffles inside a wave, LDS across the waves of the line)
template <int G>
__device__ inline void nb_exchange(double v_last, double v_first, double &from_prev,
                                   double &from_next, int lane, int wig, double *xb) {
    from_prev = shfl_up1(v_last, 1, lane);
    from_next = shfl_dn1(v_first, 1, lane);
    if constexpr (G > 1) {
        if (lane == WAVE - 1) xb[2 * wig] = v_last;
        if (lane == 0) xb[2 * wig + 1] = v_first;
        __syncthreads();
        if (lane == 0 && wig > 0) from_prev = xb[2 * (wig - 1)];
        if (lane == WAVE - 1 && wig < G - 1) from_next = xb[2 * (wig + 1) + 1];
        __syncthreads();
    }
}

// Row tables and laws in LDS (dynamic shared memory); all threads call it.
// STEPPED (eq. (9)): the terminal lines' tables too, after the row sums
// (sgw2, sge2, sinf2; the full lines' tables otherwise).
// POLY: the polynomial laws of eqs. (23), (24) (the stepping kernel's
// coefficient blob) instead of the power tables.
template <bool POLY>
struct AdjLds {
    const double *sgw, *sge;
    const uint32_t *sinf;
    const double *sgw2, *sge2;
    const uint32_t *sinf2;
    std::conditional_t<POLY, LawPoly<double>, LawLds<double>> law;
};
template <bool STEPPED, bool POLY = false>
__device__ inline AdjLds<POLY> adj_stage(const StepArgs<double> &a, unsigned char *smem, int rpl) {
    double *sgw = (double *)(smem + ((law_lds_bytes<double>(a.laws.L) + 15) & ~(size_t)15));
    double *sge = sgw + a.np;
    uint32_t *sinf = (uint32_t *)(sge + a.np);
    double *sgw2 = (double *)(smem + adj_lds_bytes(a.laws.L, a.np, rpl));
    double *sge2 = sgw2 + a.np;
    uint32_t *sinf2 = (uint32_t *)(sge2 + a.np);
    for (int i = threadIdx.x; i < a.np; i += blockDim.x) {
        sgw[i] = a.gw[i];
        sge[i] = a.ge[i];
        sinf[i] = a.info[i];
        if constexpr (STEPPED) {
            sgw2[i] = a.gw2[i];
            sge2[i] = a.ge2[i];
            sinf2[i] = a.info2[i];
        }
    }
    AdjLds<POLY> t;
    t.sgw = sgw;
    t.sge = sge;
    t.sinf = sinf;
    t.sgw2 = STEPPED ? sgw2 : sgw;
    t.sge2 = STEPPED ? sge2 : sge;
    t.sinf2 = STEPPED ? sinf2 : sinf;
    if constexpr (POLY) t.law = stage_poly<double>(a, smem);   // ends with a barrier
    else t.law = stage_laws<double>(a, smem);
    return t;
}

// Derivatives of the polynomial laws for the adjoint: the derivative
// polynomial of sum_k c_k x^k (k <= 4), by Horner's rule.
__device__ inline double poly_dlaw(const LawPoly<double> &l, int id, double x) {
    const double *c = l.c + POLY_BLK * id;
    return fma(fma(fma(4.0 * c[4], x, 3.0 * c[3]), x, 2.0 * c[2]), x, c[1]);
}

// lambda'(x) / lambda(x) of a polynomial law (0 for the zero law)
__device__ inline double poly_dlog(const LawPoly<double> &l, int id, double x) {
    const double v = l.lawc(id, x);
    return v != 0.0 ? poly_dlaw(l, id, x) / v : 0.0;
}

// weight of interior line j's outer node in the surface mean (lines
// 0..z_full of a stepped domain)
template <bool STEPPED>
__device__ inline double surf_weight(const StepArgs<double> &a, int j) {
    if constexpr (STEPPED) return j < a.z_full ? a.wz_mid : j == a.z_full ? a.wz_end : 0.0;
    else return a.wz_mid;
}

// Pass 1 of one step over this workgroup's line groups (tables staged).
template <int RPL, int G, bool CUBE, bool STEPPED = false, bool POLY = false>
// (keep: lam^{n+1} of the group's single line comes in lamR, not from memory)
// POLY: the interface row's coefficient is the quotient of its inner (slot 2)
// and outer (slot 3) layer laws, and with the Joule source (eq. (25)) a
// heater row's source is X sqrt(tref / T) at the old T (a.jsq holds
// sqrt(tref)).
__device__ inline void adj1_body(const StepArgs<double> &a, const AdjArgs &d,
                                 unsigned char *smem, const AdjLds<POLY> &tb,
                                 const double (&lamR)[RPL], bool keep) {
    constexpr int NL = WAVE * G, NG = ADJ_WAVES / G;
    __shared__ double xchg[NG][9 * G];
    __shared__ double xb[NG][2 * G];
    const double *sgw = tb.sgw, *sge = tb.sge;       // this line's tables
    const uint32_t *sinf = tb.sinf;
    const auto &law = tb.law;
    const int lane = threadIdx.x & (WAVE - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int grp = wv / G, wig = wv % G, lg = wig * WAVE + lane;
    const int gidx = blockIdx.x * NG + grp;                  // line group
    const int j0 = 1 + gidx * a.lpw;
    const int j1 = min(j0 + a.lpw, a.nz - 1);
    const size_t LS = a.np;
    const int qW = lg > 0 ? (RPL - 1) * NL + lg - 1 : 0;
    const int qE = lg < NL - 1 ? lg + 1 : (RPL - 1) * NL + lg;
    const double cS = d.cS ? *d.cS : 0.0;                    // dJ/dS of this state
    // per-row sums over the group's lines, in LDS (registers): [wave][row][lane]
    double *accW = (double *)(smem + adj_acc_offset(a.laws.L, a.np)) + (size_t)wv * RPL * WAVE + lane;
    double *accE = accW + (size_t)ADJ_WAVES * RPL * WAVE;
    double gS = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) accW[r * WAVE] = accE[r * WAVE] = 0.0;
    for (int it = 0; it < a.lpw; ++it) {
        const int jr = j0 + it;
        const bool active = jr < j1;
        const int j = min(jr, a.nz - 2);
        const size_t base = (size_t)j * LS;
        if constexpr (STEPPED) {                      // the terminal's lines
            const bool up = j > a.z_full;
            sgw = up ? tb.sgw2 : tb.sgw;
            sge = up ? tb.sge2 : tb.sge;
            sinf = up ? tb.sinf2 : tb.sinf;
        }
        double T[RPL], MU[RPL], fw[RPL], fe[RPL];
        // the line's loads up front (latency overlaps the row work)
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int q = r * NL + lg;
            T[r] = d.T[base + q];
            MU[r] = keep ? lamR[r] : d.lam_in[base + q];
        }
        // boundary-copy lines feed their sensitivity back to the copied line
        if (j == 1 && !a.held[2]) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) MU[r] += d.lam_in[r * NL + lg];
        }
        if (j == a.nz - 2 && !a.held[3]) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) MU[r] += d.lam_in[(size_t)(a.nz - 1) * LS + r * NL + lg];
        }
        const double TwF = d.T[base + qW], TeL = d.T[base + qE];
        // west face of the chunk's first row
        double lamW = law.lawc((sinf[qW] >> 6) & 63, 0.5 * (TwF + T[0]));
        double a0 = 0, b0 = 1, c0 = 0, d0 = 0, ccm2 = 0, bbm1 = 1, ccm1 = 0, mum1 = 0;
        double al[RPL], ga[RPL], de[RPL];
        double aa0 = 0, ccL = 0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int q = r * NL + lg;
            const uint32_t inf_r = sinf[q];
            const uint32_t kind = inf_r & 7;
            const bool cap = kind == K_CAP, ifc = kind == K_IFACE;
            const double t = T[r], Te = (r < RPL - 1) ? T[r + 1] : TeL;
            const int le = (inf_r >> 6) & 63, l2 = (inf_r >> 12) & 63;
            const int lc = (inf_r >> 24) & 63;
            const double lamE = law.lawc(le, 0.5 * (t + Te));
            // rows in the stepping kernel's scaled form: an interface row's
            // west coefficient is the ratio law at the node and its east one
            // h_i; boundary rows have their unit or zero laws folded into gw,
            // ge (slot 2 is the unit law there, the zero law on padding)
            double l2v = l2 == law_unit(a.laws.L) ? 1.0 : 0.0;
            if (__any(ifc)) {
                double va = law.lawc(l2, t);
                if constexpr (POLY) va = va / law.lawc((inf_r >> 18) & 63, t);
                if (ifc) l2v = va;
            }
            double rc;
            if constexpr (CUBE) rc = law.cube(lc, t);
            else rc = law.lawc(lc, t);
            fw[r] = sgw[q] * (cap ? lamW : l2v);
            fe[r] = sge[q] * (cap ? lamE : 1.0);
            const double aa = -fw[r], bb = fw[r] + fe[r] + rc, cc = -fe[r];
            const double mu = MU[r];
            // transposed row r-1 = (cc_{r-2}, bb_{r-1}, aa_r | mu_{r-1})
            if (r == 0) {
                aa0 = aa;
                b0 = bb;
                d0 = mu;
            } else if (r == 1) {
                c0 = aa;          // sup of the first transposed row
            } else {
                elim_row<double, RPL>(r - 1, ccm2, bbm1, aa, mum1, al, ga, de);
                // eliminate here rather than at the solve (register pressure)
                asm volatile("" : "+v"(al[r - 1]), "+v"(ga[r - 1]), "+v"(de[r - 1]));
            }
            ccm2 = ccm1;
            ccm1 = cc;
            bbm1 = bb;
            mum1 = mu;
            if (r == RPL - 1) ccL = cc;
            lamW = lamE;
            __builtin_amdgcn_sched_barrier(0);
        }
        // chunk ends: sub of the first row = cc of the previous row, sup of the
        // last row = aa of the next row
        double ccPrev, aaNext;
        nb_exchange<G>(ccL, aa0, ccPrev, aaNext, lane, wig, xb[grp]);
        a0 = ccPrev;
        if (RPL == 2) {
            // the first row's sup is the second row's aa, already in c0
        }
        elim_row<double, RPL>(RPL - 1, ccm2, bbm1, aaNext, mum1, al, ga, de);
        double y[RPL];
        solve_tail<double, RPL, G>(a0, b0, c0, d0, al, ga, de, y, lane, wig, xchg[grp]);
        // T^{n+1} of the line, loaded after the solve (registers)
        double X[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) X[r] = d.X[base + r * NL + lg];
        const double XwF = d.X[base + qW], XeL = d.X[base + qE];
        // radial part of lam^n:  dJ - [y_i dr_i/dT_i + y_{i-1} dr_{i-1}/dT_i + y_{i+1} dr_{i+1}/dT_i]
        // face conductivity derivatives: d(gw lam_W)/dT_i = (1/2) e lam' ... on
        // capacity rows (face-mean argument), e lam / T at interface nodes.
        // Row r's factors: Dw, De (differences of T^{n+1}), fwT, feT; ie is
        // 1/2 e / (face mean) of the east face, carried as the next row's west.
        auto factors = [&](int r, double ieW, double &Dw, double &De, double &fwT, double &feT,
                           double &ieE) {
            const int q = r * NL + lg;
            const double xw = (r > 0) ? X[r - 1] : XwF, xe = (r < RPL - 1) ? X[r + 1] : XeL;
            Dw = X[r] - xw;
            De = X[r] - xe;
            const uint32_t inf_r = sinf[q];
            const uint32_t kind = inf_r & 7;
            const double t = T[r], Te = (r < RPL - 1) ? T[r + 1] : TeL;
            const bool cap = kind == K_CAP, ifc = kind == K_IFACE;
            if constexpr (POLY) {
                // the scaled interface row's west coefficient is the quotient
                // lambda_a / lambda_b at the node; its east one is constant
                ieE = 0.5 * poly_dlog(law, (inf_r >> 6) & 63, 0.5 * (t + Te));
                const double dq = ifc ? poly_dlog(law, (inf_r >> 12) & 63, t) -
                                            poly_dlog(law, (inf_r >> 18) & 63, t)
                                      : 0.0;
                fwT = cap ? fw[r] * ieW : ifc ? fw[r] * dq : 0.0;
                feT = cap ? fe[r] * ieE : 0.0;
            } else {
                ieE = 0.5 * law.expo((inf_r >> 6) & 63) * rcp(0.5 * (t + Te));
                const double it = rcp(t);
                fwT = cap ? fw[r] * ieW : ifc ? fw[r] * law.expo((inf_r >> 12) & 63) * it : 0.0;
                feT = cap ? fe[r] * ieE : ifc ? fe[r] * law.expo((inf_r >> 18) & 63) * it : 0.0;
            }
        };
        double ieW0;               // 1/2 e_W / tf_W of row 0 (west face of the chunk)
        {
            const uint32_t iw = sinf[qW];
            if constexpr (POLY) ieW0 = 0.5 * poly_dlog(law, (iw >> 6) & 63, 0.5 * (TwF + T[0]));
            else ieW0 = 0.5 * law.expo((iw >> 6) & 63) * rcp(0.5 * (TwF + T[0]));
        }
        // coupling terms leaving the chunk towards the neighbouring lanes'
        // rows (capacity rows: the face conductivity depends on both nodes)
        double qwF, qeL;
        {
            double Dw, De, fwT, feT, ie;
            factors(0, ieW0, Dw, De, fwT, feT, ie);
            qwF = (sinf[lg] & 7) == K_CAP ? y[0] * fwT * Dw : 0.0;            // to row i0-1
            const uint32_t il = sinf[(RPL - 2) * NL + lg];
            const double TL = T[RPL - 2];
            double ieL = ieW0;
            if constexpr (POLY) {
                if (RPL >= 2) ieL = 0.5 * poly_dlog(law, (il >> 6) & 63, 0.5 * (TL + T[RPL - 1]));
            } else {
                if (RPL >= 2) ieL = 0.5 * law.expo((il >> 6) & 63) * rcp(0.5 * (TL + T[RPL - 1]));
            }
            factors(RPL - 1, RPL >= 2 ? ieL : ieW0, Dw, De, fwT, feT, ie);
            qeL = (sinf[(RPL - 1) * NL + lg] & 7) == K_CAP ? y[RPL - 1] * feT * De : 0.0;
        }
        double qePrev, qwNext;
        nb_exchange<G>(qeL, qwF, qePrev, qwNext, lane, wig, xb[grp]);
        if (active) {
            // one pass over the rows: row r's coupling into row r-1 completes
            // row r-1, which is stored one row late
            double ieW = ieW0, oe_prev = qePrev, lp_prev = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int q = r * NL + lg;
                const uint32_t inf_r = sinf[q];
                const uint32_t kind = inf_r & 7;
                const bool cap = kind == K_CAP, ifc = kind == K_IFACE;
                double Dw, De, fwT, feT, ieE;
                factors(r, ieW, Dw, De, fwT, feT, ieE);
                ieW = ieE;
                const double t = T[r];
                const int lc = (inf_r >> 24) & 63;
                double rc, drc;
                if constexpr (POLY) {
                    rc = law.lawc(lc, t);
                    drc = poly_dlaw(law, lc, t);
                } else if constexpr (CUBE) {
                    rc = law.cube(lc, t);
                    drc = 3.0 * law.cka[2 * lc] * t * t;
                } else {
                    rc = law.lawc(lc, t);
                    drc = law.expo(lc) * rc * rcp(t);
                }
                const bool cf = cap || ifc;
                double self = cf ? fwT * Dw + feT * De + drc * (X[r] - t) - rc : 0.0;
                // the Joule source X sqrt(tref / T): d(-source)/dT = source / (2 T)
                double chi = 1.0;
                if constexpr (POLY) {
                    if (a.joule && ((inf_r >> 3) & 1)) {
                        chi = a.jsq * rsqrt(t);
                        self += 0.5 * a.pulse.amplitude * d.s * chi * rcp(t);
                    }
                }
                const double ow = cap ? y[r] * fwT * Dw : 0.0;       // into row r-1
                const double oe = cap ? y[r] * feT * De : 0.0;       // into row r+1
                double lp = -(y[r] * self + oe_prev);
                if (lg == a.surf_lane && r == a.surf_reg) lp += cS * surf_weight<STEPPED>(a, j);
                if (r > 0) d.lpart[base + q - NL] = lp_prev - ow;
                d.Y[base + q] = y[r];
                oe_prev = oe;
                lp_prev = lp;
                // (unconditional: a read under a row test is a branch that
                // waits for it at once)
                const double aw = accW[r * WAVE], ae = accE[r * WAVE];
                accW[r * WAVE] = cf ? fma(y[r] * fw[r], Dw, aw) : aw;
                accE[r * WAVE] = cf ? fma(y[r] * fe[r], De, ae) : ae;
                gS += ((inf_r >> 3) & 1) ? (POLY ? y[r] * chi : y[r]) : 0.0;
                __builtin_amdgcn_sched_barrier(0);
            }
            d.lpart[base + (RPL - 1) * NL + lg] = lp_prev - qwNext;
        }
    }
    // heater sums: lane-order tree inside each wave
    double v = gS;
    for (int s = WAVE / 2; s >= 1; s >>= 1) v += __shfl_down(v, s, WAVE);
    __shared__ double gsum[ADJ_WAVES];
    if (lane == 0) gsum[wv] = v;
    __syncthreads();
    // this workgroup's running sums (one slot per workgroup: no other writer),
    // its line groups added in a fixed order
    const double *accL = (const double *)(smem + adj_acc_offset(a.laws.L, a.np));
    double *acc = d.acc + (size_t)blockIdx.x * 3 * a.np;
    for (int q = threadIdx.x; q < a.np; q += blockDim.x) {
        const int r = q / NL, lq = q % NL, w0 = lq / WAVE, ln = lq % WAVE;
        double sw = 0.0, se = 0.0;
        for (int g = 0; g < NG; ++g) {
            const size_t o = (size_t)(g * G + w0) * RPL * WAVE + (size_t)r * WAVE + ln;
            sw += accL[o];
            se += accL[(size_t)ADJ_WAVES * RPL * WAVE + o];
        }
        acc[q] += sw;
        acc[a.np + q] += se;
    }
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < ADJ_WAVES; ++w) tot += gsum[w];
        d.accg[2 * blockIdx.x] += tot * d.xs * d.s;
        d.accg[2 * blockIdx.x + 1] += tot * a.pulse.amplitude * d.ds;
    }
}

template <int RPL, int G, bool CUBE, bool STEPPED, bool POLY = false>
__global__ __launch_bounds__(ADJ_WAVES *WAVE) void k_adj1(StepArgs<double> a, AdjArgs d) {
    extern __shared__ __align__(16) unsigned char smem[];
    const AdjLds<POLY> tb = adj_stage<STEPPED, POLY>(a, smem, RPL);
    const double none[RPL] = {};
    adj1_body<RPL, G, CUBE, STEPPED, POLY>(a, d, smem, tb, none, false);
}

// Pass 2: axial faces.  Each interior line j adds the terms of its two
// axial faces (capacity rows), and the lines next to the z-boundaries write
// the boundary lines' lam^n.
template <int RPL, int G, bool STEPPED = false, bool POLY = false>
// (keep: lam^n of the group's single line goes to lamR, not to memory; the
// boundary lines' lam^n is always written)
__device__ inline void adj2_body(const StepArgs<double> &a, const AdjArgs &d,
                                 unsigned char *smem, const AdjLds<POLY> &tb,
                                 double (&lamR)[RPL], bool keep) {
    constexpr int NL = WAVE * G, NG = ADJ_WAVES / G;
    const uint32_t *sinf = tb.sinf;                      // this line's table
    const auto &law = tb.law;
    const int lane = threadIdx.x & (WAVE - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int grp = wv / G, wig = wv % G, lg = wig * WAVE + lane;
    const int gidx = blockIdx.x * NG + grp;
    const int j0 = 1 + gidx * a.lpw;
    const int j1 = min(j0 + a.lpw, a.nz - 1);
    const size_t LS = a.np;
    const double cS = d.cS ? *d.cS : 0.0;                    // dJ/dS of this state
    double accZ[RPL];
    // carried from the previous line of the group: the face (j-1, j) flux
    // F = lam (T_j - T_{j-1}) and dF/dT_j; and the lines j, j-1 (T, Y)
    double cF[RPL], cdF[RPL], Tc[RPL], Yc[RPL], Ys[RPL];
    // groups past the last line read line nz-2 and do no line
    const int jb = min(j0, a.nz - 2);
    const size_t bb = (size_t)jb * LS;
    if constexpr (STEPPED) sinf = jb > a.z_full ? tb.sinf2 : tb.sinf;
    // start-up: the south faces (jb-1, jb) of the group's first line, and for
    // line 1 the lower boundary line's lam^n (that face's dF/dT_0)
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int q = r * NL + lg;
        const uint32_t inf_r = sinf[q];
        const bool cap = (inf_r & 7) == K_CAP;
        const int lz = cap ? (inf_r >> 12) & 63 : law_zero(a.laws.L);
        const double t = d.T[bb + q], ts = d.T[bb - LS + q];
        const double y = d.Y[bb + q];
        const double fs = 0.5 * (t + ts);
        const double ls = law.lawc(lz, fs), ds = t - ts;
        double gs;
        if constexpr (POLY) gs = 0.5 * poly_dlaw(law, lz, fs);
        else gs = 0.5 * law.expo(lz) * ls * rcp(fs);
        accZ[r] = 0.0;
        cF[r] = ls * ds;
        cdF[r] = gs * ds + ls;                                 // d F_S / d T_j
        Tc[r] = t;
        Yc[r] = y;
        Ys[r] = jb - 1 >= 1 ? d.Y[bb - LS + q] : 0.0;
        if (j0 == 1 && j0 < j1) {
            double l0 = (gs * ds - ls) * (0.0 - y);            // d F_S / d T_0
            if (lg == a.surf_lane && r == a.surf_reg) l0 += cS * a.wz_end;
            d.lam_out[q] = l0;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int j = j0; j < j1; ++j) {
        const size_t base = (size_t)j * LS;
        if constexpr (STEPPED) sinf = j > a.z_full ? tb.sinf2 : tb.sinf;
        // the line above and this line's partial lam^n, up front
        double Tn[RPL], Yn[RPL], LP[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int q = r * NL + lg;
            Tn[r] = d.T[base + LS + q];
            Yn[r] = (j + 1 <= a.nz - 2) ? d.Y[base + LS + q] : 0.0;
            LP[r] = d.lpart[base + q];
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int q = r * NL + lg;
            const uint32_t inf_r = sinf[q];
            bool cap = (inf_r & 7) == K_CAP;
            // the step face (eq. (9)): closed where the terminal's row above
            // is not a capacity row
            if constexpr (STEPPED)
                if (j == a.z_full && (tb.sinf2[q] & 7) != K_CAP) cap = false;
            // non-capacity rows take the zero law: every face term vanishes
            const int lz = cap ? (inf_r >> 12) & 63 : law_zero(a.laws.L);
            const double t = Tc[r], tn = Tn[r];
            const double y = Yc[r], yn = Yn[r], ys = Ys[r];
            // north face (j, j+1); the south face (j-1, j) is carried
            const double fn = 0.5 * (t + tn);
            const double ln = law.lawc(lz, fn);
            const double dn = tn - t;
            double gn;
            if constexpr (POLY) gn = 0.5 * poly_dlaw(law, lz, fn);
            else gn = 0.5 * law.expo(lz) * ln * rcp(fn);
            const double dFlN = gn * dn - ln;                       // d F_N / d T_j
            const double lam = LP[r] + dFlN * (y - yn) + cdF[r] * (ys - y);
            accZ[r] += y * (ln * dn - cF[r]);
            cF[r] = ln * dn;
            cdF[r] = gn * dn + ln;                                  // d F_N / d T_{j+1}
            if (j == a.nz - 2) {
                // the upper boundary line: its face with line nz-2
                double le_ = cdF[r] * (y - 0.0);                    // d F_N / d T_{nz-1}
                // (on a stepped domain the top line is not on the surface)
                if (!STEPPED && lg == a.surf_lane && r == a.surf_reg) le_ += cS * a.wz_end;
                d.lam_out[(size_t)(a.nz - 1) * LS + q] = le_;
            }
            if (keep) lamR[r] = lam;
            else d.lam_out[base + q] = lam;
            // one row at a time (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            Ys[r] = Yc[r];
            Yc[r] = Yn[r];
            Tc[r] = Tn[r];
        }
    }
    // this workgroup's sums, its line groups added in a fixed order
    double *accL = (double *)(smem + adj_acc_offset(a.laws.L, a.np));
#pragma unroll
    for (int r = 0; r < RPL; ++r) accL[(size_t)wv * RPL * WAVE + r * WAVE + lane] = accZ[r];
    __syncthreads();
    double *acc = d.acc + (size_t)blockIdx.x * 3 * a.np + 2 * a.np;
    for (int q = threadIdx.x; q < a.np; q += blockDim.x) {
        const int r = q / NL, lq = q % NL, w0 = lq / WAVE, ln = lq % WAVE;
        double sz = 0.0;
        for (int g = 0; g < NG; ++g)
            sz += accL[(size_t)(g * G + w0) * RPL * WAVE + (size_t)r * WAVE + ln];
        acc[q] += sz;
    }
}

template <int RPL, int G, bool STEPPED, bool POLY = false>
__global__ __launch_bounds__(ADJ_WAVES *WAVE) void k_adj2(StepArgs<double> a, AdjArgs d) {
    extern __shared__ __align__(16) unsigned char smem[];
    const AdjLds<POLY> tb = adj_stage<STEPPED, POLY>(a, smem, RPL);
    double lamR[RPL];
    adj2_body<RPL, G, STEPPED, POLY>(a, d, smem, tb, lamR, false);
}

// Pass 2 of step k and pass 1 of step k - 1 in one launch: each line group
// finishes lam^k of its lines (in registers for one line per group, else
// written to memory and read back by the same lanes), then runs the next
// step's line solves on it.  Every value that
// crosses line groups (y^k of the neighbouring lines) is read in the first
// phase and written only to the other buffer in the second.
template <int RPL, int G, bool CUBE, bool KEEP, bool STEPPED, bool POLY = false>
__global__ __launch_bounds__(ADJ_WAVES *WAVE) void k_adj21(StepArgs<double> a, AdjArgs d2,
                                                           AdjArgs d1) {
    extern __shared__ __align__(16) unsigned char smem[];
    const AdjLds<POLY> tb = adj_stage<STEPPED, POLY>(a, smem, RPL);
    // one line per group: lam^k stays in registers between the phases (no
    // other group reads it)
    double lamR[RPL] = {};
    adj2_body<RPL, G, STEPPED, POLY>(a, d2, smem, tb, lamR, KEEP);
    __syncthreads();           // the LDS row sums area passes to the next phase
    adj1_body<RPL, G, CUBE, STEPPED, POLY>(a, d1, smem, tb, lamR, KEEP);
}

// lam^N = dJ_N / dT^N: the surface weights on the outer row
__global__ void k_adj_init(double *lam, int nz, int np, int q_surf, const double *cSp,
                           double wz_end, double wz_mid, int J) {
    const double cS = *cSp;
    size_t n = (size_t)nz * np;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(idx / np), q = (int)(idx % np);
        double v = 0.0;
        // the surface mean's lines 0..J (nz - 1, or a stepped domain's z_full)
        if (q == q_surf && j <= J) v = cS * ((j == 0 || j == J) ? wz_end : wz_mid);
        lam[idx] = v;
    }
}

__global__ void k_zero(double *p, size_t n) {
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * blockDim.x)
        p[idx] = 0.0;
}

static cryo_status check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CRYO_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return CRYO_OK;
}

int adj_grid(const cryo_plan *p) {
    const int groups = (p->nz - 2 + p->lpw - 1) / p->lpw;
    const int per_wg = ADJ_WAVES / p->wpl;
    return (groups + per_wg - 1) / per_wg;
}

// row-sum slots: one per workgroup of the adjoint passes
int adj_slots(const cryo_plan *p) { return adj_grid(p); }

// dynamic LDS of the adjoint passes (a stepped domain adds the terminal's
// tables)
size_t adj_lds(const cryo_plan *p) {
    return adj_lds_bytes(p->L, p->np, p->rpl) + (p->stepped ? step_tables_bytes<double>(p->np) : 0);
}

StepArgs<double> step_args_f64(const cryo_plan *p, int *flag);

// one pass (1, 2, or 21: pass 2 of step k with d, pass 1 of step k-1 with
// d1) of one adjoint shape
template <int R_, int G_, bool ST>
static void adj_launch_poly(int pass, bool keep, dim3 g, dim3 b, size_t lds, hipStream_t s,
                            const StepArgs<double> &a, const AdjArgs &d, const AdjArgs *d1) {
    if (pass == 2) hipLaunchKernelGGL((k_adj2<R_, G_, ST, true>), g, b, lds, s, a, d);
    else if (pass == 21 && keep)
        hipLaunchKernelGGL((k_adj21<R_, G_, false, true, ST, true>), g, b, lds, s, a, d, *d1);
    else if (pass == 21)
        hipLaunchKernelGGL((k_adj21<R_, G_, false, false, ST, true>), g, b, lds, s, a, d, *d1);
    else hipLaunchKernelGGL((k_adj1<R_, G_, false, ST, true>), g, b, lds, s, a, d);
}

template <int R_, int G_, bool ST>
static void adj_launch(int pass, bool cube, bool keep, dim3 g, dim3 b, size_t lds, hipStream_t s,
                       const StepArgs<double> &a, const AdjArgs &d, const AdjArgs *d1) {
    if (pass == 2) hipLaunchKernelGGL((k_adj2<R_, G_, ST>), g, b, lds, s, a, d);
    else if (pass == 21 && cube && keep)
        hipLaunchKernelGGL((k_adj21<R_, G_, true, true, ST>), g, b, lds, s, a, d, *d1);
    else if (pass == 21 && cube)
        hipLaunchKernelGGL((k_adj21<R_, G_, true, false, ST>), g, b, lds, s, a, d, *d1);
    else if (pass == 21 && keep)
        hipLaunchKernelGGL((k_adj21<R_, G_, false, true, ST>), g, b, lds, s, a, d, *d1);
    else if (pass == 21)
        hipLaunchKernelGGL((k_adj21<R_, G_, false, false, ST>), g, b, lds, s, a, d, *d1);
    else if (cube) hipLaunchKernelGGL((k_adj1<R_, G_, true, ST>), g, b, lds, s, a, d);
    else hipLaunchKernelGGL((k_adj1<R_, G_, false, ST>), g, b, lds, s, a, d);
}

// pass 1, pass 2, or (pass 21) pass 2 of step k with d and pass 1 of step k-1
// with d1
cryo_status launch_adj(const cryo_plan *p, int pass, const AdjArgs &d, int *flag, hipStream_t s,
                       const AdjArgs *d1) {
    StepArgs<double> a = step_args_f64(p, flag);
    dim3 g(adj_grid(p)), b(ADJ_WAVES * WAVE);
    const size_t lds = adj_lds(p);
    const int key = p->rpl * 10 + p->wpl;
    if (pass == 21 && !d1) return fail(CRYO_ERR_ARG, "fused adjoint passes need two steps");
    const bool cube = a.laws.cube, keep = a.lpw == 1;
#define ADJ_CASE(R_, G_)                                                                    \
    case R_ * 10 + G_:                                                                      \
        if (p->poly && p->stepped)                                                          \
            adj_launch_poly<R_, G_, true>(pass, keep, g, b, lds, s, a, d, d1);              \
        else if (p->poly) adj_launch_poly<R_, G_, false>(pass, keep, g, b, lds, s, a, d, d1); \
        else if (p->stepped) adj_launch<R_, G_, true>(pass, cube, keep, g, b, lds, s, a, d, d1); \
        else adj_launch<R_, G_, false>(pass, cube, keep, g, b, lds, s, a, d, d1);             \
        break;
    switch (key) {
        ADJ_CASE(2, 1)
        ADJ_CASE(4, 1)
        ADJ_CASE(8, 1)
        ADJ_CASE(8, 2)
        ADJ_CASE(8, 4)
        ADJ_CASE(4, 2)
        ADJ_CASE(4, 4)
    default: return fail(CRYO_ERR_UNSUPPORTED, "radial chunk shape");
    }
#undef ADJ_CASE
    return check_launch(pass == 1 ? "adjoint pass 1" : pass == 2 ? "adjoint pass 2"
                                                                  : "adjoint passes 2+1");
}

cryo_status launch_adj_init(const cryo_plan *p, double *lam, const double *cS, hipStream_t s) {
    const int q = p->surf_reg * (WAVE * p->wpl) + p->surf_lane;
    size_t n = (size_t)p->nz * p->np;
    int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
    const int J = p->stepped ? p->z_full : p->nz - 1;
    hipLaunchKernelGGL(k_adj_init, dim3(blocks), dim3(256), 0, s, lam, p->nz, p->np, q, cS,
                       0.5 / J, 1.0 / J, J);
    return check_launch("adjoint init");
}

cryo_status launch_zero(double *ptr, size_t n, hipStream_t s) {
    int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, ptr, n);
    return check_launch("zero");
}

}  // namespace cryo
