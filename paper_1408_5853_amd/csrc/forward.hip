// gfx950 kernels of one explicit-implicit step (eq. (8)) and the layout
// conversions around it.
//
// Layout.  Inside the library a field is [nz][np] with np = 64 * rpl and each
// line stored lane-major: row i = lane * rpl + reg lives at reg * 64 + lane.
// One wave (64 lanes) owns one radial line; lane k owns the contiguous rows
// k*rpl .. k*rpl+rpl-1, so every load and store of a line is coalesced and
// the r-neighbours across chunk ends come from the adjacent lane.
//
// Step (delta form).  For the line j each row gets coefficients from the old
// field (eq. (13) capacity rows, eq. (18) interface rows, eq. (15) or held
// boundary rows) and the right-hand side is the explicit residual, so the
// unknown is the increment dT = T^ - T:
//   A dT_{i-1} + B dT_i + C dT_{i+1} = Lambda_i[T] + Lambda_j[T] + X.
// The rows are solved in scaled form (same solution): capacity rows times
// eta^2, so the axial faces take the radial law, and interface rows divided
// by the outer layer's law at the node, so they need one ratio law; the
// plan's forward tables (fgw, fge, finfo, flaws) hold that form.
// The tridiagonal system is solved by partition: every lane eliminates its
// chunk down to two unknowns (first and last row), the 128 chunk-end unknowns
// are reduced to one per lane, and parallel cyclic reduction across the wave
// solves those; lanes then back-substitute their chunk.
#include <math.h>
#include <string.h>

#include "device_common.h"

namespace cryo {

// One step of eq. (8).  A line is spread over G waves (NL = 64 G lanes, each
// lane a chunk of RPL rows); a workgroup of STEP_WAVES waves runs
// STEP_WAVES / G lines side by side.  Each line group marches through a
// block of lpw consecutive interior lines (up or down), keeping the flux
// through the face between the current and the next line: the flux into
// line j from line j+1 is minus the flux into line j+1 from line j (eq. (11)),
// so a capacity row evaluates two conductivities per line (east r-face, the
// face towards the next line) instead of three.
// CUBE: every capacity law has exponent 3 (c(T) by multiplication).
// POLY: polynomial laws (eqs. (23), (24)), interface rows as the quotient
// of two laws, and the optional Joule source (eq. (25)).
template <typename R, bool POLY>
__device__ inline auto stage_law_of(const StepArgs<R> &a, unsigned char *smem) {
    if constexpr (POLY) return stage_poly<R>(a, smem);
    else return stage_laws<R>(a, smem);
}

// STEPPED: the stepped domain of eq. (9).  Lines above z_full use the
// terminal's row tables (rows past its wall are identity rows), the axial
// face between lines z_full and z_full + 1 is closed where the terminal's row
// is not a capacity row, the held outer wall belongs to the layered lines,
// and the surface mean covers lines 0..z_full.
template <typename R, int RPL, int G, bool CUBE, bool POLY = false, bool STEPPED = false>
__device__ inline void step_body(const StepArgs<R> &a, const int blk, const R *__restrict__ Tin,
                                 R *__restrict__ Tout, const R X, double *partial) {
    constexpr bool PAIR = Pair<R>::on;
    constexpr int NPL = PAIR ? 2 : 1;                 // planes per line (pairs: hi, lo)
    constexpr int NL = WAVE * G;                      // lanes per line
    constexpr int NG = STEP_WAVES / G;                // lines per workgroup
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double wsum[STEP_WAVES];
    __shared__ R xchg[NG][9 * G];
    // per-row tables of the line (shared by every line) after the law tables
    R *sgw = (R *)(smem + ((law_lds_bytes<R>(a.laws.L) + 15) & ~(size_t)15));
    R *sge = sgw + a.np;
    uint32_t *sinf = (uint32_t *)(sge + a.np);
    // STEPPED: the terminal's tables next, where the ring or carried fluxes
    // would otherwise start (those move up by tbytes)
    const size_t tbytes = STEPPED ? step_tables_bytes<R>(a.np) : 0;
    R *sgw2 = (R *)(smem + ring_lds_offset<R>(a.laws.L, a.np));
    R *sge2 = sgw2 + a.np;
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
    const auto law = stage_law_of<R, POLY>(a, smem);   // ends with a barrier
    const int t = threadIdx.x;
    // the wave index is uniform: line indices and bases live in scalar registers
    const int lane = t & (WAVE - 1), wv = __builtin_amdgcn_readfirstlane(t / WAVE);
    const int grp = wv / G, wig = wv % G, lg = wig * WAVE + lane;
    const int L = a.laws.L;
    const int j0 = 1 + (blk * NG + grp) * a.lpw;
    const int j1 = min(j0 + a.lpw, a.nz - 1);             // exclusive
    // Line order: even line groups march up, odd ones down, so that the
    // halo line two neighbouring groups share is read by both at about the
    // same time (both at their start or both at their end) and stays in L2.
    // The LDS line ring marches up only.  dir is uniform.
    constexpr bool RING_ = ring_used<R>(RPL);
    const int dir = (!RING_ && ((blk * NG + grp) & 1)) ? -1 : 1;
    // line of iteration it, clamped: active iterations first (it < j1 - j0),
    // then inactive ones on real lines (results discarded)
    auto line_at = [&](int it) {
        const int jr = dir > 0 ? j0 + it : j1 - 1 - it;
        return min(max(jr, 1), a.nz - 2);
    };
    const size_t LS = (size_t)a.np * NPL;                 // line stride
    const size_t LO = PAIR ? (size_t)a.np : 0;            // offset of the low plane
    R *xch = xchg[grp];
    // neighbour rows across the chunk ends (the row itself at the line ends)
    const int qW = lg > 0 ? (RPL - 1) * NL + lg - 1 : 0;
    const int qE = lg < NL - 1 ? lg + 1 : (RPL - 1) * NL + lg;
    double sv = 0.0;
    int bad = 0;
    // Line ring (FP32 pairs, ring_used): two LDS slots per wave hold the wave's
    // part of the next line and of the line after it, loaded straight from
    // memory into LDS (no registers in flight) one iteration ahead.  Slot
    // layout: element (row r, plane p, lane) at (r NPL + p) WAVE + lane.  Other
    // cases read the next line from memory directly.  Groups past the last
    // line march on clamped line indices (real lines, results discarded).
    constexpr int SLOT = RPL * NPL * WAVE;
    constexpr bool RING = ring_used<R>(RPL);
    constexpr int EPL = 16 / (int)sizeof(R);              // elements per lane per load
    constexpr int LPS = WAVE / EPL;                       // lanes per row-plane
    R *ring = (R *)(smem + ring_lds_offset<R>(L, a.np) + tbytes) + (size_t)wv * 2 * SLOT;
    auto prefetch = [&](int slot, size_t lbase) {
        if constexpr (!RING) return;
        R *dst = ring + slot * SLOT;
        const int sub = lane / LPS, e0 = EPL * (lane % LPS);
#pragma unroll
        for (int i = 0; i < RPL * NPL / EPL; ++i) {
            const int rp = i * EPL + sub;                 // row-plane of this lane
            const R *src = Tin + lbase + (size_t)(rp % NPL) * LO + (size_t)(rp / NPL) * NL +
                           wig * WAVE + e0;
            __builtin_amdgcn_global_load_lds((const void *)src,
                                             (__attribute__((address_space(3))) void *)(dst + i * EPL * WAVE),
                                             16, 0, 0);
        }
    };
    // carried south-face fluxes: registers, or (FP64, 10+ rows per lane) LDS
    constexpr bool FS_LDS = fs_in_lds<R>(RPL);
    R FSr[FS_LDS ? 1 : RPL];
    R *fsl = (R *)(smem + ring_lds_offset<R>(L, a.np) + tbytes) + (size_t)wv * RPL * WAVE + lane;
    auto fs_get = [&](int r) -> R {
        if constexpr (FS_LDS) return fsl[r * WAVE];
        else return FSr[r];
    };
    auto fs_set = [&](int r, R v) {
        if constexpr (FS_LDS) fsl[r * WAVE] = v;
        else FSr[r] = v;
    };
    R Tc[RPL], Lc[RPL];
    R TwF, TeL, LwF = 0, LeL = 0;
    {
        const int jb = line_at(0);
        const size_t bc = (size_t)jb * LS;
        const size_t bp = (size_t)(jb - dir) * LS;       // the line before it
        const uint32_t *tinf = (STEPPED && jb > a.z_full) ? sinf2 : sinf;
        const bool trans = STEPPED && min(jb, jb - dir) == a.z_full;
        prefetch(1, bc + LS);
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int q = r * NL + lg;
            Tc[r] = Tin[bc + q];
            Lc[r] = PAIR ? Tin[bc + LO + q] : (R)0;
        }
        TwF = Tin[bc + qW];
        TeL = Tin[bc + qE];
        if constexpr (PAIR) {
            LwF = Tin[bc + LO + qW];
            LeL = Tin[bc + LO + qE];
        }
        // axial flux into the block's first line from the line before it
        // (capacity rows); that line is loaded up front
        R Tpv[RPL], Tplv[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            Tpv[r] = Tin[bp + r * NL + lg];
            Tplv[r] = PAIR ? Tin[bp + LO + r * NL + lg] : (R)0;
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int q = r * NL + lg;
            const R Tp = Tpv[r], Tpl = Tplv[r];
            const uint32_t inf_r = tinf[q];
            const bool cap = (inf_r & 7) == K_CAP;
            const int l2 = (inf_r >> 12) & 63;
            if constexpr (!PAIR) bad |= !LawLds<R>::in_range(Tp);
            const R lamS = law.lawm(cap ? l2 : law_zero(L), Tc[r] + Tp);
            R Fs = lamS * dif<R>(Tp, Tpl, Tc[r], Lc[r]);
            if constexpr (STEPPED)                          // the step face
                if (trans && (sinf2[q] & 7) != K_CAP) Fs = (R)0;
            fs_set(r, Fs);
            if (r & 1) __builtin_amdgcn_sched_barrier(0);      // register pressure
        }
        // the next line's slot must have landed before the first row reads it
        if constexpr (RING) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    // the first rows of the line above the current one, loaded one line ahead
    constexpr int PF = 2;
    R TnQ[PF], LnQ[PF];
    if constexpr (!RING) {
        const size_t bq = (size_t)(line_at(0) + dir) * LS;
#pragma unroll
        for (int r = 0; r < PF && r < RPL; ++r) {
            TnQ[r] = Tin[bq + r * NL + lg];
            LnQ[r] = PAIR ? Tin[bq + LO + r * NL + lg] : (R)0;
        }
    }
    for (int it = 0; it < a.lpw; ++it) {
        const bool active = it < j1 - j0;
        const int j = line_at(it);
        const size_t base = (size_t)j * LS;
        const size_t bo = (size_t)(j + dir) * LS;        // the other line: the next one
        // stepped domain: this line's tables, and whether its face with the
        // other line is the one at the step
        const bool up = STEPPED && j > a.z_full;
        const bool trans = STEPPED && min(j, j + dir) == a.z_full;
        const R *tgw = up ? sgw2 : sgw, *tge = up ? sge2 : sge;
        const uint32_t *tinf = up ? sinf2 : sinf;
        const R *sn = ring + ((it + 1) & 1) * SLOT;      // line j+1
        // the other slot (line j, already read into registers) takes line j+2;
        // its reads must have completed before the load overwrites it
        if constexpr (RING) {
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            prefetch(it & 1, (size_t)min(j + 2, a.nz - 1) * LS);
        }
        R TwP, TeP, LwP = 0, LeP = 0;                      // next line's chunk-end neighbours
        {
            const size_t bn = (size_t)line_at(it + 1) * LS;
            TwP = Tin[bn + qW];
            TeP = Tin[bn + qE];
            if constexpr (PAIR) {
                LwP = Tin[bn + LO + qW];
                LeP = Tin[bn + LO + qE];
            }
        }
        // west face of the chunk's first row: east face of the previous row
        R lamW = law.lawm((tinf[qW] >> 6) & 63, TwF + Tc[0]);
        R a0 = 0, b0 = 1, c0 = 0, d0 = 0;
        R al[RPL], ga[RPL], de[RPL];
        // without the ring: the next line's values come from memory two rows
        // ahead of their use (software pipelined across the rows' regions);
        // the first two were loaded before the previous line's solve
        R TnP[RPL], LnP[RPL];
        if constexpr (!RING) {
#pragma unroll
            for (int r = 0; r < PF && r < RPL; ++r) {
                TnP[r] = TnQ[r];
                LnP[r] = LnQ[r];
            }
        }
        // the held outer wall's row (uniform; -1 for none): its test below is
        // a scalar branch per row, not a select kept in registers for every row
        int hrow = (a.held[1] && !up) ? a.surf_reg : -1;
        hrow = __builtin_amdgcn_readfirstlane(hrow);
        const bool hlane = lg == a.surf_lane;
        // the rows' info words, one row ahead (they head each row's chain of
        // table lookups)
        uint32_t infn = tinf[lg];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int q = r * NL + lg;
            const uint32_t inf_r = infn;
            if (r + 1 < RPL) infn = tinf[q + NL];
            if constexpr (!RING) {
                if (r + PF < RPL) {
                    TnP[r + PF] = Tin[bo + q + PF * NL];
                    LnP[r + PF] = PAIR ? Tin[bo + LO + q + PF * NL] : (R)0;
                }
            }
            const uint32_t kind = inf_r & 7;
            const bool cap = kind == K_CAP;
            const R T = Tc[r], Tl = Lc[r];
            R Tnr, Lnr = 0;
            if constexpr (RING) {
                Tnr = sn[r * NPL * WAVE + lane];
                if constexpr (PAIR) Lnr = sn[(r * NPL + 1) * WAVE + lane];
            } else {
                Tnr = TnP[r];
                if constexpr (PAIR) Lnr = LnP[r];
            }
            // the carried flux into this line from the previous line, read
            // unconditionally at the row's start (a read under the capacity
            // test becomes a branch that waits for it at once)
            const R Fc = fs_get(r);
            const R Tw = (r > 0) ? Tc[r - 1] : TwF;
            const R Te = (r < RPL - 1) ? Tc[r + 1] : TeL;
            const R Lw = (r > 0) ? Lc[r - 1] : LwF;
            const R Le = (r < RPL - 1) ? Lc[r + 1] : LeL;
            const int le = (inf_r >> 6) & 63, l2 = (inf_r >> 12) & 63;
            const int lc = (inf_r >> 24) & 63;
            // every face mean lies between two nodes: one range check per node
            if constexpr (!PAIR) bad |= !LawLds<R>::in_range(T);
            // laws are evaluated from the sum of the two values they average
            const R lamE = law.lawm(le, T + Te);
            // slot 2: the north axial face of a capacity row (the row's radial
            // law: capacity rows are scaled by eta^2), the ratio of the inner
            // to the outer layer's law at an interface node (its row divided
            // by the outer law), or unit / zero (boundary, padding)
            R lam2 = law.lawm(l2, T + (cap ? Tnr : T));
            if constexpr (POLY) lam2 = lam2 / law.lawm((inf_r >> 18) & 63, T + T);
            R rc;
            if constexpr (CUBE) rc = law.cube(lc, T);
            else rc = law.lawm(lc, T + T);
            const R fw = tgw[q] * (cap ? lamW : lam2);
            const R fe = tge[q] * (cap ? lamE : (R)1);
            // flux into this line from the next one (carried on, negated)
            R Fo = lam2 * dif<R>(Tnr, Lnr, T, Tl);
            if constexpr (STEPPED)                          // the step face
                if (trans && (sinf2[q] & 7) != K_CAP) Fo = (R)0;
            R dd = fw * dif<R>(Tw, Lw, T, Tl) + fe * dif<R>(Te, Le, T, Tl);
            dd += cap ? Fo + Fc : (R)0;
            if constexpr (POLY)                                 // heater rows, eq. (25)
                dd += (R)((inf_r >> 3) & 1) * (a.joule ? X * rsqrt(T) : X);
            else
                dd += (R)((inf_r >> 3) & 1) * X;                // heater capacity rows
            // held walls: rows 0 and nr - 1 are unit rows with dT = value - T
            if (r == 0 && a.held[0]) dd = lg == 0 ? dif<R>(a.val[0], (R)0, T, Tl) : dd;
            if (r == hrow) {
                asm volatile("" ::: "memory");               // keeps the branch
                dd = hlane ? dif<R>(a.val[1], (R)0, T, Tl) : dd;
            }
            fs_set(r, -Fo);
            lamW = lamE;
            const R aa = -fw, bb = fw + fe + rc, cc = -fe;
            if (r == 0) {
                a0 = aa;
                b0 = bb;
                c0 = cc;
                d0 = dd;
            } else {
                elim_row<R, RPL>(r, aa, bb, cc, dd, al, ga, de);
                // eliminate here, not where the results are first used (the
                // solve): sinking it would keep every row's coefficients live
                asm volatile("" : "+v"(al[r]), "+v"(ga[r]), "+v"(de[r]));
            }
            // keep the scheduler from hoisting every row's law evaluations
            // at once (register pressure); rows still overlap pairwise
            if (RPL >= 10 || (r & 1)) __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (!RING) {
            // the next iteration's first rows of its other line (a boundary
            // line only for inactive iterations)
            const size_t bq = (size_t)(line_at(it + 1) + dir) * LS;
#pragma unroll
            for (int r = 0; r < PF && r < RPL; ++r) {
                TnQ[r] = Tin[bq + r * NL + lg];
                LnQ[r] = PAIR ? Tin[bq + LO + r * NL + lg] : (R)0;
            }
        }
        R X[RPL];
        // the line solve is the step's longest dependent chain (the cyclic
        // reduction's exchanges): a wave inside it issues before a wave still
        // in its rows, whose independent work fills the gaps (measured: 1 %
        // on the 1024 x 4096 FP64 step, results bit for bit the same)
        __builtin_amdgcn_s_setprio(2);
        solve_tail<R, RPL, G>(a0, b0, c0, d0, al, ga, de, X, lane, wig, xch);
        __builtin_amdgcn_s_setprio(0);
        // the line after next (slot) and the next neighbours have landed
        if constexpr (RING) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        if (active) {
            // new state: T + dT (pairs: error-free sum, then renormalise)
            R Hn[RPL], Lnw[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                if constexpr (PAIR) {
                    const R x = X[r], h = Tc[r];
                    const R s = h + x;
                    const R bp = s - h;
                    const R err = (h - (s - bp)) + (x - bp);
                    const R lo = Lc[r] + err;
                    const R h2 = s + lo;
                    Hn[r] = h2;
                    Lnw[r] = lo - (h2 - s);
                } else {
                    Hn[r] = Tc[r] + X[r];
                    Lnw[r] = (R)0;
                }
                Tout[base + r * NL + lg] = Hn[r];
                if constexpr (PAIR) Tout[base + LO + r * NL + lg] = Lnw[r];
            }
            // z-boundary lines: copied (insulated) or held, after the solve
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const bool mine = side == 0 ? j == 1 : j == a.nz - 2;
                if (!mine) continue;
                const bool held = a.held[2 + side];
                // formed here (cold path), not hoisted out of the line loop
                size_t ob = side == 0 ? (size_t)0 : (size_t)(a.nz - 1) * LS;
                asm volatile("" : "+v"(ob));
                R *o = Tout + ob;
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    o[r * NL + lg] = held ? a.val[2 + side] : Hn[r];
                    if constexpr (PAIR) o[LO + r * NL + lg] = held ? (R)0 : Lnw[r];
                }
            }
            if (partial && lg == a.surf_lane) {
                // the surface row's register is uniform: one scalar test per
                // register, and only the matching register's value is read
                int sreg = __builtin_amdgcn_readfirstlane(a.surf_reg);
                asm volatile("" : "+s"(sreg));               // cold path: no hoisting
                double v = 0.0;
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    if (r == sreg) {
                        asm volatile("" ::: "memory");       // keeps the branch
                        v = (double)Hn[r] + (double)Lnw[r];
                    }
                if constexpr (STEPPED) {                    // lines 0..z_full
                    sv += j < a.z_full ? a.wz_mid * v : j == a.z_full ? a.wz_end * v : 0.0;
                    if (j == 1) sv += a.wz_end * (a.held[2] ? (double)a.val[2] : v);
                } else {
                    sv += a.wz_mid * v;
                    if (j == 1) sv += a.wz_end * (a.held[2] ? (double)a.val[2] : v);
                    if (j == a.nz - 2) sv += a.wz_end * (a.held[3] ? (double)a.val[3] : v);
                }
            }
        }
        // next line: registers from its ring slot, or the values the rows
        // read as their north neighbours (line j + 1; past the last interior
        // line only inactive iterations use them)
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            if constexpr (RING) {
                Tc[r] = sn[r * NPL * WAVE + lane];
                Lc[r] = PAIR ? sn[(r * NPL + 1) * WAVE + lane] : (R)0;
            } else {
                Tc[r] = TnP[r];
                Lc[r] = LnP[r];
            }
        }
        TwF = TwP;
        TeL = TeP;
        LwF = LwP;
        LeL = LeP;
    }
    if (__any(bad)) {
        if (lane == 0) atomicOr(a.flag, 2);
    }
    if (partial) {
        if (lane == (a.surf_lane & (WAVE - 1))) wsum[wv] = sv;
        __syncthreads();
        if (t == 0) {
            double s = 0.0;
            for (int w = 0; w < STEP_WAVES; ++w) s += wsum[w];
            partial[blk] = s;
        }
    }
}

// Workgroups are dealt to the 8 XCDs in turn (workgroup b on XCD b mod 8);
// each XCD gets a contiguous range of line groups, so that the lines shared by
// neighbouring groups meet in the same L2.  A bijection of 0..nb-1.
__device__ inline int xcd_block(int b, int nb) {
    const int x = b & 7, i = b >> 3, per = nb >> 3, rem = nb & 7;
    return x * per + min(x, rem) + i;
}

template <typename R, int RPL, int G, bool CUBE, bool POLY = false, bool STEPPED = false>
__global__ __launch_bounds__(STEP_WAVES *WAVE) void k_step(StepArgs<R> a) {
    step_body<R, RPL, G, CUBE, POLY, STEPPED>(a, xcd_block(blockIdx.x, gridDim.x), a.Tin, a.Tout,
                                              a.X, a.partial);
}

// Pulse average over step k (eq. (4)), step units; the host's schedule.
__device__ inline double source_fraction_dev(const Pulse &p, int64_t k) {
    if (!(p.W > 0)) return 0.0;
    const double lo = (double)k, hi = lo + 1.0;
    double s = 0.0;
    int64_t n = (int64_t)floor((lo - p.b0 - p.W) / p.P);
    if (n < 0) n = 0;
    for (int guard = 0; guard < 64; ++guard, ++n) {
        const double b = p.b0 + (double)n * p.P;
        if (b >= hi) break;
        const double o = fmin(hi, b + p.W) - fmax(lo, b);
        if (o > 0) s += o;
    }
    return s;
}

// One step of many instances: workgroup -> (instance, workgroup of that
// instance); global step k = *k0 + n; buffers by the parity of n.
template <typename R, int RPL, int G, bool CUBE, bool POLY = false, bool STEPPED = false>
__global__ __launch_bounds__(STEP_WAVES *WAVE) void k_step_batch(const StepArgs<R> *descs,
                                                                 const int2 *wg_map, int64_t n,
                                                                 const int64_t *k0) {
    const int2 m = wg_map[blockIdx.x];
    const StepArgs<R> &a = descs[m.x];
    double X = a.pulse.amplitude * source_fraction_dev(a.pulse, *k0 + n);
    if constexpr (POLY) X *= a.jsq;                 // the Joule source's sqrt(T_J)
    double *part = a.partial ? a.partial + (size_t)(n % SURF_CHUNK) * a.groups : nullptr;
    step_body<R, RPL, G, CUBE, POLY, STEPPED>(a, m.y, a.buf[n & 1], a.buf[(n + 1) & 1], (R)X,
                                              part);
}

// ABI field -> internal lines.  FP32 fields are two planes [2][nz][nr]
// (rounded value, residual) and become [nz][2][np] internally.
template <typename R>
__global__ void k_to_internal(const R *T, R *Ti, int nz, int nr, int np, int rpl, R pad,
                              int *flag) {
    constexpr int NPL = Pair<R>::on ? 2 : 1;
    size_t n = (size_t)nz * NPL * np;
    size_t start = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (start == 0 && flag) *flag = 0;
    for (size_t idx = start; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        int j = (int)(idx / ((size_t)NPL * np));
        int rem = (int)(idx % ((size_t)NPL * np));
        int plane = rem / np, q = rem % np;
        const int nl = np / rpl;                      // lanes per line
        int i = (q % nl) * rpl + q / nl;
        R v = plane == 0 ? pad : (R)0;
        if (i < nr) v = T[((size_t)plane * nz + j) * nr + i];
        Ti[idx] = v;
    }
}

template <typename R>
__global__ void k_from_internal(const R *Ti, R *T, int nz, int nr, int np, int rpl, int *flag) {
    constexpr int NPL = Pair<R>::on ? 2 : 1;
    size_t n = (size_t)NPL * nz * nr;
    int bad = 0;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * blockDim.x) {
        int plane = (int)(idx / ((size_t)nz * nr));
        size_t rem = idx % ((size_t)nz * nr);
        int j = (int)(rem / nr), i = (int)(rem % nr);
        const int nl = np / rpl;
        R v = Ti[((size_t)j * NPL + plane) * np + (i % rpl) * nl + i / rpl];
        T[idx] = v;
        bad |= !isfinite(v);
    }
    if (bad) atomicOr(flag, 1);
}

template <typename R>
__global__ void k_fill(R *T, size_t n, R v, size_t n_lo) {
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n + n_lo;
         idx += (size_t)gridDim.x * blockDim.x)
        T[idx] = idx < n ? v : (R)0;
}

// S[k] = sum over workgroups of the step-k partial sums, in a fixed order
__global__ void k_surf_reduce(const double *part, int nsteps, int G, double *out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsteps) return;
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += part[(size_t)k * G + g];
    out[k] = s;
}

static int blocks_for(size_t n) {
    size_t b = (n + 255) / 256;
    return (int)std::min<size_t>(b, 65536);
}

static cryo_status launch_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CRYO_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return CRYO_OK;
}

int step_grid(const cryo_plan *p) {
    const int groups = (p->nz - 2 + p->lpw - 1) / p->lpw;
    const int per_wg = STEP_WAVES / p->wpl;
    return (groups + per_wg - 1) / per_wg;
}

template <typename R>
static cryo_status to_internal_t(const cryo_plan *p, const void *T, void *Ti, int *flag,
                                 hipStream_t s) {
    size_t n = (size_t)p->nz * p->np * (Pair<R>::on ? 2 : 1);
    hipLaunchKernelGGL(k_to_internal<R>, dim3(blocks_for(n)), dim3(256), 0, s, (const R *)T,
                       (R *)Ti, p->nz, p->nr, p->np, p->rpl, (R)p->prob.T_init, flag);
    return launch_check("to_internal");
}

cryo_status launch_to_internal(const cryo_plan *p, const void *T, void *Ti, int *flag,
                               hipStream_t s) {
    return p->dtype == CRYO_F64 ? to_internal_t<double>(p, T, Ti, flag, s)
                                : to_internal_t<float>(p, T, Ti, flag, s);
}

cryo_status launch_from_internal(const cryo_plan *p, const void *Ti, void *T, int *flag,
                                 hipStream_t s) {
    size_t n = (size_t)p->nz * p->nr * (p->dtype == CRYO_F32 ? 2 : 1);
    if (p->dtype == CRYO_F64)
        hipLaunchKernelGGL(k_from_internal<double>, dim3(blocks_for(n)), dim3(256), 0, s,
                           (const double *)Ti, (double *)T, p->nz, p->nr, p->np, p->rpl, flag);
    else
        hipLaunchKernelGGL(k_from_internal<float>, dim3(blocks_for(n)), dim3(256), 0, s,
                           (const float *)Ti, (float *)T, p->nz, p->nr, p->np, p->rpl, flag);
    return launch_check("from_internal");
}

cryo_status launch_fill(const cryo_plan *p, void *T, hipStream_t s) {
    size_t n = (size_t)p->nz * p->nr;
    if (p->dtype == CRYO_F64)
        hipLaunchKernelGGL(k_fill<double>, dim3(blocks_for(n)), dim3(256), 0, s, (double *)T, n,
                           p->prob.T_init, (size_t)0);
    else
        hipLaunchKernelGGL(k_fill<float>, dim3(blocks_for(2 * n)), dim3(256), 0, s, (float *)T, n,
                           (float)p->prob.T_init, n);
    return launch_check("fill");
}

// Arguments of the stepping kernel (its row tables and laws: capacity rows
// scaled by eta^2, so the source is too); the adjoint kernels take the same.
template <typename R>
static StepArgs<R> step_args(const cryo_plan *p, const void *Tin, void *Tout, double X,
                             double *partial, int *flag) {
    StepArgs<R> a;
    const double xs = p->eta * p->eta;
    a.flag = flag;
    a.Tin = (const R *)Tin;
    a.Tout = (R *)Tout;
    a.gw = (const R *)p->d_rows;
    a.ge = a.gw + p->np;
    a.info = p->d_info;
    a.pow_blob = p->d_pow;
    a.laws = p->flaws;
    a.nz = p->nz;
    a.np = p->np;
    a.lpw = p->lpw;
    a.joule = p->poly && p->joule_tref > 0;
    a.jsq = a.joule ? sqrt(p->joule_tref) : 1.0;
    a.X = (R)(X * xs * a.jsq);
    for (int s = 0; s < 4; ++s) {
        a.held[s] = p->prob.bc.kind[s] == CRYO_HELD;
        a.val[s] = (R)p->prob.bc.value[s];
    }
    a.partial = partial;
    a.wz_mid = 1.0 / (p->nz - 1);
    a.wz_end = 0.5 / (p->nz - 1);
    a.surf_lane = p->surf_lane;
    a.surf_reg = p->surf_reg;
    // stepped domain: the terminal's tables, and the surface over lines
    // 0..z_full
    a.z_full = p->stepped ? p->z_full : p->nz - 1;
    a.gw2 = p->stepped ? (const R *)p->d_rows2 : a.gw;
    a.ge2 = p->stepped ? a.gw2 + p->np : a.ge;
    a.info2 = p->stepped ? p->d_info2 : a.info;
    if (p->stepped) {
        a.wz_mid = 1.0 / p->z_full;
        a.wz_end = 0.5 / p->z_full;
    }
    a.groups = step_grid(p);
    a.pulse = p->pulse;
    a.pulse.amplitude *= xs;
    a.buf[0] = a.buf[1] = nullptr;
    return a;
}

template <typename R>
static cryo_status step_t(const cryo_plan *p, const void *Tin, void *Tout, double X,
                          double *partial, int *flag, hipStream_t s) {
    StepArgs<R> a = step_args<R>(p, Tin, Tout, X, partial, flag);
    dim3 g(step_grid(p)), b(STEP_WAVES * WAVE);
    const size_t lds = step_lds(p);
    const int key = p->rpl * 10 + p->wpl;
    switch (key) {
#define STEP_CASE(RP, GW) \
    case RP * 10 + GW: \
        if (p->stepped && p->poly) { \
            hipLaunchKernelGGL((k_step<R, RP, GW, false, true, true>), g, b, lds, s, a); \
            break; \
        } \
        if (p->stepped) { \
            if (a.laws.cube) hipLaunchKernelGGL((k_step<R, RP, GW, true, false, true>), g, b, lds, s, a); \
            else hipLaunchKernelGGL((k_step<R, RP, GW, false, false, true>), g, b, lds, s, a); \
            break; \
        } \
        if (p->poly) { \
            hipLaunchKernelGGL((k_step<R, RP, GW, false, true>), g, b, lds, s, a); \
            break; \
        } \
        if (a.laws.cube) hipLaunchKernelGGL((k_step<R, RP, GW, true>), g, b, lds, s, a); \
        else hipLaunchKernelGGL((k_step<R, RP, GW, false>), g, b, lds, s, a); \
        break;
        CRYO_FOR_SHAPES(STEP_CASE)
#undef STEP_CASE
    default: return fail(CRYO_ERR_UNSUPPORTED, "radial chunk shape");
    }
    return launch_check("step");
}

cryo_status launch_step(const cryo_plan *p, const void *Tin, void *Tout, double X,
                        double *partial, int *flag, hipStream_t s) {
    return p->dtype == CRYO_F64 ? step_t<double>(p, Tin, Tout, X, partial, flag, s)
                                : step_t<float>(p, Tin, Tout, X, partial, flag, s);
}

cryo_status launch_surf_reduce(const cryo_plan *p, const double *partial, int nsteps,
                               double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_surf_reduce, dim3((nsteps + 255) / 256), dim3(256), 0, s, partial,
                       nsteps, step_grid(p), out);
    return launch_check("surf_reduce");
}

}  // namespace cryo

namespace cryo {

// ---- batch support -------------------------------------------------------
size_t step_desc_bytes(cryo_dtype dt) {
    return dt == CRYO_F64 ? sizeof(StepArgs<double>) : sizeof(StepArgs<float>);
}

size_t step_lds(const cryo_plan *p) {
    // a stepped domain stages the terminal's tables too
    return p->dtype == CRYO_F64
               ? step_lds_bytes<double>(p->L, p->np, p->rpl) +
                     (p->stepped ? step_tables_bytes<double>(p->np) : 0)
               : step_lds_bytes<float>(p->L, p->np, p->rpl) +
                     (p->stepped ? step_tables_bytes<float>(p->np) : 0);
}

void step_desc_fill(const cryo_plan *p, void *out, void *buf0, void *buf1, int *flag) {
    if (p->dtype == CRYO_F64) {
        StepArgs<double> a = step_args<double>(p, nullptr, nullptr, 0.0, nullptr, flag);
        a.buf[0] = (double *)buf0;
        a.buf[1] = (double *)buf1;
        memcpy(out, &a, sizeof(a));
    } else {
        StepArgs<float> a = step_args<float>(p, nullptr, nullptr, 0.0, nullptr, flag);
        a.buf[0] = (float *)buf0;
        a.buf[1] = (float *)buf1;
        memcpy(out, &a, sizeof(a));
    }
}

template <typename R>
static cryo_status step_batch_t(int rpl, int wpl, bool cube, bool poly, bool stepped,
                                const void *desc, const int2 *map, int nwg, size_t lds,
                                int64_t n, const int64_t *k0, hipStream_t s) {
    const StepArgs<R> *d = (const StepArgs<R> *)desc;
    dim3 g(nwg), b(STEP_WAVES * WAVE);
    switch (rpl * 10 + wpl) {
#define BATCH_CASE(RP, GW) \
    case RP * 10 + GW: \
        if (poly && stepped) \
            hipLaunchKernelGGL((k_step_batch<R, RP, GW, false, true, true>), g, b, lds, s, d, map, \
                               n, k0); \
        else if (stepped && cube) \
            hipLaunchKernelGGL((k_step_batch<R, RP, GW, true, false, true>), g, b, lds, s, d, map, \
                               n, k0); \
        else if (stepped) \
            hipLaunchKernelGGL((k_step_batch<R, RP, GW, false, false, true>), g, b, lds, s, d, \
                               map, n, k0); \
        else if (poly) \
            hipLaunchKernelGGL((k_step_batch<R, RP, GW, false, true>), g, b, lds, s, d, map, n, k0); \
        else if (cube) \
            hipLaunchKernelGGL((k_step_batch<R, RP, GW, true>), g, b, lds, s, d, map, n, k0); \
        else \
            hipLaunchKernelGGL((k_step_batch<R, RP, GW, false>), g, b, lds, s, d, map, n, k0); \
        break;
        CRYO_FOR_SHAPES(BATCH_CASE)
#undef BATCH_CASE
    default: return fail(CRYO_ERR_UNSUPPORTED, "radial chunk shape");
    }
    return launch_check("step_batch");
}

cryo_status launch_step_batch(cryo_dtype dt, int rpl, int wpl, bool cube, bool poly,
                              bool stepped, const void *desc, const int2 *map, int nwg,
                              size_t lds, int64_t n, const int64_t *k0, hipStream_t s) {
    return dt == CRYO_F64
               ? step_batch_t<double>(rpl, wpl, cube, poly, stepped, desc, map, nwg, lds, n, k0, s)
               : step_batch_t<float>(rpl, wpl, cube, poly, stepped, desc, map, nwg, lds, n, k0, s);
}

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }
__global__ void k_add_i64(int64_t *p, int64_t v) { *p += v; }

cryo_status launch_set_i64(int64_t *ptr, int64_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, ptr, v);
    return launch_check("set_i64");
}

cryo_status launch_add_i64(int64_t *ptr, int64_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_add_i64, dim3(1), dim3(1), 0, s, ptr, v);
    return launch_check("add_i64");
}

}  // namespace cryo

namespace cryo {
StepArgs<double> step_args_f64(const cryo_plan *p, int *flag) {
    return step_args<double>(p, nullptr, nullptr, 0.0, nullptr, flag);
}
}  // namespace cryo
