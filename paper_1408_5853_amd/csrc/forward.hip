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
// The tridiagonal system is solved by partition: every lane eliminates its
// chunk down to two unknowns (first and last row), the 128 chunk-end unknowns
// are reduced to one per lane, and parallel cyclic reduction across the wave
// solves those; lanes then back-substitute their chunk.
#include <math.h>

#include "internal.h"

namespace cryo {

template <typename R>
__device__ inline R lg2(R x);
template <>
__device__ inline double lg2<double>(double x) { return log2(x); }
template <>
__device__ inline float lg2<float>(float x) { return log2f(x); }
template <typename R>
__device__ inline R ex2(R x);
template <>
__device__ inline double ex2<double>(double x) { return exp2(x); }
template <>
__device__ inline float ex2<float>(float x) { return exp2f(x); }

template <typename R>
struct LawTable {
    R p[2 * MAX_LAYERS], lk[2 * MAX_LAYERS];
    R q[MAX_LAYERS], lrc[MAX_LAYERS];
};

template <typename R>
struct StepArgs {
    const R *Tin;
    R *Tout;
    const R *gw, *ge;
    const uint32_t *info;
    Laws laws;
    int nz, np;
    R X;                      // amplitude * pulse average of this step
    int held[4];              // r_inner, r_outer, z_low, z_high
    R val[4];
    double *partial;          // nullable: per-workgroup surface partial sums
    double wz_end, wz_mid;    // trapezoid weights of the surface mean
    int surf_lane, surf_reg;
};

constexpr int STEP_WAVES = 4;

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

// Solve the wave's tridiagonal system; on entry lane k holds rows
// k*RPL..k*RPL+RPL-1 in (a, b, c, d); on exit d holds the solution.
template <typename R, int RPL>
__device__ inline void wave_solve(R (&a)[RPL], R (&b)[RPL], R (&c)[RPL], R (&d)[RPL],
                                  int lane) {
    static_assert(RPL >= 2, "chunks of at least two rows");
    // forward elimination of rows 1..RPL-1 with a fill-in column on row 0:
    //   al_r x_0 + x_r + ga_r x_{r+1} = de_r
    R al[RPL], ga[RPL], de[RPL];
    {
        R inv = (R)1 / b[1];
        al[1] = a[1] * inv;
        ga[1] = c[1] * inv;
        de[1] = d[1] * inv;
    }
#pragma unroll
    for (int r = 2; r < RPL; ++r) {
        R inv = (R)1 / (b[r] - a[r] * ga[r - 1]);
        al[r] = -a[r] * al[r - 1] * inv;
        ga[r] = c[r] * inv;
        de[r] = (d[r] - a[r] * de[r - 1]) * inv;
    }
    // backward elimination of rows RPL-3..1 onto the chunk ends x_0, x_e
#pragma unroll
    for (int r = RPL - 3; r >= 1; --r) {
        de[r] = de[r] - ga[r] * de[r + 1];
        al[r] = al[r] - ga[r] * al[r + 1];
        ga[r] = -ga[r] * ga[r + 1];
    }
    // first row: a0 x_e(k-1) + sb x_0 + sc x_e(k) = sd
    R sb, sc, sd;
    if (RPL == 2) {
        sb = b[0];
        sc = c[0];
        sd = d[0];
    } else {
        sb = b[0] - c[0] * al[1];
        sc = -c[0] * ga[1];
        sd = d[0] - c[0] * de[1];
    }
    R isb = (R)1 / sb;
    R sig = a[0] * isb, tau = sc * isb, rho = sd * isb;    // x_0 = rho - sig x_e(k-1) - tau x_e(k)
    const int e = RPL - 1;
    R sigN = shfl_dn1(sig, 1, lane), tauN = shfl_dn1(tau, 1, lane), rhoN = shfl_dn1(rho, 1, lane);
    // one unknown per lane: x_e(k)
    R A = -al[e] * sig;
    R B = (R)1 - al[e] * tau - ga[e] * sigN;
    R C = -ga[e] * tauN;
    R D = de[e] - al[e] * rho - ga[e] * rhoN;
    {
        R ib = (R)1 / B;
        A *= ib;
        C *= ib;
        D *= ib;
    }
#pragma unroll
    for (int s = 1; s < WAVE; s <<= 1) {
        R Am = shfl_up1(A, s, lane), Cm = shfl_up1(C, s, lane), Dm = shfl_up1(D, s, lane);
        R Ap = shfl_dn1(A, s, lane), Cp = shfl_dn1(C, s, lane), Dp = shfl_dn1(D, s, lane);
        R nb = (R)1 - A * Cm - C * Ap;
        R ib = (R)1 / nb;
        R nA = -A * Am * ib;
        R nC = -C * Cp * ib;
        R nD = (D - A * Dm - C * Dp) * ib;
        A = nA;
        C = nC;
        D = nD;
    }
    R xe = D;
    R xeP = shfl_up1(xe, 1, lane);
    R x0 = rho - sig * xeP - tau * xe;
#pragma unroll
    for (int r = 1; r < RPL - 1; ++r) d[r] = de[r] - al[r] * x0 - ga[r] * xe;
    d[0] = x0;
    d[e] = xe;
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

template <typename R, int RPL>
__global__ __launch_bounds__(STEP_WAVES *WAVE) void k_step(StepArgs<R> a) {
    constexpr bool PAIR = Pair<R>::on;
    __shared__ LawTable<R> lw;
    __shared__ double wsum[STEP_WAVES];
    const int t = threadIdx.x;
    if (t < a.laws.n) {
        lw.p[t] = (R)a.laws.p[t];
        lw.lk[t] = (R)a.laws.lk[t];
    }
    if (t < a.laws.L) {
        lw.q[t] = (R)a.laws.q[t];
        lw.lrc[t] = (R)a.laws.lrc[t];
    }
    __syncthreads();
    const int lane = t & (WAVE - 1), wv = t / WAVE;
    const int j = 1 + blockIdx.x * STEP_WAVES + wv;
    const size_t LS = (size_t)a.np * (PAIR ? 2 : 1);      // line stride
    double sv = 0.0;
    if (j <= a.nz - 2) {
        const size_t base = (size_t)j * LS;
        R Tc[RPL], Tn[RPL], Ts[RPL], gw[RPL], ge[RPL];
        R Lc[RPL], Ln[RPL], Ls[RPL];                       // low parts (pairs)
        uint32_t inf[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int q = r * WAVE + lane;
            Tc[r] = a.Tin[base + q];
            Tn[r] = a.Tin[base + LS + q];
            Ts[r] = a.Tin[base - LS + q];
            if constexpr (PAIR) {
                Lc[r] = a.Tin[base + a.np + q];
                Ln[r] = a.Tin[base + LS + a.np + q];
                Ls[r] = a.Tin[base - LS + a.np + q];
            } else {
                Lc[r] = Ln[r] = Ls[r] = (R)0;
            }
            inf[r] = a.info[q];
            gw[r] = a.gw[q];
            ge[r] = a.ge[q];
        }
        // r-neighbours across the chunk ends
        const R TwF = __shfl_up(Tc[RPL - 1], 1, WAVE);
        const R TeL = __shfl_down(Tc[0], 1, WAVE);
        R LwF = (R)0, LeL = (R)0;
        if constexpr (PAIR) {
            LwF = __shfl_up(Lc[RPL - 1], 1, WAVE);
            LeL = __shfl_down(Lc[0], 1, WAVE);
        }
        // east r-face conductivities, one per face (eq. (10), face-mean T)
        R lamE[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const R Te = (r < RPL - 1) ? Tc[r + 1] : TeL;
            const uint32_t le = (inf[r] >> 4) & 31;
            lamE[r] = ex2<R>(lw.p[le] * lg2<R>((R)0.5 * (Tc[r] + Te)) + lw.lk[le]);
        }
        const R lamWF = __shfl_up(lamE[RPL - 1], 1, WAVE);
        R A[RPL], B[RPL], C[RPL], D[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const uint32_t kind = inf[r] & 7;
            const bool cap = kind == K_CAP;
            const R T = Tc[r], Tl = Lc[r];
            const R Tw = (r > 0) ? Tc[r - 1] : TwF;
            const R Te = (r < RPL - 1) ? Tc[r + 1] : TeL;
            const R Lw = (r > 0) ? Lc[r - 1] : LwF;
            const R Le = (r < RPL - 1) ? Lc[r + 1] : LeL;
            const R lW = (r > 0) ? lamE[r - 1] : lamWF;
            // slots 2/3: axial faces of a capacity row (eq. (11)), or the two
            // layer laws at the node for an interface row (eq. (18))
            const uint32_t l2 = (inf[r] >> 9) & 31, l3 = (inf[r] >> 14) & 31;
            const uint32_t lc = (inf[r] >> 19) & 31;
            const R th2 = cap ? (R)0.5 * (T + Tn[r]) : T;
            const R th3 = cap ? (R)0.5 * (T + Ts[r]) : T;
            const R lam2 = ex2<R>(lw.p[l2] * lg2<R>(th2) + lw.lk[l2]);
            const R lam3 = ex2<R>(lw.p[l3] * lg2<R>(th3) + lw.lk[l3]);
            const R rc = cap ? ex2<R>(lw.q[lc] * lg2<R>(T) + lw.lrc[lc]) : (R)0;
            const R fw = gw[r] * (cap ? lW : lam2);
            const R fe = ge[r] * (cap ? lamE[r] : lam3);
            const R dW = dif<R>(Tw, Lw, T, Tl), dE = dif<R>(Te, Le, T, Tl);
            R dd = fw * dW + fe * dE;
            if (cap) {
                dd += lam2 * dif<R>(Tn[r], Ln[r], T, Tl) - lam3 * dif<R>(T, Tl, Ts[r], Ls[r]);
                if ((inf[r] >> 3) & 1) dd += a.X;
            }
            R aa = -fw, bb = fw + fe + rc, cc = -fe;
            if (kind == K_LO) {
                aa = 0;
                bb = 1;
                cc = a.held[0] ? (R)0 : (R)-1;
                dd = a.held[0] ? dif<R>(a.val[0], (R)0, T, Tl) : dE;
            } else if (kind == K_HI) {
                cc = 0;
                bb = 1;
                aa = a.held[1] ? (R)0 : (R)-1;
                dd = a.held[1] ? dif<R>(a.val[1], (R)0, T, Tl) : dW;
            } else if (kind == K_PAD) {
                aa = 0;
                bb = 1;
                cc = 0;
                dd = 0;
            }
            A[r] = aa;
            B[r] = bb;
            C[r] = cc;
            D[r] = dd;
        }
        wave_solve<R, RPL>(A, B, C, D, lane);
        // new state: T + dT (pairs: error-free sum, then renormalise)
        R Hn[RPL], Lnw[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            if constexpr (PAIR) {
                const R x = D[r], h = Tc[r];
                const R s = h + x;
                const R bp = s - h;
                const R err = (h - (s - bp)) + (x - bp);
                const R lo = Lc[r] + err;
                const R h2 = s + lo;
                Hn[r] = h2;
                Lnw[r] = lo - (h2 - s);
            } else {
                Hn[r] = Tc[r] + D[r];
                Lnw[r] = (R)0;
            }
            a.Tout[base + r * WAVE + lane] = Hn[r];
            if constexpr (PAIR) a.Tout[base + a.np + r * WAVE + lane] = Lnw[r];
        }
        // z-boundary lines: copied (insulated) or held, after the solve
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const bool mine = side == 0 ? j == 1 : j == a.nz - 2;
            if (!mine) continue;
            const bool held = a.held[2 + side];
            R *o = a.Tout + (side == 0 ? (size_t)0 : (size_t)(a.nz - 1) * LS);
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                o[r * WAVE + lane] = held ? a.val[2 + side] : Hn[r];
                if constexpr (PAIR) o[a.np + r * WAVE + lane] = held ? (R)0 : Lnw[r];
            }
        }
        if (a.partial && lane == a.surf_lane) {
            double v = (double)Hn[0] + (double)Lnw[0];
#pragma unroll
            for (int r = 1; r < RPL; ++r)
                if (r == a.surf_reg) v = (double)Hn[r] + (double)Lnw[r];
            sv = a.wz_mid * v;
            if (j == 1) sv += a.wz_end * (a.held[2] ? (double)a.val[2] : v);
            if (j == a.nz - 2) sv += a.wz_end * (a.held[3] ? (double)a.val[3] : v);
        }
    }
    if (a.partial) {
        if (lane == a.surf_lane) wsum[wv] = sv;
        __syncthreads();
        if (t == 0) {
            double s = 0.0;
            for (int w = 0; w < STEP_WAVES; ++w) s += wsum[w];
            a.partial[blockIdx.x] = s;
        }
    }
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
        int i = (q % WAVE) * rpl + q / WAVE;
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
        R v = Ti[((size_t)j * NPL + plane) * np + (i % rpl) * WAVE + i / rpl];
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

int step_grid(const cryo_plan *p) { return (p->nz - 2 + STEP_WAVES - 1) / STEP_WAVES; }

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

template <typename R>
static StepArgs<R> step_args(const cryo_plan *p, const void *Tin, void *Tout, double X,
                             double *partial) {
    StepArgs<R> a;
    a.Tin = (const R *)Tin;
    a.Tout = (R *)Tout;
    a.gw = (const R *)p->d_gw;
    a.ge = (const R *)p->d_ge;
    a.info = p->d_info;
    a.laws = p->laws;
    a.nz = p->nz;
    a.np = p->np;
    a.X = (R)X;
    for (int s = 0; s < 4; ++s) {
        a.held[s] = p->prob.bc.kind[s] == CRYO_HELD;
        a.val[s] = (R)p->prob.bc.value[s];
    }
    a.partial = partial;
    a.wz_mid = 1.0 / (p->nz - 1);
    a.wz_end = 0.5 / (p->nz - 1);
    a.surf_lane = p->surf_lane;
    a.surf_reg = p->surf_reg;
    return a;
}

template <typename R>
static cryo_status step_t(const cryo_plan *p, const void *Tin, void *Tout, double X,
                          double *partial, hipStream_t s) {
    StepArgs<R> a = step_args<R>(p, Tin, Tout, X, partial);
    dim3 g(step_grid(p)), b(STEP_WAVES * WAVE);
    switch (p->rpl) {
    case 2: hipLaunchKernelGGL((k_step<R, 2>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_step<R, 4>), g, b, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_step<R, 8>), g, b, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_step<R, 16>), g, b, 0, s, a); break;
    case 32: hipLaunchKernelGGL((k_step<R, 32>), g, b, 0, s, a); break;
    default: return fail(CRYO_ERR_UNSUPPORTED, "radial chunk length");
    }
    return launch_check("step");
}

cryo_status launch_step(const cryo_plan *p, const void *Tin, void *Tout, double X,
                        double *partial, hipStream_t s) {
    return p->dtype == CRYO_F64 ? step_t<double>(p, Tin, Tout, X, partial, s)
                                : step_t<float>(p, Tin, Tout, X, partial, s);
}

cryo_status launch_surf_reduce(const cryo_plan *p, const double *partial, int nsteps,
                               double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_surf_reduce, dim3((nsteps + 255) / 256), dim3(256), 0, s, partial,
                       nsteps, step_grid(p), out);
    return launch_check("surf_reduce");
}

}  // namespace cryo
