// rve_solve.hip -- persistent batched periodic-RVE solver for gfx950.
//
// One workgroup (256 threads, four wave64; or 512 threads, eight wave64, when
// compiled with FEHMM_NT=512 into namespace fehmm::nt512) owns one workspace
// slot and pulls RVE ids from a device queue until the batch is exhausted.  Per RVE it runs the
// micro Newton iteration of Sec. 3.3 (residual, tangent, linear solve, update;
// the PBC form in which G^T dLambda = 0), then the post-convergence outputs:
// Pbar = <P> (eq. Average-of-P-and-F) and the tangent transfer of Sec. 3.2 for
// the d^2 unit macro-gradient states, condensed as
//     Abar = <A> - Y^T K_ff^-1 Y = <A> - Z^T D^-1 Z,  Z = L^-1 Y,
// with K_ff = L D L^T the tangent at the converged state (end of Sec. 3.3).
//
// Constitutive law (Sec. 6, neo-Hookean, plane strain in 2D) in first-Piola
// form with Fi = F^-1, g_a = F^-T grad N_a (spatial gradient of N_a),
// c1 = mu - lambda/2 (J^2 - 1), c2 = lambda J^2:
//     P = mu F - c1 F^-T
//     A_iJkL = mu d_ik d_JL + c1 Fi_Jk Fi_Li + c2 Fi_Ji Fi_Lk
//     f_(a,i)       = sum_gp (mu (F grad N_a)_i - c1 g_a,i) w|J|
//     k_(a,i),(b,k) = sum_gp (mu d_ik grad N_a . grad N_b + c1 g_a,k g_b,i + c2 g_a,i g_b,k) w|J|
//     Y_(a,i),(kL)  = sum_gp (mu d_ik dN_a,L + c1 g_a,k Fi_Li + c2 g_a,i Fi_Lk) w|J|
// which equal int B^T S and int B^T C B + S_hat 1 of the paper's eqs. (DG^h,
// G_IK, S_IK) written with P and A = dP/dF.  The two other laws of the paper's
// micro-convergence comparisons (Sec. 6) take a generic path with P and A
// evaluated at the Gauss point (law_PA): St. Venant-Kirchhoff, P = F S with
// S = lambda tr(E) 1 + 2 mu E, A_iJkL = d_ik S_JL + lambda F_iJ F_kL +
// mu (F_iL F_kJ + (F F^T)_ik d_JL); and the fully linear case, P = sigma(eps),
// eps = sym(F - 1), A the constant elasticity tensor.
//
// The linear solve is a multifrontal LDL^T (no pivoting: the tangent can be
// indefinite at the initial guess past a micro-instability of a stiff inclusion)
// driven by the (d, n) plan: element matrices are gathered straight into the
// dense fronts, children's update matrices are extended-added from a stack, the
// forward substitution is fused into the factorization, and the backward
// substitution walks the fronts in reverse.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mesh_common.h"
#include "solver_dev.h"

#ifndef FEHMM_NT
#define FEHMM_NT 256
#define FEHMM_VARIANT nt256
#endif

namespace fehmm {
namespace FEHMM_VARIANT {

constexpr int NT = FEHMM_NT;
constexpr int NWAVE = NT / 64;
static_assert(NT == 256 || NT == 512, "workgroup size");

// Optional per-phase clock accounting (slot 0, thread 0), compiled in only
// with -DFEHMM_PHASE_PROF=1; the default build records nothing.
#ifndef FEHMM_PHASE_PROF
#define FEHMM_PHASE_PROF 0
#endif
enum { PH_ELEM, PH_GATHER, PH_ASM, PH_DIAG, PH_TRSM, PH_MFMA, PH_OUT, PH_BACK, PH_LINE, PH_FINAL, PH_TOTAL, PH_N };
#if FEHMM_PHASE_PROF
__device__ unsigned long long g_phase[PH_N];
#define PROF_T0() unsigned long long _pt = clock64()
#define PROF_MARK(ph)                                                        \
    do {                                                                     \
        if (blockIdx.x == 0 && threadIdx.x == 0) {                           \
            unsigned long long _n = clock64();                               \
            g_phase[ph] += _n - _pt;                                         \
            _pt = _n;                                                        \
        }                                                                    \
    } while (0)
#define PROF_RESET() _pt = clock64()
#else
#define PROF_T0()
#define PROF_MARK(ph)
#define PROF_RESET()
#endif

struct Smem {
    double pub[kStepFronts][2][18 + kMaxNrhs];  // pivot publication per front group (double-buffered)
    double red[NWAVE * 81];
    double dN[8 * 8 * 3];    // [gp][a][k]
    double Fbar[9];
    double outv[96];
    double wJ, r0, rnorm, atol, alpha;
    int flag;
    int rve;
    int stop;
};

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// deterministic block reduction of K values per thread; result in sm.outv[0..K)
template <int K>
__device__ inline void block_sum(double (&v)[K], Smem& sm) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) sm.red[wave * K + k] = s;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0;
        for (int w = 0; w < NWAVE; ++w) s += sm.red[w * K + threadIdx.x];
        sm.outv[threadIdx.x] = s;
    }
    __syncthreads();
}

template <int D>
__device__ inline void inv_det(const double* F, double* Fi, double& J) {
    if (D == 2) {
        J = F[0] * F[3] - F[1] * F[2];
        double r = 1.0 / J;
        Fi[0] = F[3] * r; Fi[1] = -F[1] * r; Fi[2] = -F[2] * r; Fi[3] = F[0] * r;
    } else {
        double c00 = F[4] * F[8] - F[5] * F[7], c01 = F[5] * F[6] - F[3] * F[8], c02 = F[3] * F[7] - F[4] * F[6];
        J = F[0] * c00 + F[1] * c01 + F[2] * c02;
        double r = 1.0 / J;
        Fi[0] = c00 * r;
        Fi[1] = (F[2] * F[7] - F[1] * F[8]) * r;
        Fi[2] = (F[1] * F[5] - F[2] * F[4]) * r;
        Fi[3] = c01 * r;
        Fi[4] = (F[0] * F[8] - F[2] * F[6]) * r;
        Fi[5] = (F[2] * F[3] - F[0] * F[5]) * r;
        Fi[6] = c02 * r;
        Fi[7] = (F[1] * F[6] - F[0] * F[7]) * r;
        Fi[8] = (F[0] * F[4] - F[1] * F[3]) * r;
    }
}

struct RveCtx {
    const DevPlan* plan;
    int d, n, ne, nn, nen, nd;
    int law;  // RVE_LAW_*: 0 neo-Hookean, 1 St. Venant-Kirchhoff, 2 fully linear
    int elem; // RVE_ELEM_*: 0 Q1 / hex8 with 2^d Gauss points, 1 P1 (d! Kuhn simplices per cell)
    int ke32; // Newton element tangents stored in FP32 (FP32 factors); FP64 at the converged state
    const uint8_t* phase;
    const double* lame;
    double* w;
    double* wt;
    double* R;
    double* rhs;
    double* x;
    double* fe;
    double* ke;
    double* re;
    double* L;
    double* U;
    double* S;
};

// node v holds w = 0: node 0 under periodic coupling, every boundary node
// (some grid index 0) under linear displacements
__device__ inline bool is_pinned(const DevPlan& pl, int v) { return plan_pinned(pl.bc, pl.d, pl.n, v); }

// zero x at the pinned nodes' dofs (node-major [dof][nc]): the triangular
// solves write the free rows only
template <int D>
__device__ inline void zero_pinned(const RveCtx& c, double* x, int nc) {
    const DevPlan& pl = *c.plan;
    if (pl.bc == 0) {
        for (int t = threadIdx.x; t < D * nc; t += NT) x[t] = 0.0;
        return;
    }
    for (int t = threadIdx.x; t < c.nn * D * nc; t += NT)
        if (is_pinned(pl, t / (D * nc))) x[t] = 0.0;
}

// P and A = dP/dF (row-major [(i*D+J)*D*D + k*D+L]) of the St. Venant-Kirchhoff
// law (law 1) or of the fully linear law (law 2) at F; plane strain in 2D
template <int D>
__device__ inline void law_PA(int law, double lam, double mu, const double* F, double* P, double* A) {
    constexpr int D2 = D * D;
    if (law == 1) {
        double S[D2], B[D2];
        double trE = 0.0;
#pragma unroll
        for (int I = 0; I < D; ++I)
#pragma unroll
            for (int J = 0; J < D; ++J) {
                double c = 0.0, b = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    c += F[k * D + I] * F[k * D + J];
                    b += F[I * D + k] * F[J * D + k];
                }
                S[I * D + J] = 0.5 * (c - (I == J ? 1.0 : 0.0));  // E for now
                B[I * D + J] = b;
            }
#pragma unroll
        for (int I = 0; I < D; ++I) trE += S[I * D + I];
#pragma unroll
        for (int q = 0; q < D2; ++q) S[q] = 2.0 * mu * S[q] + ((q % (D + 1)) == 0 ? lam * trE : 0.0);
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int J = 0; J < D; ++J) {
                double v = 0.0;
#pragma unroll
                for (int K = 0; K < D; ++K) v += F[i * D + K] * S[K * D + J];
                P[i * D + J] = v;
            }
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int J = 0; J < D; ++J)
#pragma unroll
                for (int k = 0; k < D; ++k)
#pragma unroll
                    for (int L = 0; L < D; ++L)
                        A[(i * D + J) * D2 + k * D + L] = (i == k ? S[J * D + L] : 0.0) + lam * F[i * D + J] * F[k * D + L] +
                                                          mu * (F[i * D + L] * F[k * D + J] + (J == L ? B[i * D + k] : 0.0));
    } else {
        double tr = 0.0;
#pragma unroll
        for (int I = 0; I < D; ++I) tr += F[I * D + I] - 1.0;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int J = 0; J < D; ++J)
                P[i * D + J] = mu * (F[i * D + J] + F[J * D + i] - (i == J ? 2.0 : 0.0)) + (i == J ? lam * tr : 0.0);
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int J = 0; J < D; ++J)
#pragma unroll
                for (int k = 0; k < D; ++k)
#pragma unroll
                    for (int L = 0; L < D; ++L)
                        A[(i * D + J) * D2 + k * D + L] = (i == J && k == L ? lam : 0.0) +
                                                          mu * ((i == k && J == L ? 1.0 : 0.0) + (i == L && J == k ? 1.0 : 0.0));
    }
}

// F at Gauss point gp of element e for nodal fluctuation w
template <int D>
__device__ inline void gp_F(const RveCtx& c, const Smem& sm, const double* wl, int gp, double* F) {
    constexpr int NEN = 1 << D;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int J = 0; J < D; ++J) {
            double s = sm.Fbar[i * D + J];
#pragma unroll
            for (int b = 0; b < NEN; ++b) s += wl[b * D + i] * sm.dN[(gp * 8 + b) * 3 + J];
            F[i * D + J] = s;
        }
}

template <int D>
__device__ inline void load_wl(const RveCtx& c, const double* w, int e, double* wl, int* nodes) {
    constexpr int NEN = 1 << D;
    element_nodes(D, c.n, e, nodes);
#pragma unroll
    for (int b = 0; b < NEN; ++b)
#pragma unroll
        for (int i = 0; i < D; ++i) wl[b * D + i] = w[nodes[b] * D + i];
}

// Mode 4 (2D): one work item's share of the condensation in the stationary
// form, sum over the element rows t of X_t^T y_t + y_t^T X_t - X_t^T (k_t X_e)
// (the assembled Y^T X + X^T Y - X^T K X), with X [dof][ldx] at xv (zero on the
// pinned dofs) and the FP64 tangent and Y rows of the state, into acc.
template <int D, int RPI>
__device__ inline void cond_item(int row0, const double (&kr)[RPI][(1 << D) * D], const double (&yr)[RPI][D * D],
                                 const double* xv, int ldx, const int* nodes, double* acc) {
    constexpr int NEN = 1 << D, ND = NEN * D, D2 = D * D;
#pragma unroll
    for (int r = 0; r < RPI; ++r) {
        const int row = row0 + r;
        const double* xr = xv + ((int64_t)nodes[row / D] * D + row % D) * ldx;
        double x[D2], kx[D2];
#pragma unroll
        for (int g = 0; g < D2; ++g) {
            x[g] = xr[g];
            kx[g] = 0.0;
        }
#pragma unroll
        for (int q = 0; q < ND; ++q) {
            const double* xq = xv + ((int64_t)nodes[q / D] * D + q % D) * ldx;
#pragma unroll
            for (int h = 0; h < D2; ++h) kx[h] += kr[r][q] * xq[h];
        }
#pragma unroll
        for (int g = 0; g < D2; ++g)
#pragma unroll
            for (int h = 0; h < D2; ++h) acc[g * D2 + h] += x[g] * yr[r][h] + yr[r][g] * x[h] - x[g] * kx[h];
    }
}

// Outputs of an element pass work item (element e, rows row0 .. row0 + RPI - 1):
// mode 0 the internal forces and tangent rows (FP32 when c.ke32, the factors'
// input); mode 2 the Y rows and, when c.ke32, the FP64 tangent rows at the
// converged state (the condensation's input); mode 3 the FP64 product of the
// tangent rows with xv at the element's nodes, into the force slots.
template <int D, int RPI>
__device__ inline void element_store(const RveCtx& c, int e, int row0, int mode, const double (&fr)[RPI],
                                     const double (&kr)[RPI][(1 << D) * D], const double (&yr)[RPI][D * D],
                                     const double* xv, const int* nodes) {
    constexpr int NEN = 1 << D, ND = NEN * D, D2 = D * D;
    if (mode == 0) {
#pragma unroll
        for (int r = 0; r < RPI; ++r) {
            const int64_t row = (int64_t)e * ND + row0 + r;
            c.fe[row] = fr[r];
            if (c.ke32) {
                float* kd = reinterpret_cast<float*>(c.ke) + row * ND;
#pragma unroll
                for (int q = 0; q < ND; ++q) kd[q] = (float)kr[r][q];
            } else {
                double* kd = c.ke + row * ND;
#pragma unroll
                for (int q = 0; q < ND; ++q) kd[q] = kr[r][q];
            }
        }
    } else if (mode == 2) {
#pragma unroll
        for (int r = 0; r < RPI; ++r) {
            const int64_t row = (int64_t)e * ND + row0 + r;
            double* yd = c.re + row * D2;
#pragma unroll
            for (int q = 0; q < D2; ++q) yd[q] = yr[r][q];
            if (c.ke32) {
                double* kd = c.ke + row * ND;
#pragma unroll
                for (int q = 0; q < ND; ++q) kd[q] = kr[r][q];
            }
        }
    } else if (mode == 3) {
        double xl[ND];
#pragma unroll
        for (int b = 0; b < NEN; ++b)
#pragma unroll
            for (int k = 0; k < D; ++k) xl[b * D + k] = xv[nodes[b] * D + k];
#pragma unroll
        for (int r = 0; r < RPI; ++r) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < ND; ++q) s += kr[r][q] * xl[q];
            c.fe[(int64_t)e * ND + row0 + r] = s;
        }
    }
}

// Element pass of the St. Venant-Kirchhoff and fully linear laws: as
// element_pass_nh, with P and A evaluated at each Gauss point (law_PA) and the rows
// contracted with the material gradients,
//     f_(a,i) = sum P_iJ dN_a,J w|J|,  k_(a,i),(b,k) = sum dN_a,J A_iJkL dN_b,L w|J|,
//     Y_(a,i),(kL) = sum dN_a,J A_iJkL w|J|.
template <int D, int NPT>
__device__ __noinline__ void element_pass_law(const RveCtx& c, Smem& sm, const double* w, int mode, double* accP,
                                              double* accA, const double* xv, int ldx) {
    constexpr int NEN = 1 << D, ND = NEN * D, D2 = D * D, RPI = (D == 2) ? 2 : 1;
    const int nitems = c.ne * NEN * (D / RPI);
    const double wJ = sm.wJ;
    constexpr int NCOND = D == 2 ? 16 : 1;  // mode 4 (2D): the condensation's share of this thread
    double accC[NCOND];
#pragma unroll
    for (int q = 0; q < NCOND; ++q) accC[q] = 0.0;
    for (int it = threadIdx.x; it < nitems; it += NT) {
        int e, a, i0;
        if (D == 2) { e = it / NEN; a = it % NEN; i0 = 0; }
        else { e = it / (NEN * D); a = (it / D) % NEN; i0 = it % D; }
        if (mode == 1 && (a != 0 || i0 != 0)) continue;
        double wl[ND];
        int nodes[NEN];
        load_wl<D>(c, w, e, wl, nodes);
        const int ph = c.phase[e];
        const double lam = c.lame[2 * ph], mu = c.lame[2 * ph + 1];
        double kr[RPI][ND];
        double fr[RPI];
        double yr[RPI][D2];
#pragma unroll
        for (int r = 0; r < RPI; ++r) {
            fr[r] = 0;
#pragma unroll
            for (int q = 0; q < ND; ++q) kr[r][q] = 0;
#pragma unroll
            for (int q = 0; q < D2; ++q) yr[r][q] = 0;
        }
        for (int gp = 0; gp < NPT; ++gp) {
            double F[D2], Fi[D2], J;
            gp_F<D>(c, sm, wl, gp, F);
            inv_det<D>(F, Fi, J);
            if (!(J > 0.0)) { sm.flag = 1; continue; }
            if (mode == 1) continue;
            double Pg[D2], Ag[D2 * D2];
            law_PA<D>(c.law, lam, mu, F, Pg, Ag);
            if ((mode == 2 || mode == 4) && a == 0 && i0 == 0) {
#pragma unroll
                for (int q = 0; q < D2; ++q) accP[q] += Pg[q] * wJ;
#pragma unroll
                for (int q = 0; q < D2 * D2; ++q) accA[q] += Ag[q] * wJ;
            }
            const double* dNa = &sm.dN[(gp * 8 + a) * 3];
#pragma unroll
            for (int r = 0; r < RPI; ++r) {
                const int i = i0 + r;
                if (mode == 0) {
                    double f = 0.0;
#pragma unroll
                    for (int Jj = 0; Jj < D; ++Jj) f += Pg[i * D + Jj] * dNa[Jj];
                    fr[r] += f * wJ;
                }
                if (mode == 0 || mode == 3 || mode == 4 || (mode == 2 && c.ke32)) {
#pragma unroll
                    for (int b = 0; b < NEN; ++b) {
                        const double* dNb = &sm.dN[(gp * 8 + b) * 3];
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            double v = 0.0;
#pragma unroll
                            for (int Jj = 0; Jj < D; ++Jj)
#pragma unroll
                                for (int L = 0; L < D; ++L) v += dNa[Jj] * Ag[(i * D + Jj) * D2 + k * D + L] * dNb[L];
                            kr[r][b * D + k] += v * wJ;
                        }
                    }
                }
                if (mode == 2 || mode == 4) {
#pragma unroll
                    for (int k = 0; k < D; ++k)
#pragma unroll
                        for (int L = 0; L < D; ++L) {
                            double v = 0.0;
#pragma unroll
                            for (int Jj = 0; Jj < D; ++Jj) v += dNa[Jj] * Ag[(i * D + Jj) * D2 + k * D + L];
                            yr[r][k * D + L] += v * wJ;
                        }
                }
            }
        }
        if constexpr (D == 2) {
            if (mode == 4) {
                cond_item<D, RPI>(a * D + i0, kr, yr, xv, ldx, nodes, accC);
                continue;
            }
        }
        element_store<D, RPI>(c, e, a * D + i0, mode, fr, kr, yr, xv, nodes);
    }
    if constexpr (D == 2)
        if (mode == 4)
#pragma unroll
            for (int q = 0; q < NCOND; ++q) accA[q] -= accC[q];
}

// Element pass of the neo-Hookean law.  mode 0: residual + tangent rows
// (Newton); mode 1: J > 0 check only (on w); mode 2: final outputs (Pbar, <A>,
// Y rows); mode 3: the FP64 tangent applied to xv, matrix-free (refinement of
// FP32 solves); mode 4 (2D): Pbar and <A> minus the condensation in the
// stationary form with X at xv (cond_item), nothing stored.  Work item = (e, a)
// in 2D (rows i = 0,1), (e, a, i) in 3D.
template <int D, int NPT>
__device__ __noinline__ void element_pass_nh(const RveCtx& c, Smem& sm, const double* w, int mode, double* accP,
                                             double* accA, const double* xv, int ldx) {
    constexpr int NEN = 1 << D, ND = NEN * D, RPI = (D == 2) ? 2 : 1;
    const int nitems = c.ne * NEN * (D / RPI);
    const double wJ = sm.wJ;
    constexpr int NCOND = D == 2 ? 16 : 1;  // mode 4 (2D): the condensation's share of this thread
    double accC[NCOND];
#pragma unroll
    for (int q = 0; q < NCOND; ++q) accC[q] = 0.0;
    for (int it = threadIdx.x; it < nitems; it += NT) {
        int e, a, i0;
        if (D == 2) { e = it / NEN; a = it % NEN; i0 = 0; }
        else { e = it / (NEN * D); a = (it / D) % NEN; i0 = it % D; }
        if (mode == 1 && (a != 0 || i0 != 0)) continue;
        double wl[ND];
        int nodes[NEN];
        load_wl<D>(c, w, e, wl, nodes);
        const int ph = c.phase[e];
        const double lam = c.lame[2 * ph], mu = c.lame[2 * ph + 1];
        double kr[RPI][ND];
        double fr[RPI];
        double yr[RPI][D * D];
#pragma unroll
        for (int r = 0; r < RPI; ++r) {
            fr[r] = 0;
#pragma unroll
            for (int q = 0; q < ND; ++q) kr[r][q] = 0;
#pragma unroll
            for (int q = 0; q < D * D; ++q) yr[r][q] = 0;
        }
        for (int gp = 0; gp < NPT; ++gp) {
            double F[D * D], Fi[D * D], J;
            gp_F<D>(c, sm, wl, gp, F);
            inv_det<D>(F, Fi, J);
            if (!(J > 0.0)) { sm.flag = 1; continue; }
            if (mode == 1) continue;
            const double c1 = mu - 0.5 * lam * (J * J - 1.0), c2 = lam * J * J;
            if ((mode == 2 || mode == 4) && a == 0 && i0 == 0) {
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int Jj = 0; Jj < D; ++Jj) accP[i * D + Jj] += (mu * F[i * D + Jj] - c1 * Fi[Jj * D + i]) * wJ;
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int Jj = 0; Jj < D; ++Jj)
#pragma unroll
                        for (int k = 0; k < D; ++k)
#pragma unroll
                            for (int L = 0; L < D; ++L)
                                accA[(i * D + Jj) * D * D + k * D + L] +=
                                    ((i == k && Jj == L ? mu : 0.0) + c1 * Fi[Jj * D + k] * Fi[L * D + i] +
                                     c2 * Fi[Jj * D + i] * Fi[L * D + k]) * wJ;
            }
            // spatial gradients g_b = F^-T grad N_b
            double g[NEN][D];
#pragma unroll
            for (int b = 0; b < NEN; ++b)
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    double s = 0;
#pragma unroll
                    for (int Jj = 0; Jj < D; ++Jj) s += Fi[Jj * D + k] * sm.dN[(gp * 8 + b) * 3 + Jj];
                    g[b][k] = s;
                }
            const double* dNa = &sm.dN[(gp * 8 + a) * 3];
            double ga[D];
#pragma unroll
            for (int k = 0; k < D; ++k) ga[k] = 0;
            for (int b = 0; b < NEN; ++b)
                if (b == a)
#pragma unroll
                    for (int k = 0; k < D; ++k) ga[k] = g[b][k];
#pragma unroll
            for (int r = 0; r < RPI; ++r) {
                const int i = i0 + r;
                if (mode == 0) {
                    double FdN = 0;
#pragma unroll
                    for (int Jj = 0; Jj < D; ++Jj) FdN += F[i * D + Jj] * dNa[Jj];
                    fr[r] += (mu * FdN - c1 * ga[i]) * wJ;
                }
                if (mode == 0 || mode == 3 || mode == 4 || (mode == 2 && c.ke32)) {
#pragma unroll
                    for (int b = 0; b < NEN; ++b) {
                        double dab = 0.0;
#pragma unroll
                        for (int k2 = 0; k2 < D; ++k2) dab += dNa[k2] * sm.dN[(gp * 8 + b) * 3 + k2];
#pragma unroll
                        for (int k = 0; k < D; ++k)
                            kr[r][b * D + k] += ((i == k ? mu * dab : 0.0) + c1 * ga[k] * g[b][i] + c2 * ga[i] * g[b][k]) * wJ;
                    }
                }
                if (mode == 2 || mode == 4) {
#pragma unroll
                    for (int k = 0; k < D; ++k)
#pragma unroll
                        for (int L = 0; L < D; ++L)
                            yr[r][k * D + L] += ((i == k ? mu * dNa[L] : 0.0) + c1 * ga[k] * Fi[L * D + i] +
                                                 c2 * ga[i] * Fi[L * D + k]) * wJ;
                }
            }
        }
        if constexpr (D == 2) {
            if (mode == 4) {
                cond_item<D, RPI>(a * D + i0, kr, yr, xv, ldx, nodes, accC);
                continue;
            }
        }
        element_store<D, RPI>(c, e, a * D + i0, mode, fr, kr, yr, xv, nodes);
    }
    if constexpr (D == 2)
        if (mode == 4)
#pragma unroll
            for (int q = 0; q < NCOND; ++q) accA[q] -= accC[q];
}

// the element pass of the RVE's law (neo-Hookean closed forms, or the generic
// path) and element kind (2^d Gauss points of Q1 / hex8, or d! P1 simplices)
template <int D>
__device__ inline void element_pass(const RveCtx& c, Smem& sm, const double* w, int mode, double* accP, double* accA,
                                    const double* xv = nullptr, int ldx = 0) {
    constexpr int NQ1 = 1 << D, NP1 = D == 2 ? 2 : 6;
    if (c.elem == 0) {
        if (c.law != 0) element_pass_law<D, NQ1>(c, sm, w, mode, accP, accA, xv, ldx);
        else element_pass_nh<D, NQ1>(c, sm, w, mode, accP, accA, xv, ldx);
    } else {
        if (c.law != 0) element_pass_law<D, NP1>(c, sm, w, mode, accP, accA, xv, ldx);
        else element_pass_nh<D, NP1>(c, sm, w, mode, accP, accA, xv, ldx);
    }
}

// out = sb * b - K x on the free dofs (0 on the pinned ones), from the element
// products k_e x_e that element pass mode 3 left in the force slots
template <int D>
__device__ void residual_act(const RveCtx& c, const double* b, double sb, double* out) {
    constexpr int NEN = 1 << D, ND = NEN * D;
    for (int vi = threadIdx.x; vi < c.nn * D; vi += NT) {
        const int v = vi / D, i = vi % D;
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < NEN; ++a) s += c.fe[(int64_t)element_of_node(D, c.n, v, a) * ND + a * D + i];
        out[vi] = is_pinned(*c.plan, v) ? 0.0 : sb * b[vi] - s;
    }
}

// node gather of element vectors: out[(v*D+i)*ldo + q0 + col] = sum_a src[e_a(v)][(a*D+i)*nc + col]
// (ldo = nc, q0 = 0 by default)
template <int D>
__device__ void node_gather(const RveCtx& c, const double* src, int nc, double* out, double sign, int ldo = 0,
                            int q0 = 0) {
    constexpr int NEN = 1 << D, ND = NEN * D;
    const int tot = c.nn * D * nc, ld = ldo > 0 ? ldo : nc;
    for (int t = threadIdx.x; t < tot; t += NT) {
        int col = t % nc, vi = t / nc, v = vi / D, i = vi % D;
        double s = 0;
#pragma unroll
        for (int a = 0; a < NEN; ++a) {
            int e = element_of_node(D, c.n, v, a);
            s += src[((int64_t)e * ND + a * D + i) * nc + col];
        }
        out[(int64_t)vi * ld + q0 + col] = sign * s;
    }
}

// The element tangents a factorization with NRHS right-hand sides reads: the
// Newton factorizations (one rhs, or d^2 + 1 with the condensation's columns)
// read them in the factor type (FP32 for FP32 factors), the condensation
// factorizations at the converged state (d^2 rhs) in FP64.  (The global path
// factors the condensation in FP64 and passes NRHS = 1 with T = double.)
template <int D, int NRHS, typename T>
using KeType = typename std::conditional<NRHS != D * D, T, double>::type;
template <int D, int NRHS, typename T>
__device__ inline const KeType<D, NRHS, T>* ke_of(const RveCtx& c) {
    return reinterpret_cast<const KeType<D, NRHS, T>*>(c.ke);
}

// ---------------------------------------------------------------- LDS fronts
// A front that fits in LDS is held there whole as a packed lower triangle,
// column-major: entry (i, j), i >= j, at cpk(j, m) + i - j.  The first p columns
// are the L panel and the trailing columns are exactly the packed update matrix,
// so both leave the front with one contiguous copy each.

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ inline int cpk(int j, int m) { return j * m - ((j * (j - 1)) >> 1); }

// 1/x for a pivot on the elimination's dependent chain: the hardware reciprocal
// estimate refined by two Newton-Raphson steps r <- r + r (1 - x r), each of
// which squares the relative error (full double precision for the normal pivots
// that pass the vanishing-pivot test; a pivot that fails it is flagged whatever
// this returns)
__device__ inline double recip_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

__device__ inline double readlane_d(double v, int l) {
    union { double d; int i[2]; } u;
    u.d = v;
    u.i[0] = __builtin_amdgcn_readlane(u.i[0], l);
    u.i[1] = __builtin_amdgcn_readlane(u.i[1], l);
    return u.d;
}

// the same in the factor type: LDS-front eliminations run in the precision the
// front is stored in (FP32 fronts: one readlane per broadcast, FP32 arithmetic;
// the Newton step is refined against the FP64 residual)
__device__ inline double readlane_t(double v, int l) { return readlane_d(v, l); }
__device__ inline float readlane_t(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double recip_t(double x) { return recip_nr(x); }
__device__ inline float recip_t(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// ---------------------------------------------------------------- global fronts
// Plans whose fronts exceed LDS (3D from 5^3 up) keep each front in the slot's
// global workspace in the factor type T: the m x p panel column-major (column j
// at Fp + j m, rows i >= j used), its p pivots, and the mu x mu update matrix
// U_s column-major (lower part used) followed by its FP64 rhs rows; the
// forward-substituted rhs stays FP64.  The panel is factored left-looking in
// 64-column blocks: a block first takes the updates of all columns left of it
// as LDS-staged MFMA tiles, then each of its 16-column sub-blocks takes the
// updates of the earlier sub-blocks, wave 0 factors the 16 x 16 diagonal block
// in registers (readlane broadcasts) and forms W = L11^-T D^-1, and the rows
// below become L21 = A21 W on MFMA.  The Schur complement U_s - L21 D L21^T
// goes through the same tiles, straight onto the update stack.

// MFMA 16 x 16 x 4 of the factor type: operand lanes A[l % 16][l / 16] and
// B[l / 16][l % 16]; element v of lane l of the result is at column l % 16 and
// row row(l, v) (FP64: l / 16 + 4 v; FP32: 4 (l / 16) + v; both verified by
// in-bounds probes of the builtins)
typedef float flt4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Mfma16;
template <>
struct Mfma16<double> {
    typedef dbl4 V;
    static __device__ inline V mma(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
    static __device__ inline V zero() { return V{0.0, 0.0, 0.0, 0.0}; }
};
template <>
struct Mfma16<float> {
    typedef flt4 V;
    static __device__ inline V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
    static __device__ inline V zero() { return V{0.f, 0.f, 0.f, 0.f}; }
};

// FP64 rhs rows that follow an mu x mu matrix of T in an update region
template <typename T>
__device__ inline double* urhs(double* base, int mu) {
    return base + ((int64_t)mu * mu * (int64_t)sizeof(T) + 7) / 8;
}

// 16 x 16 diagonal block of a panel by wave 0: LDL^T with readlane broadcasts
// (FP64 arithmetic, stored in T), rhs of the block rows, W = L11^-T D^-1 (16 x
// 16, row-major) into W.  A(r, cc) is the block entry (K + r, K + cc) at
// Ap[cc * ldA + r]; rhs column q of the block rows at yv_base[q * ldy + r].
template <typename T>
__device__ inline void diag_block_wave(T* Ap, int ldA, T* Dd, const T* d0v, int kb, double* yv_base, int ldy,
                                       int nrhs, T* W, int* flag) {
    const int lane = threadIdx.x & 63;
    const bool own = lane < kb;
    double row[16];
    double yv[kMaxNrhs];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc)
        row[cc] = (own && cc < kb && cc <= lane) ? (double)Ap[(int64_t)cc * ldA + lane] : 0.0;
#pragma unroll
    for (int q = 0; q < kMaxNrhs; ++q) yv[q] = (own && q < nrhs) ? yv_base[(int64_t)q * ldy + lane] : 0.0;
    const double d0 = own ? (double)d0v[lane] : 1.0;
    double dpiv = 1.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j < kb) {
            const double piv = readlane_d(row[j], j);
            const double rp = 1.0 / piv;
            if (lane == j) {
                dpiv = piv;
                if (!(fabs(piv) > 1e-14 * fabs(d0)) || !isfinite(piv)) *flag = 2;
            }
            const double l = (lane > j) ? row[j] * rp : 0.0;
            const double lpv = l * piv;
#pragma unroll
            for (int cc = j + 1; cc < 16; ++cc) {
                if (cc < kb) {
                    const double lc = readlane_d(l, cc);
                    if (cc <= lane) row[cc] -= lpv * lc;
                }
            }
#pragma unroll
            for (int q = 0; q < kMaxNrhs; ++q) {
                if (q < nrhs) {
                    const double yj = readlane_d(yv[q], j);
                    if (lane > j) yv[q] -= l * yj;
                }
            }
            if (lane > j) row[j] = l;
        }
    }
    double inv[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) inv[cc] = (cc == lane) ? 1.0 : 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        if (e < kb) {
            const double le = (lane > e) ? row[e] : 0.0;
#pragma unroll
            for (int cc = 0; cc <= e; ++cc) {
                const double ie = readlane_d(inv[cc], e);
                inv[cc] -= le * ie;
            }
        }
    }
    const double rdp = 1.0 / dpiv;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc)
        if (lane < 16) W[cc * 16 + lane] = (T)((own && cc < kb && cc <= lane) ? inv[cc] * rdp : 0.0);
#pragma unroll
    for (int cc = 0; cc < 16; ++cc)
        if (own && cc < kb && cc <= lane) Ap[(int64_t)cc * ldA + lane] = (T)((cc == lane) ? dpiv : row[cc]);
    if (own) Dd[lane] = (T)dpiv;
#pragma unroll
    for (int q = 0; q < kMaxNrhs; ++q)
        if (own && q < nrhs) yv_base[(int64_t)q * ldy + lane] = yv[q];
}

// Rank-kdim update of the lower triangle of an nrows x ncols block through LDS:
//   Cout(r, c) = Cin(r, c) - sum_{j < kdim} A(r, j) dv(j) A(c, j),   r >= c,
// with A(r, j) at A[j lda + r] and C(r, c) at C[c ldc + r].  The block is
// covered by kTileM x TN tiles (column tiles from the left, row tiles from the
// diagonal down), all processed in one software pipeline: 16-column slabs of A
// (scaled by dv) for the tile rows and columns are staged in LDS
// (double-buffered, one barrier per slab); each step issues the next slab's
// global loads first, runs the MFMAs of the current slab while they are in
// flight, and stages the next slab at its end.  Loads are unconditional at
// clamped addresses; rows and columns past the block only reach outputs that
// are never written, and columns past kdim are zeroed through dv.  Each wave
// computes a 64 x TN/2 quarter of a tile as 4 x TN/32 MFMA tiles.  Every
// thread of the workgroup must call it; it ends with a barrier.
static_assert(kTileLdsElems == 2 * kTileSlab * 2 * kTileStride, "tile update LDS size");
template <typename T, int TN>
struct TileRegs {
    T a[8], b[TN / 16], d[4];
    int j0;  // first column of the slab
};
// global-address-space view of a workspace pointer: its loads count only on
// the vector-memory counter, so the LDS waits before the MFMAs do not also wait
// for prefetches in flight (generic pointers give flat loads, which count on both)
template <typename T>
__device__ inline const __attribute__((address_space(1))) T* as_global(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}
// wave-uniform copies of values a non-inlined function receives in vector
// registers: with them the compiler keeps loop bounds and addresses scalar, so
// loops stay uniform and its wait counts across loop edges stay exact
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uni(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename P>
__device__ inline P* uni(P* p) {
    return (P*)(uintptr_t)uni((int64_t)(uintptr_t)p);
}

// walk of the tiles: column tiles c0 = 0, TN, ...; row tiles r0 = c0, c0 + kTileM, ...
template <int TN>
struct TileCursor {
    int r0, c0;
    __device__ inline void next(int nrows) {
        r0 += kTileM;
        if (r0 >= nrows) {
            c0 += TN;
            r0 = c0;
        }
    }
};
template <typename T, int TN>
__device__ __attribute__((noinline)) void tiles_update(const T* A, const T* dv, int64_t lda, int kdim, const T* Cin,
                                                       T* Cout, int64_t ldc, int nrows, int ncols, T* lds) {
    static_assert(TN == 64 || TN == 128, "tile width");
    typedef Mfma16<T> M;
    constexpr int NB = TN / 64;   // B rows per loader thread and column
    constexpr int WT = TN / 32;   // MFMA column tiles per wave
    A = uni(A);
    dv = uni(dv);
    lda = uni(lda);
    kdim = uni(kdim);
    Cin = uni(Cin);
    Cout = uni(Cout);
    ldc = uni(ldc);
    nrows = uni(nrows);
    ncols = uni(ncols);  // (lds stays as passed: its LDS address space is inferred from the caller)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = tid & 63, lj = (tid >> 6) * 4;
    constexpr int BUF = kTileSlab * 2 * kTileStride;
    const auto* Ag = as_global(A);
    const auto* dg = as_global(dv);
    // slab count rounded up to even: slabs past kdim are zeros
    const int ns = 2 * ((kdim + 2 * kTileSlab - 1) / (2 * kTileSlab));
    // load side of the pipeline: tile and slab of the next load; once every
    // slab is loaded it stays on the last one (loaded again, never computed)
    TileCursor<TN> lc{0, 0};
    int ls = 0;
    auto load = [&](TileRegs<T, TN>& R) {
        const int j0 = kTileSlab * ls;
        R.j0 = j0;
        const int ra0 = min(lc.r0 + lr, nrows - 1), ra1 = min(lc.r0 + lr + 64, nrows - 1);
        int rb[NB];
#pragma unroll
        for (int h = 0; h < NB; ++h) rb[h] = min(lc.c0 + lr + 64 * h, ncols - 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = min(j0 + lj + q, kdim - 1);
            const auto* Aj = Ag + (int64_t)j * lda;
            R.a[q] = Aj[ra0];
            R.a[4 + q] = Aj[ra1];
#pragma unroll
            for (int h = 0; h < NB; ++h) R.b[4 * h + q] = Aj[rb[h]];
            R.d[q] = dg[j];
        }
        // advance with selects only: a branch here would split the loop body
        // and make the compiler drain the loads in flight
        const bool wrap = ls + 1 == ns;
        const bool colwrap = lc.r0 + kTileM >= nrows;
        const int nc0 = colwrap ? lc.c0 + TN : lc.c0;
        const int nr0 = colwrap ? nc0 : lc.r0 + kTileM;
        const bool more = nc0 < ncols;
        lc.r0 = (wrap && more) ? nr0 : lc.r0;
        lc.c0 = (wrap && more) ? nc0 : lc.c0;
        ls = wrap ? (more ? 0 : ns - 1) : ls + 1;
    };
    auto store = [&](const TileRegs<T, TN>& R, int buf) {
        T* As = lds + buf * BUF;
        T* Bs = As + kTileSlab * kTileStride;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T dq = R.j0 + lj + q < kdim ? R.d[q] : T(0);  // columns past kdim
            As[(lj + q) * kTileStride + lr] = R.a[q] * dq;
            As[(lj + q) * kTileStride + lr + 64] = R.a[4 + q] * dq;
#pragma unroll
            for (int h = 0; h < NB; ++h) Bs[(lj + q) * kTileStride + lr + 64 * h] = R.b[4 * h + q];
        }
    };
    typename M::V acc[4][WT];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w2 = 0; w2 < WT; ++w2) acc[u][w2] = M::zero();
    const int wr = 64 * (wave >> 1), wc = (TN / 2) * (wave & 1);
    auto compute = [&](int buf) {
        const T* As = lds + buf * BUF;
        const T* Bs = As + kTileSlab * kTileStride;
#pragma unroll
        for (int ks = 0; ks < kTileSlab / 4; ++ks) {
            const int kk = 4 * ks + (lane >> 4);
            T av[4], bv[WT];
#pragma unroll
            for (int u = 0; u < 4; ++u) av[u] = As[kk * kTileStride + wr + 16 * u + (lane & 15)];
#pragma unroll
            for (int w2 = 0; w2 < WT; ++w2) bv[w2] = Bs[kk * kTileStride + wc + 16 * w2 + (lane & 15)];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int w2 = 0; w2 < WT; ++w2) acc[u][w2] = M::mma(av[u], bv[w2], acc[u][w2]);
        }
    };
    // one pipeline step: the next slab's loads are issued first, the MFMAs of
    // LDS buffer buf run while they are in flight, and the slab is staged into
    // the other buffer at the end (no load stays in flight across steps)
    auto step = [&](int buf, TileRegs<T, TN>& R) {
        load(R);
        __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
        compute(buf);
        __builtin_amdgcn_sched_barrier(0);  // and the staging (which waits for it) behind them
        store(R, buf ^ 1);
        __syncthreads();
    };
    TileRegs<T, TN> R0;
    if (ns > 0) {  // kdim = 0: Cout = Cin
        load(R0);
        store(R0, 0);
    }
    __syncthreads();
    for (TileCursor<TN> cc{0, 0}; cc.c0 < ncols; cc.next(nrows)) {
        for (int s = 0; s < ns; s += 2) {
            step(0, R0);
            step(1, R0);
        }
        const int nr = nrows - cc.r0, nc = ncols - cc.c0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int w2 = 0; w2 < WT; ++w2) {
                const int col = wc + 16 * w2 + (lane & 15);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = wr + 16 * u + M::row(lane, v);
                    if (rr < nr && col < nc && cc.r0 + rr >= cc.c0 + col) {
                        const int64_t o = (int64_t)(cc.c0 + col) * ldc + cc.r0 + rr;
                        Cout[o] = Cin[o] - acc[u][w2][v];
                    }
                }
                acc[u][w2] = M::zero();
            }
    }
}

// Multifrontal LDL^T of K_ff with nrhs right-hand sides in c.rhs (node-major
// [dof][nrhs]); forward substitution fused.  Returns via sm.flag = 2 on a
// vanishing pivot.  Fronts in global memory (any size) in the factor type T;
// lds holds the staged slabs of tile_update.
template <int D, typename T>
__device__ __attribute__((noinline)) void factorize_glb(const RveCtx& c, Smem& sm, int nrhs, T* lds) {
    typedef Mfma16<T> M;
    constexpr int NEN = 1 << D, ND = NEN * D;
    const DevPlan& pl = *c.plan;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if constexpr (NWAVE != 4) {
        // the global-front tiles are laid out for four waves; the host launches
        // the eight-wave solver for LDS plans only, and anything else fails here
        if (tid == 0) sm.flag = 2;
        __syncthreads();
        return;
    }
    T* W = reinterpret_cast<T*>(sm.red);  // 16 x 16
    nrhs = uni(nrhs);
    double* const cL = uni(c.L);
    double* const cU = uni(c.U);
    double* const cS = uni(c.S);
    PROF_T0();
    const int nfront = uni(pl.nfront);
    for (int s = 0; s < nfront; ++s) {
        const DevFront fr = pl.fronts[s];
        const int m = uni(fr.m), p = uni(fr.p), mu = m - p;
        const int32_t* rows = uni(pl.rows + fr.rows_off);
        T* Fp = reinterpret_cast<T*>(cL + uni(fr.L_off));
        T* Dg = reinterpret_cast<T*>(cL + uni(fr.D_off));
        double* y = cL + uni(fr.y_off);
        T* Us = reinterpret_cast<T*>(cS);
        double* rus = urhs<T>(cS, mu);
        // 1. zero the parts that are read later (the panel on and below its
        //    diagonal, the lower triangle of U_s), load the pivot rhs
        for (int j = wave; j < p; j += NWAVE)
            for (int i = j + lane; i < m; i += 64) Fp[(int64_t)j * m + i] = T(0);
        for (int k = wave; k < mu; k += NWAVE)
            for (int i = k + lane; i < mu; i += 64) Us[(int64_t)k * mu + i] = T(0);
        for (int t = threadIdx.x; t < mu * nrhs; t += NT) rus[t] = 0.0;
        for (int t = threadIdx.x; t < p * nrhs; t += NT) {
            int j = t % p, col = t / p;
            y[t] = c.rhs[(int64_t)rows[j] * nrhs + col];
        }
        __syncthreads();
        // 2. original entries K(b, a) of the pivot nodes a
        const int nk = (fr.kmap_end - fr.kmap_begin) * D * D;
        for (int t = threadIdx.x; t < nk; t += NT) {
            const KPair kp = pl.kpair[fr.kmap_begin + t / (D * D)];
            const int k = (t % (D * D)) / D, l = t % D;
            const int r = kp.row_node * D + k, col = kp.col_node * D + l;
            if (r < col) continue;
            // at most 2^d elements share a node pair: every contribution's loads
            // are issued together (clamped, zeros selected; the sum order is kept)
            KContrib cbs[NEN];
#pragma unroll
            for (int q = 0; q < NEN; ++q) cbs[q] = pl.kcontrib[kp.c_begin + min(q, kp.c_count - 1)];
            double v = 0;
#pragma unroll
            for (int q = 0; q < NEN; ++q) {
                const double kv = (double)ke_of<D, 1, T>(c)[((int64_t)cbs[q].elem * ND + cbs[q].lb * D + k) * ND +
                                                         cbs[q].la * D + l];
                v += (q < kp.c_count) ? kv : 0.0;
            }
            Fp[(int64_t)col * m + r] = (T)v;
            if (r == col) Dg[col] = (T)v;
        }
        __syncthreads();
        // 3. extend-add of the children's update matrices and rhs updates
        for (int q = fr.child_begin; q < fr.child_end; ++q) {
            const DevFront ch = pl.fronts[pl.children[q]];
            const int mc = ch.m - ch.p;
            const int32_t* rel = pl.relind + ch.relind_off;
            const T* Uc = reinterpret_cast<const T*>(c.U + ch.U_off);
            const double* ruc = urhs<T>(c.U + ch.U_off, mc);
            // lower triangle, 8 columns per pass: a thread first issues the 8
            // loads of its row, then the 8 read-modify-writes, so each pass costs
            // two memory round trips instead of sixteen
            for (int k0 = 0; k0 < mc; k0 += 8) {
                int Ck[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) Ck[u] = rel[min(k0 + u, mc - 1)];
                for (int i = k0 + threadIdx.x; i < mc; i += NT) {
                    const int R = rel[i];
                    T v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = Uc[(int64_t)min(k0 + u, mc - 1) * mc + i];
                    T* dstp[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int C = Ck[u];
                        dstp[u] = C < p ? Fp + (int64_t)C * m + R : Us + (int64_t)(C - p) * mu + (R - p);
                    }
                    T old[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) old[u] = (k0 + u < mc && i >= k0 + u) ? *dstp[u] : T(0);
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (k0 + u < mc && i >= k0 + u) *dstp[u] = old[u] + v[u];
                }
            }
            for (int t = threadIdx.x; t < mc * nrhs; t += NT) {
                const int i = t % mc, col = t / mc;
                const int R = rel[i];
                const double v = ruc[(int64_t)col * mc + i];
                if (R < p) y[(int64_t)col * p + R] += v;
                else rus[(int64_t)col * mu + (R - p)] += v;
            }
            __syncthreads();
        }
        PROF_MARK(PH_ASM);
        // 4. panel LDL^T in 64-column blocks (left-looking), forward rhs.  A
        // block first takes the updates of all columns left of it as LDS tiles,
        // then its four 16-column sub-blocks are factored in turn.
        for (int K64 = 0; K64 < p; K64 += 64) {
            const int kb64 = min(64, p - K64);
            if (K64 > 0) {
                T* Ct = Fp + (int64_t)K64 * m + K64;
                tiles_update<T, 64>(Fp + K64, Dg, m, K64, Ct, Ct, m, m - K64, kb64, lds);
            }
            for (int K = K64; K < K64 + kb64; K += 16) {
                const int kb = min(16, p - K);
                // (a) updates of the earlier columns of the block:
                //     A(i, K + c) -= sum_{K64 <= j < K} L(i, j) D(j) L(K + c, j)
                if (K > K64) {
                    const int nt = (m - K + 15) >> 4;
                    for (int t0 = 2 * wave; t0 < nt; t0 += 2 * NWAVE) {
                        typename M::V acc[2] = {M::zero(), M::zero()};
                        const int cb = K + (lane & 15);
                        // at most 48 earlier columns in the block: unrolled to 12
                        // k-steps so that all operand loads are issued together
                        T av[12][2], bv[12];
#pragma unroll
                        for (int q = 0; q < 12; ++q) {
                            const int j = min(K64 + 4 * q + (lane >> 4), K - 1);
                            const T* colj = Fp + (int64_t)j * m;
                            bv[q] = colj[min(cb, m - 1)];
                            const T dj = Dg[j];
#pragma unroll
                            for (int u = 0; u < 2; ++u)
                                av[q][u] = colj[min(K + 16 * (t0 + u) + (lane & 15), m - 1)] * dj;
                        }
#pragma unroll
                        for (int q = 0; q < 12; ++q) {
                            if (K64 + 4 * q < K) {
                                const bool okb = (lane & 15) < kb;
#pragma unroll
                                for (int u = 0; u < 2; ++u) {
                                    const bool oka = K + 16 * (t0 + u) + (lane & 15) < m;
                                    acc[u] = M::mma(oka ? av[q][u] : T(0), okb ? bv[q] : T(0), acc[u]);
                                }
                            }
                        }
                        const int cc = lane & 15;
#pragma unroll
                        for (int u = 0; u < 2; ++u)
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int rr = K + 16 * (t0 + u) + M::row(lane, v);
                                if (t0 + u < nt && rr < m && cc < kb && rr >= K + cc)
                                    Fp[(int64_t)(K + cc) * m + rr] -= acc[u][v];
                            }
                    }
                    __syncthreads();
                }
                PROF_MARK(PH_MFMA);
                // (b) diagonal block and its rhs rows by wave 0
                if (wave == 0)
                    diag_block_wave<T>(Fp + (int64_t)K * m + K, m, Dg + K, Dg + K, kb, y + K, p, nrhs, W, &sm.flag);
                __syncthreads();
                PROF_MARK(PH_DIAG);
                // (c) rows below: L21 = A21 W (MFMA)
                const int R0 = K + kb;
                {
                    const int nt = (m - R0 + 15) >> 4;
                    for (int t = wave; t < nt; t += NWAVE) {
                        const int ra = R0 + 16 * t + (lane & 15);
                        typename M::V acc = M::zero();
#pragma unroll
                        for (int ks = 0; ks < 4; ++ks) {
                            const int kk = 4 * ks + (lane >> 4);
                            const T av = (kk < kb && ra < m) ? Fp[(int64_t)(K + kk) * m + ra] : T(0);
                            acc = M::mma(av, W[kk * 16 + (lane & 15)], acc);
                        }
                        const int cc = lane & 15;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int rr = R0 + 16 * t + M::row(lane, v);
                            if (rr < m && cc < kb) Fp[(int64_t)(K + cc) * m + rr] = acc[v];
                        }
                    }
                }
                __syncthreads();
                // (d) rhs of the rows below: b_i -= sum_c L(i, K + c) y(K + c),
                //     one row per thread for every column (the row's 16 L entries
                //     read once)
                for (int i = R0 + tid; i < m; i += NT) {
                    double lk[16];
#pragma unroll
                    for (int cc = 0; cc < 16; ++cc) lk[cc] = cc < kb ? (double)Fp[(int64_t)(K + cc) * m + i] : 0.0;
                    for (int q = 0; q < nrhs; ++q) {
                        const double* yq = y + (int64_t)q * p + K;
                        double acc = 0.0;
#pragma unroll
                        for (int cc = 0; cc < 16; ++cc)
                            if (cc < kb) acc += lk[cc] * yq[cc];
                        if (i < p) y[(int64_t)q * p + i] -= acc;
                        else rus[(int64_t)q * mu + (i - p)] -= acc;
                    }
                }
                __syncthreads();
                PROF_MARK(PH_TRSM);
            }
        }
        // 5. Schur complement U = U_s - L21 D L21^T over the tiles of its lower
        //    triangle, written straight onto the update stack with its rhs rows
        if (mu > 0) {
            T* dst = reinterpret_cast<T*>(cU + uni(fr.U_off));
            double* drhs = urhs<T>(cU + uni(fr.U_off), mu);
            tiles_update<T, 128>(Fp + p, Dg, m, p, Us, dst, mu, mu, mu, lds);
            for (int t = tid; t < mu * nrhs; t += NT) drhs[t] = rus[t];
        }
        __syncthreads();
        PROF_MARK(PH_OUT);
    }
}

// forward substitution L y = b with stored global-memory factors, for a new
// rhs b (node-major [dof][NRHS], FP64, overwritten): fronts in elimination
// order; per front the pivot rows are solved in 16-pivot blocks (readlane
// chain in wave 0) and folded into the rows below, whose update goes straight
// into b at the rows' dofs (each is a pivot of a later front); the pivot part
// is stored as the front's forward-substituted rhs for backsolve_glb.
template <int D, int NRHS, typename T>
__device__ __attribute__((noinline)) void forward_glb(const RveCtx& c, Smem& sm, double* b) {
    const DevPlan& pl = *c.plan;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* const cL = uni(c.L);
    b = uni(b);
    const int nfront = uni(pl.nfront);
    for (int s = 0; s < nfront; ++s) {
        const DevFront fr = pl.fronts[s];
        const int m = uni(fr.m), p = uni(fr.p);
        const int32_t* rows = uni(pl.rows + fr.rows_off);
        const T* Fp = reinterpret_cast<const T*>(cL + uni(fr.L_off));
        double* y = cL + uni(fr.y_off);
        for (int t = tid; t < p * NRHS; t += NT) {
            const int j = t % p, q = t / p;
            y[t] = b[(int64_t)rows[j] * NRHS + q];
        }
        __syncthreads();
        for (int K = 0; K < p; K += 16) {
            const int kb = min(16, p - K);
            if (wave == 0) {
                const bool own = lane < kb;
                double Lr[16];
#pragma unroll
                for (int cc = 0; cc < 16; ++cc)
                    Lr[cc] = (own && cc < kb && cc < lane) ? (double)Fp[(int64_t)(K + cc) * m + K + lane] : 0.0;
#pragma unroll
                for (int q = 0; q < NRHS; ++q) {
                    double vv = own ? y[(int64_t)q * p + K + lane] : 0.0;
#pragma unroll
                    for (int cc = 0; cc < 16; ++cc) {
                        if (cc < kb) {
                            const double yc = readlane_d(vv, cc);
                            if (lane > cc) vv -= Lr[cc] * yc;
                        }
                    }
                    if (own) y[(int64_t)q * p + K + lane] = vv;
                }
            }
            __syncthreads();
            for (int i = K + kb + tid; i < m; i += NT) {
                double lk[16];
#pragma unroll
                for (int cc = 0; cc < 16; ++cc) lk[cc] = (cc < kb) ? (double)Fp[(int64_t)(K + cc) * m + i] : 0.0;
#pragma unroll
                for (int q = 0; q < NRHS; ++q) {
                    double acc = 0.0;
#pragma unroll
                    for (int cc = 0; cc < 16; ++cc)
                        if (cc < kb) acc += lk[cc] * y[(int64_t)q * p + K + cc];
                    if (i < p) y[(int64_t)q * p + i] -= acc;
                    else b[(int64_t)rows[i] * NRHS + q] -= acc;
                }
            }
            __syncthreads();
        }
    }
}

// backward substitution L^T x = D^-1 y with global-memory factors; x
// node-major [dof][NRHS].  Per front: the update rows' contribution (thread
// per pivot), then 16-pivot blocks from the last: wave 0 solves the block
// triangle with readlane broadcasts, all threads fold the block into the
// earlier pivots.
template <int D, int NRHS, typename T>
__device__ __attribute__((noinline)) void backsolve_glb(const RveCtx& c, Smem& sm, double* xo) {
    const DevPlan& pl = *c.plan;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    zero_pinned<D>(c, xo, NRHS);
    __syncthreads();
    double* const cL = uni(c.L);
    xo = uni(xo);
    for (int s = uni(pl.nfront) - 1; s >= 0; --s) {
        const DevFront fr = pl.fronts[s];
        const int m = uni(fr.m), p = uni(fr.p);
        const int32_t* rows = uni(pl.rows + fr.rows_off);
        const T* Fp = reinterpret_cast<const T*>(cL + uni(fr.L_off));
        const T* Dg = reinterpret_cast<const T*>(cL + uni(fr.D_off));
        double* y = cL + uni(fr.y_off);
        for (int j = tid; j < p; j += NT) {
            const double rd = 1.0 / (double)Dg[j];
            double v[NRHS];
#pragma unroll
            for (int q = 0; q < NRHS; ++q) v[q] = y[(int64_t)q * p + j] * rd;
            const T* cj = Fp + (int64_t)j * m;
#pragma unroll 4
            for (int i = p; i < m; ++i) {
                const double l = (double)cj[i];
                const double* xr = xo + (int64_t)rows[i] * NRHS;
#pragma unroll
                for (int q = 0; q < NRHS; ++q) v[q] -= l * xr[q];
            }
#pragma unroll
            for (int q = 0; q < NRHS; ++q) y[(int64_t)q * p + j] = v[q];
        }
        __syncthreads();
        const int nb = (p + 15) >> 4;
        for (int bk = nb - 1; bk >= 0; --bk) {
            const int K = 16 * bk, kb = min(16, p - K);
            if (wave == 0) {
                const bool own = lane < kb;
                double Lr[16];
#pragma unroll
                for (int cc = 0; cc < 16; ++cc)
                    Lr[cc] = (own && cc < kb && cc > lane) ? (double)Fp[(int64_t)(K + lane) * m + K + cc] : 0.0;
#pragma unroll
                for (int q = 0; q < NRHS; ++q) {
                    double vv = own ? y[(int64_t)q * p + K + lane] : 0.0;
#pragma unroll
                    for (int cc = 15; cc >= 0; --cc) {
                        if (cc < kb) {
                            const double xc = readlane_d(vv, cc);
                            if (lane < cc) vv -= Lr[cc] * xc;
                        }
                    }
                    if (own) y[(int64_t)q * p + K + lane] = vv;
                }
            }
            __syncthreads();
            for (int j = tid; j < K; j += NT) {
                const T* cj = Fp + (int64_t)j * m + K;
                double lk[16];
#pragma unroll
                for (int cc = 0; cc < 16; ++cc) lk[cc] = (cc < kb) ? (double)cj[cc] : 0.0;
#pragma unroll
                for (int q = 0; q < NRHS; ++q) {
                    double acc = y[(int64_t)q * p + j];
#pragma unroll
                    for (int cc = 0; cc < 16; ++cc)
                        if (cc < kb) acc -= lk[cc] * y[(int64_t)q * p + K + cc];
                    y[(int64_t)q * p + j] = acc;
                }
            }
            __syncthreads();
        }
        for (int t = tid; t < p * NRHS; t += NT) {
            const int j = t % p, q = t / p;
            xo[(int64_t)rows[j] * NRHS + q] = y[(int64_t)q * p + j];
        }
        __syncthreads();
    }
}

// Multifrontal LDL^T, fronts in LDS (F: packed front, rl: m x nrhs rhs rows).
// Small subtrees first, one front per wave (wave_front); then the workgroup
// fronts in the plan's steps of 1, 2 or 4 independent fronts side by side
// (wg_front).  Per pivot block of 16 columns: a row-owner sweep (one barrier per
// pivot) gives the 16 L columns of every row and the forward-substituted rhs;
// the trailing lower triangle is then updated with v_mfma_f64_16x16x4 (lane
// layouts: A[l%16][l/16], B[l/16][l%16], D row = l/16 + 4 v, col = l%16).


// Original entries of an LDS front from the element matrices (one gather level)
// and the extend-add of a child's packed update matrix: U strides of the list
// per pass, every index load first, then every value load (clamped addresses,
// zeros selected), then the stores, so a pass costs one or two memory round
// trips for all its strides.  first / stride: the caller's lane (wave-level) or
// thread (workgroup-level) numbering.  D0 (LDS) receives the original diagonal
// of the pivot columns, the scale of the vanishing-pivot test.
template <int NEN, int U = 4, typename KT, typename T>
__device__ inline void gather_original(const DevPlan& pl, const KT* ke, int a0, int a1, int first, int stride,
                                       T* F, int m, T* D0) {
    for (int t0 = a0 + first; t0 < a1; t0 += U * stride) {
        int rc[U], src[U][NEN];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = min(t0 + u * stride, a1 - 1);
            rc[u] = pl.asm_rc[t];
#pragma unroll
            for (int q = 0; q < NEN; ++q) src[u][q] = pl.asm_src[(int64_t)t * NEN + q];
        }
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v[u] = 0.0;
#pragma unroll
            for (int q = 0; q < NEN; ++q) {
                const double kv = (double)ke[max(src[u][q], 0)];
                v[u] += (src[u][q] >= 0) ? kv : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (t0 + u * stride < a1) {
                const int r = rc[u] >> 16, col = rc[u] & 0xffff;
                F[cpk(col, m) + r - col] = v[u];
                if (r == col) D0[col] = v[u];
            }
        }
    }
}
// global -> LDS copy, eight strides per pass: all loads first, then all stores
// (the compiler does not move a load past a store that may alias it)
template <typename T>
__device__ inline void copy_in(T* dst, const T* src, int n, int first, int stride) {
    for (int t0 = first; t0 < n; t0 += 8 * stride) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[min(t0 + u * stride, n - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (t0 + u * stride < n) dst[t0 + u * stride] = v[u];
    }
}
template <int U = 8, typename T>
__device__ inline void extend_add_packed(const int32_t* ea, const T* Uc, int nu, int first, int stride, T* F) {
    for (int t0 = first; t0 < nu; t0 += U * stride) {
        int e[U];
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = min(t0 + u * stride, nu - 1);
            e[u] = ea[t];
            v[u] = Uc[t];
        }
        // the targets of a pass are distinct (a child adds to each parent entry
        // once; clamped duplicates are read, never written): every target is read
        // before any is written, one LDS round trip per pass
        T o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) o[u] = F[e[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t0 + u * stride < nu) F[e[u]] = o[u] + v[u];
    }
}

// One small front (m <= 64) processed by a single wave: lane i owns front row i.
// Assembly as in the workgroup path, then a right-looking LDL^T sweep over the
// p pivots done in place in LDS (the wave's slice: front, rhs rows, original
// diagonal); within a wave LDS accesses complete in issue order, so no barrier
// is needed between pivots.
template <int D, int NRHS, typename T>
__device__ void wave_front(const RveCtx& c, Smem& sm, int s, T* F, T* rl) {
    const DevPlan& pl = *c.plan;
    constexpr int NEN = 1 << D;
    const int lane = threadIdx.x & 63;
    const DevFront fr = pl.fronts[uni(s)];  // (uniform per wave: scalar loads)
    const int m = uni(fr.m), p = uni(fr.p), mu = m - p;
    const int32_t* rows = pl.rows + fr.rows_off;
    T* Lg = reinterpret_cast<T*>(c.L + fr.L_off);
    double* Dg = c.L + fr.D_off;
    double* yg = c.L + fr.y_off;
    const int tot = cpk(m, m);
    // the rhs rows (lane = row, m <= 64) are loaded first and stored after the
    // gather, so their two round trips overlap the gather's; the gather takes
    // eight strides per pass (one pass for the usual front), and a child's rhs
    // rows travel with its update matrix, sixteen strides per pass
    T rv[NRHS];
    {
        const int ri = rows[min(lane, m - 1)];  // (the value is used on the pivot rows only)
#pragma unroll
        for (int q = 0; q < NRHS; ++q) rv[q] = lane < p ? (T)c.rhs[(int64_t)ri * NRHS + q] : T(0);
    }
    for (int t = lane; t < tot; t += 64) F[t] = 0.0;
    __builtin_amdgcn_wave_barrier();
    T* const D0 = rl + m * NRHS;
    gather_original<NEN, 8>(pl, ke_of<D, NRHS, T>(c), fr.asm_begin, fr.asm_end, lane, 64, F, m, D0);
    if (lane < m)
#pragma unroll
        for (int q = 0; q < NRHS; ++q) rl[q * m + lane] = rv[q];
    __builtin_amdgcn_wave_barrier();
    for (int q = fr.child_begin; q < fr.child_end; ++q) {
        const DevFront ch = pl.fronts[pl.children[q]];
        const int mc = ch.m - ch.p;  // < 64: the child is a wave front too
        const int32_t* rel = pl.relind + ch.relind_off;
        const T* Uc = reinterpret_cast<const T*>(c.U + ch.U_off);
        const int nu = cpk(mc, mc);
        const T* ruc = Uc + nu;
        const int32_t* ea = pl.ea_dst + ch.ea_off;
        const int li = max(min(lane, mc - 1), 0);
        const int ci = mc > 0 ? rel[li] : 0;
        T cr[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) cr[k] = mc > 0 ? ruc[(int64_t)k * mc + li] : T(0);
        extend_add_packed<16>(ea, Uc, nu, lane, 64, F);
        if (lane < mc)
#pragma unroll
            for (int k = 0; k < NRHS; ++k) rl[k * m + ci] += cr[k];
        __builtin_amdgcn_wave_barrier();
    }
    for (int K = 0; K < p; K += 16) {
        const int kb = min(16, p - K);
        // the 16 columns of the block by elimination on every front row at once
        // (lane = row, rows below the block included): readlane broadcasts of
        // the pivot and of the block rows' multipliers; the rows below leave
        // with their L entries and forward-substituted rhs
        {
            const int r = lane;
            const bool act = r >= K && r < m;
            T row[16];
            T yv[NRHS];
            // (clamped reads inside the front, masked: no branch per entry)
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) {
                const int col = min(K + cc, m - 1);
                const int idx = min(max(cpk(col, m) + r - col, 0), cpk(m, m) - 1);
                row[cc] = F[idx] * ((act && cc < kb && K + cc <= r) ? T(1) : T(0));
            }
            // (clamped reads; lanes off the front never store or broadcast these,
            // and only the pivot's own lane tests its d0)
#pragma unroll
            for (int q = 0; q < NRHS; ++q) yv[q] = rl[q * m + min(r, m - 1)];
            const double d0 = (double)D0[min(r, m - 1)];
            T mypiv = T(1);  // the pivot of this lane's row, tested after the block
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (j < kb) {
                    const T piv = readlane_t(row[j], K + j);
                    const T rp = recip_t(piv);
                    mypiv = r == K + j ? piv : mypiv;
                    const bool below = act && r > K + j;
                    const T l = below ? row[j] * rp : T(0);
                    const T lpv = l * piv;
                    // unconditional updates, past the block bound too (lane K + cc
                    // <= 63 since K <= 48): l = 0 off the rows below the pivot, and
                    // the only other entries touched, row[cc] with K + cc > r or
                    // cc >= kb, lie above the diagonal or outside the block and are
                    // neither stored nor read as a pivot
#pragma unroll
                    for (int cc = j + 1; cc < 16; ++cc) {
                        const T lc = readlane_t(l, K + cc);
                        row[cc] -= lpv * lc;
                    }
#pragma unroll
                    for (int q = 0; q < NRHS; ++q) {
                        const T yj = readlane_t(yv[q], K + j);
                        yv[q] -= l * yj;
                    }
                    if (below) row[j] = l;
                }
            }
            if (r >= K && r < K + kb &&
                (!(fabs((double)mypiv) > 1e-14 * fabs(d0)) || !isfinite((double)mypiv)))
                sm.flag = 2;
#pragma unroll
            for (int cc = 0; cc < 16; ++cc)
                if (act && cc < kb && K + cc <= r) F[cpk(K + cc, m) + r - K - cc] = row[cc];
#pragma unroll
            for (int q = 0; q < NRHS; ++q)
                if (act) rl[q * m + r] = yv[q];
        }
        __builtin_amdgcn_wave_barrier();
        const int R0 = K + kb;
        const int nRT = (m - R0 + 15) >> 4;
        // trailing lower triangle -= L D L^T (MFMA), two independent tiles in flight
        const int nT = nRT;
        const int ntile = nT * (nT + 1) / 2;
        // (MFMA of the factor type: v_mfma_f64_16x16x4 or v_mfma_f32_16x16x4)
        typedef Mfma16<T> M;
        for (int t0 = 0; t0 < ntile; t0 += 2) {
            typename M::V acc[2];
            int Ii[2], Jj[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                int I = 0, rem = t0 + u;
                while (rem > I) { rem -= I + 1; ++I; }
                Ii[u] = I;
                Jj[u] = rem;
                acc[u] = M::zero();
            }
            // operands from clamped addresses inside the front (column K and row
            // m - 1 stand in past the block, the front or the last tile) times 0/1
            // masks: every read of both tiles issues without branches
            T av[4][2], bv[4][2];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int kk = 4 * ks + (lane >> 4);
                const int kc = kk < kb ? K + kk : K;
                const int base = cpk(kc, m) - kc;
                const T dk = F[base + kc];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int ra = R0 + 16 * Ii[u] + (lane & 15), rb = R0 + 16 * Jj[u] + (lane & 15);
                    const bool live = (t0 + u < ntile) && kk < kb;
                    const T ma = (live && ra < m) ? T(1) : T(0), mb = (live && rb < m) ? T(1) : T(0);
                    av[ks][u] = F[base + min(ra, m - 1)] * dk * ma;
                    bv[ks][u] = F[base + min(rb, m - 1)] * mb;
                }
            }
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                for (int u = 0; u < 2; ++u) acc[u] = M::mma(av[ks][u], bv[ks][u], acc[u]);
            // the tiles' targets are distinct: all eight read (clamped), then written
            T o[2][4];
            int bs[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int cc = R0 + 16 * Jj[u] + (lane & 15), ccl = min(cc, m - 1);
                bs[u] = cpk(ccl, m) - ccl;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = R0 + 16 * Ii[u] + M::row(lane, v);
                    o[u][v] = F[bs[u] + min(max(rr, ccl), m - 1)];
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int cc = R0 + 16 * Jj[u] + (lane & 15);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = R0 + 16 * Ii[u] + M::row(lane, v);
                    if (t0 + u < ntile && cc < m && rr < m && rr >= cc) F[bs[u] + rr] = o[u][v] - acc[u][v];
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    const int lp = cpk(p, m);
    for (int t = lane; t < lp; t += 64) Lg[t] = F[t];
    for (int t = lane; t < p; t += 64) Dg[t] = F[cpk(t, m)];
    for (int t = lane; t < p * NRHS; t += 64) {
        const int j = t % p, col = t / p;
        yg[t] = rl[col * m + j];
    }
    if (mu > 0) {
        T* dst = reinterpret_cast<T*>(c.U + fr.U_off);
        const int usz = tot - lp;
        for (int t = lane; t < usz; t += 64) dst[t] = F[lp + t];
        for (int t = lane; t < mu * NRHS; t += 64) {
            const int ii = t % mu, col = t / mu;
            dst[usz + t] = rl[col * m + p + ii];
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// One workgroup front s on threads gt = 0..GT-1 and waves gw = 0..nw-1 (the
// whole workgroup, or one half of it beside a second front): assembly into the
// packed front F and rhs rows rl (original diagonal after them), 16-pivot blocks
// (row-owner sweep, one barrier per pivot, publication in pub; trailing lower
// triangle on MFMA), then L, D, y and the update matrix out.  Every barrier is
// workgroup-wide: fronts sharing a step have equal pivot and child counts, so
// both halves pass the same sequence of barriers.
template <int D, int NRHS, typename T>
__device__ inline void wg_front(const RveCtx& c, Smem& sm, int s, T* F, T* rl, int gt, int GT, int gw, int nw,
                                double (*pub)[18 + kMaxNrhs]) {
    constexpr int nrhs = NRHS;
    constexpr int NEN = 1 << D;
    const DevPlan& pl = *c.plan;
    const int lane = threadIdx.x & 63;
    PROF_T0();
    const DevFront fr = pl.fronts[uni(s)];  // (uniform per wave: scalar loads)
    const int m = uni(fr.m), p = uni(fr.p), mu = m - p;
    const int32_t* rows = pl.rows + fr.rows_off;
    T* Lg = reinterpret_cast<T*>(c.L + fr.L_off);
    double* Dg = c.L + fr.D_off;
    double* yg = c.L + fr.y_off;
    const int tot = cpk(m, m);
    for (int t = gt; t < tot; t += GT) F[t] = 0.0;
    for (int t = gt; t < m * nrhs; t += GT) {
        const int i = t % m, col = t / m;
        rl[t] = (i < p) ? c.rhs[(int64_t)rows[i] * nrhs + col] : 0.0;
    }
    __syncthreads();
    // original entries: one gather level, every source load in flight at once
    T* const D0 = rl + m * nrhs;  // original diagonal, after the rhs rows
    gather_original<NEN>(pl, ke_of<D, NRHS, T>(c), fr.asm_begin, fr.asm_end, gt, GT, F, m, D0);
    __syncthreads();
    for (int q = fr.child_begin; q < fr.child_end; ++q) {
        const DevFront ch = pl.fronts[pl.children[q]];
        const int mc = ch.m - ch.p;
        const int32_t* rel = pl.relind + ch.relind_off;
        const T* Uc = reinterpret_cast<const T*>(c.U + ch.U_off);
        const int nu = cpk(mc, mc);
        const T* ruc = Uc + nu;
        const int32_t* ea = pl.ea_dst + ch.ea_off;
        extend_add_packed(ea, Uc, nu, gt, GT, F);
        for (int t = gt; t < mc * nrhs; t += GT) {
            const int i = t % mc, col = t / mc;
            rl[col * m + rel[i]] += ruc[(int64_t)col * mc + i];
        }
        __syncthreads();
    }
    PROF_MARK(PH_ASM);
    for (int K = 0; K < p; K += 16) {
        const int kb = min(16, p - K);
        // ---- pivot block sweep: each front row below K is owned by one thread
        // that keeps its 16 block entries in registers; at pivot j the owners of
        // the block rows publish pivot, reciprocal, column-j entries and the
        // forward-substituted rhs (double-buffered, one barrier per pivot)
        const int i = K + gt;
        const bool own = i < m;
        T r[16];
        T b[NRHS];
        // (clamped reads inside the front, masked or unused: rows off the front
        // never publish, update or store these, and only a pivot's owner tests
        // its d0)
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            const int col = min(K + cc, m - 1);
            const int idx = min(max(cpk(col, m) + min(i, m - 1) - col, 0), cpk(m, m) - 1);
            r[cc] = F[idx] * ((own && cc < kb && K + cc <= i) ? T(1) : T(0));
        }
#pragma unroll
        for (int q = 0; q < NRHS; ++q) b[q] = rl[q * m + min(i, m - 1)];
        const double d0 = (double)D0[min(i, m - 1)];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (j < kb) {
                // [0] piv, [1] 1/piv, [2..17] g, [18..] y, in the factor type
                T* P = reinterpret_cast<T*>(pub[j & 1]);
                if (i == K + j) {
                    const T piv = r[j];
                    if (!(fabs((double)piv) > 1e-14 * fabs(d0)) || !isfinite((double)piv)) sm.flag = 2;
                    P[0] = piv;
                    P[1] = recip_t(piv);
#pragma unroll
                    for (int q = 0; q < NRHS; ++q) P[18 + q] = b[q];
                } else if (i > K + j && i < K + kb) {
                    P[2 + i - K] = r[j];
                }
                __syncthreads();
                if (own && i > K + j) {
                    const T l = r[j] * P[1];
                    // every P entry is read (all within the buffer; entries past the
                    // block are stale) and the multiplier selected, so the reads
                    // need no branch of their own: r[cc] above the row's diagonal
                    // (K + cc > i) is neither stored nor read, so only the block
                    // bound masks the update
#pragma unroll
                    for (int cc = j + 1; cc < 16; ++cc) {
                        const T lc = cc < kb ? l : T(0);
                        r[cc] -= lc * P[2 + cc];
                    }
                    r[j] = l;
#pragma unroll
                    for (int q = 0; q < NRHS; ++q) b[q] -= l * P[18 + q];
                }
            }
        }
        if (own) {
#pragma unroll
            for (int cc = 0; cc < 16; ++cc)
                if (cc < kb && K + cc <= i) F[cpk(K + cc, m) + i - K - cc] = r[cc];
#pragma unroll
            for (int q = 0; q < NRHS; ++q) rl[q * m + i] = b[q];
        }
        __syncthreads();
        PROF_MARK(PH_DIAG);
        // ---- trailing lower triangle (rows, cols >= T0) -= L D L^T with MFMA
        const int T0 = K + kb;
        const int nT = (m - T0 + 15) >> 4;
        const int ntile = nT * (nT + 1) / 2;
        for (int tix = gw; tix < ntile; tix += nw) {
            int I = 0, rem = tix;
            while (rem > I) { rem -= I + 1; ++I; }
            const int J = rem;
            const int ra = T0 + 16 * I + (lane & 15), rb = T0 + 16 * J + (lane & 15);
            // operands from clamped addresses inside the front (column K and row
            // m - 1 stand in past the block or the front) times 0/1 masks, so all
            // twelve reads issue together without branches
            // (MFMA of the factor type: v_mfma_f64_16x16x4 or v_mfma_f32_16x16x4)
            typedef Mfma16<T> M;
            T a[4], bb[4];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int kk = 4 * ks + (lane >> 4);
                const int kc = kk < kb ? K + kk : K;
                const int base = cpk(kc, m) - kc;
                const T dk = F[base + kc];
                const T ma = (kk < kb && ra < m) ? T(1) : T(0), mb = (kk < kb && rb < m) ? T(1) : T(0);
                a[ks] = F[base + min(ra, m - 1)] * dk * ma;
                bb[ks] = F[base + min(rb, m - 1)] * mb;
            }
            typename M::V acc = M::zero();
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) acc = M::mma(a[ks], bb[ks], acc);
            // the tile's targets are distinct: all four read (clamped), then written
            const int cc = T0 + 16 * J + (lane & 15), ccl = min(cc, m - 1);
            const int base = cpk(ccl, m) - ccl;
            T o[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = T0 + 16 * I + M::row(lane, v);
                o[v] = F[base + min(max(rr, ccl), m - 1)];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = T0 + 16 * I + M::row(lane, v);
                if (cc < m && rr < m && rr >= cc) F[base + rr] = o[v] - acc[v];
            }
        }
        __syncthreads();
        PROF_MARK(PH_MFMA);
    }
    // L panel, D, y; update matrix (packed) and its rhs onto the stack
    const int lp = cpk(p, m);
    for (int t = gt; t < lp; t += GT) Lg[t] = F[t];
    for (int t = gt; t < p; t += GT) Dg[t] = F[cpk(t, m)];
    for (int t = gt; t < p * nrhs; t += GT) {
        const int j = t % p, col = t / p;
        yg[t] = rl[col * m + j];
    }
    if (mu > 0) {
        T* dst = reinterpret_cast<T*>(c.U + fr.U_off);
        const int usz = tot - lp;
        for (int t = gt; t < usz; t += GT) dst[t] = F[lp + t];
        for (int t = gt; t < mu * nrhs; t += GT) {
            const int i = t % mu, col = t / mu;
            dst[usz + t] = rl[col * m + p + i];
        }
    }
    __syncthreads();
    PROF_MARK(PH_OUT);
}

template <int D, int NRHS, typename T>
__device__ __noinline__ void factorize_lds(const RveCtx& c, Smem& sm, T* F, T* rl, int wave_slice) {
    constexpr int nrhs = NRHS;
    const DevPlan& pl = *c.plan;
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    PROF_T0();
    // small subtrees: one front per wave, all fronts of one height at a time
    for (int h = 0; h < pl.nwave_h; ++h) {
        T* Fw = F + (int64_t)wave * wave_slice;
        for (int k = pl.wave_hbeg[h] + wave; k < pl.wave_hbeg[h + 1]; k += NWAVE) {
            const int sw = pl.wave_list[k];
            const int mw = pl.fronts[sw].m;
            wave_front<D, NRHS, T>(c, sm, sw, Fw, Fw + cpk(mw, mw));
        }
        __syncthreads();
    }
    PROF_MARK(PH_TRSM);
    // workgroup fronts: one per step on the whole workgroup, or nf = 2 or 4 side
    // by side on G equal groups of threads (at least 128 each; with fewer groups
    // than fronts each group takes nf / G of them in turn), front k's storage
    // after the rhs rows of fronts 0..k-1
    for (int st = 0; st < pl.nwg_steps; ++st) {
        const int32_t* e = pl.wg_steps + kStepFronts * st;
        const int nf = e[3] >= 0 ? 4 : (e[1] >= 0 ? 2 : 1);
        const int G = min(nf, NT / 128);
        const int GT = NT / G, NW = NWAVE / G, g = tid / GT;
        for (int r = 0; r < nf / G; ++r) {
            const int k = r * G + g;
            int off = 0;
            for (int j = 0; j < k; ++j) {
                const int mj = pl.fronts[e[j]].m;
                off += cpk(mj, mj) + mj * (nrhs + 1);
            }
            const int ms = pl.fronts[e[k]].m;
            T* const Fk = F + off;
            T* const rlk = nf > 1 ? Fk + cpk(ms, ms) : rl;
            wg_front<D, NRHS, T>(c, sm, e[k], Fk, rlk, tid - g * GT, GT, wave - g * NW, NW, sm.pub[g]);
        }
    }
}

// backward substitution of one small front (m <= 64) by one wave, lane j =
// pivot j: the packed panel is staged in the wave's LDS slice S, the update
// rows' solution values are loaded one per lane and broadcast by readlane, and
// the pivot triangle is swept from the last pivot (no barrier)
template <int D, int NRHS, typename T>
__device__ void backsolve_wave_front(const RveCtx& c, int s, T* S, double* x) {
    const DevPlan& pl = *c.plan;
    const int lane = threadIdx.x & 63;
    const DevFront fr = pl.fronts[uni(s)];  // (uniform per wave: scalar loads)
    const int m = uni(fr.m), p = uni(fr.p), mu = m - p;
    const int32_t* rows = pl.rows + fr.rows_off;
    const T* Lg = reinterpret_cast<const T*>(c.L + fr.L_off);
    const double* Dg = c.L + fr.D_off;
    const double* yg = c.L + fr.y_off;
    const int lp = cpk(p, m);
    copy_in(S, Lg, lp, lane, 64);
    double v[NRHS], xs[NRHS];
#pragma unroll
    for (int q = 0; q < NRHS; ++q) {
        v[q] = (lane < p) ? yg[(int64_t)q * p + lane] / Dg[lane] : 0.0;
        xs[q] = (lane < mu) ? x[(int64_t)rows[p + lane] * NRHS + q] : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    // column `lane` of the panel is S[cj + i], i >= lane; lanes >= p read column 0
    // (in bounds: p + i < m <= cpk(p, m)) and discard the value
    const int jl = lane < p ? lane : 0;
    const int cj = cpk(jl, m) - jl;
    // four entries per pass, read ahead of the updates (clamped indices, masked
    // values; the broadcast lanes are uniform)
    const double pm = lane < p ? 1.0 : 0.0;
    for (int i0 = 0; i0 < mu; i0 += 4) {
        double l[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) l[u] = (double)S[cj + p + min(i0 + u, mu - 1)] * (i0 + u < mu ? pm : 0.0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < NRHS; ++q) v[q] -= l[u] * readlane_d(xs[q], min(i0 + u, mu - 1));
    }
    for (int j0 = p - 1; j0 > 0; j0 -= 4) {
        double l[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int jj = max(j0 - u, 1);
            l[u] = (double)S[cj + jj] * ((j0 - u >= 1 && lane < jj) ? 1.0 : 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < NRHS; ++q) v[q] -= l[u] * readlane_d(v[q], max(j0 - u, 1));
    }
    if (lane < p)
#pragma unroll
        for (int q = 0; q < NRHS; ++q) x[(int64_t)rows[lane] * NRHS + q] = v[q];
    __builtin_amdgcn_wave_barrier();
}

// Backward substitution of one workgroup front s on threads gt = 0..GT-1 (wave
// gw of the group; the whole workgroup, or one half of it beside a second
// front): the packed L panel staged at Ls (or read from global memory when Ls is
// null), FP64 scratch vb ([NRHS][p] pivot values, [NRHS][m-p] update-row
// solution, [3][p] partial sums), then the update-row products, the pivot
// triangle in 16-pivot blocks (readlane chains in wave 0 of the group) and the
// solution scattered to x.  Fronts sharing a step have equal pivot counts, so
// both halves pass the same barriers.
template <int D, int NRHS, typename T>
__device__ inline void wg_backsolve(const RveCtx& c, int s, T* Ls, double* vb, double* x, int gt, int GT, int gw) {
    const DevPlan& pl = *c.plan;
    const int lane = threadIdx.x & 63;
    constexpr int NPART = (NRHS == 1) ? 3 : 1;
    const DevFront fr = pl.fronts[uni(s)];  // (uniform per wave: scalar loads)
    const int m = uni(fr.m), p = uni(fr.p);
    const int32_t* rows = pl.rows + fr.rows_off;
    const T* Lg = reinterpret_cast<const T*>(c.L + fr.L_off);
    const double* Dg = c.L + fr.D_off;
    const double* yg = c.L + fr.y_off;
    const int lp = cpk(p, m);
    // (FP64 panels are always staged: one address space for the reads)
    const T* Lp = Lg;
    if (sizeof(T) == sizeof(double) || Ls) {
        copy_in(Ls, Lg, lp, gt, GT);
        Lp = Ls;
    }
    double* v = vb;                 // [NRHS][p]
    double* xs = vb + NRHS * p;     // [NRHS][m - p]
    double* part = vb + NRHS * m;   // [NPART][p] (NRHS == 1)
    for (int t = gt; t < p * NRHS; t += GT) {
        const int j = t % p, q = t / p;
        v[t] = yg[(int64_t)q * p + j] / Dg[j];
    }
    for (int t = gt; t < (m - p) * NRHS; t += GT) {
        const int i = t % (m - p), q = t / (m - p);
        xs[t] = x[(int64_t)rows[p + i] * NRHS + q];
    }
    __syncthreads();
    if constexpr (NRHS == 1) {
        for (int t = gt; t < NPART * p; t += GT) {
            const int j = t % p, pt = t / p;
            const T* colj = Lp + cpk(j, m) - j;
            double acc = 0.0;
#pragma unroll 4
            for (int i = p + pt; i < m; i += NPART) acc += (double)colj[i] * xs[i - p];
            part[t] = acc;
        }
        __syncthreads();
        for (int j = gt; j < p; j += GT) v[j] -= (part[j] + part[p + j]) + part[2 * p + j];
    } else {
        for (int j = gt; j < p; j += GT) {
            const T* colj = Lp + cpk(j, m) - j;
            double acc[NRHS];
#pragma unroll
            for (int q = 0; q < NRHS; ++q) acc[q] = 0.0;
#pragma unroll 4
            for (int i = p; i < m; ++i) {
                const double l = colj[i];
#pragma unroll
                for (int q = 0; q < NRHS; ++q) acc[q] += l * xs[q * (m - p) + i - p];
            }
#pragma unroll
            for (int q = 0; q < NRHS; ++q) v[q * p + j] -= acc[q];
        }
    }
    __syncthreads();
    if (p <= 64) {
        // the pivot triangle by the group's wave 0 alone, lane = pivot, from the last pivot
        // (readlane broadcasts of the finished values, no barrier)
        if (gw == 0) {
            const int jl = lane < p ? lane : 0;
            const T* colj = Lp + cpk(jl, m) - jl;  // L(i, lane) = colj[i], i >= lane
            double vv[NRHS];
#pragma unroll
            for (int q = 0; q < NRHS; ++q) vv[q] = lane < p ? v[q * p + lane] : 0.0;
            // four pivots per pass, read ahead of the updates (row max(i, jl) of
            // column jl, inside the panel for every lane; masked values)
            for (int i0 = p - 1; i0 > 0; i0 -= 4) {
                double l[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = max(i0 - u, 1);
                    l[u] = (double)colj[max(i, jl)] * ((i0 - u >= 1 && lane < i) ? 1.0 : 0.0);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int q = 0; q < NRHS; ++q) vv[q] -= l[u] * readlane_d(vv[q], max(i0 - u, 1));
            }
#pragma unroll
            for (int q = 0; q < NRHS; ++q)
                if (lane < p) v[q * p + lane] = vv[q];
        }
        __syncthreads();
    }
    const int nb = p <= 64 ? 0 : (p + 15) >> 4;
    for (int bk = nb - 1; bk >= 0; --bk) {
        const int K = 16 * bk, kb = min(16, p - K);
        if (gw == 0) {
            const bool own = lane < kb;
            double Lr[16];
#pragma unroll
            for (int cc = 0; cc < 16; ++cc)
                Lr[cc] = (own && cc < kb && cc > lane) ? (double)Lp[cpk(K + lane, m) + cc - lane] : 0.0;
#pragma unroll
            for (int q = 0; q < NRHS; ++q) {
                double vv = own ? v[q * p + K + lane] : 0.0;
#pragma unroll
                for (int cc = 15; cc >= 0; --cc) {
                    if (cc < kb) {
                        const double xc = readlane_d(vv, cc);
                        if (lane < cc) vv -= Lr[cc] * xc;
                    }
                }
                if (own) v[q * p + K + lane] = vv;
            }
        }
        __syncthreads();
        for (int j = gt; j < K; j += GT) {
            const T* colj = Lp + cpk(j, m) - j;
            double lk[16];
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) lk[cc] = (cc < kb) ? (double)colj[K + cc] : 0.0;
#pragma unroll
            for (int q = 0; q < NRHS; ++q) {
                double acc = v[q * p + j];
#pragma unroll
                for (int cc = 0; cc < 16; ++cc)
                    if (cc < kb) acc -= lk[cc] * v[q * p + K + cc];
                v[q * p + j] = acc;
            }
        }
        __syncthreads();
    }
    for (int t = gt; t < p * NRHS; t += GT) {
        const int j = t % p, q = t / p;
        x[(int64_t)rows[j] * NRHS + q] = v[t];
    }
    __syncthreads();
}

// backward substitution L^T x = D^-1 y with NRHS columns; y is each front's
// stored forward-substituted rhs, x (node-major [dof][NRHS], FP64) receives the
// solution.  The workgroup fronts in the plan's steps, in reverse (wg_backsolve;
// panels staged in LDS, for FP32 when they fit beside the FP64 scratch), then
// the small subtrees one front per wave, parents first.
template <int D, int NRHS, typename T>
__device__ __noinline__ void backsolve_lds(const RveCtx& c, Smem& sm, T* F, T* rl, double* x, int front_elems,
                                         int wave_slice) {
    const DevPlan& pl = *c.plan;
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    zero_pinned<D>(c, x, NRHS);
    // large fronts (the top of the tree) in the plan's steps, then the small
    // subtrees wave by wave
    for (int st = pl.nwg_steps - 1; st >= 0; --st) {
        const int32_t* e = pl.wg_steps + kStepFronts * st;
        const int nf = e[3] >= 0 ? 4 : (e[1] >= 0 ? 2 : 1);
        const int G = min(nf, NT / 128);
        const int GT = NT / G, NW = NWAVE / G, g = tid / GT;
        // scratch and staged panel: one front uses the front region and (FP64) the
        // rhs region as before; several fronts split the front region, front k
        // taking [panel | FP64 scratch] (FP32: [FP64 scratch | panel]) after
        // those of fronts 0..k-1
        constexpr int dpe = sizeof(double) / sizeof(T);  // T elements per double
        for (int r = 0; r < nf / G; ++r) {
            const int k = r * G + g;
            int off = 0;
            for (int j = 0; j < k; ++j) {
                const int mj = pl.fronts[e[j]].m, pj = pl.fronts[e[j]].p;
                off += (cpk(pj, mj) + dpe * (mj * NRHS + 3 * pj) + 1) & ~1;
            }
            const int m = pl.fronts[e[k]].m, p = pl.fronts[e[k]].p, lp = cpk(p, m);
            const int vneed = dpe * (m * NRHS + 3 * p);
            T* const base = F + off;
            T* Ls;
            double* vb;
            if constexpr (sizeof(T) == sizeof(double)) {
                Ls = base;
                vb = nf > 1 ? reinterpret_cast<double*>(base + lp) : reinterpret_cast<double*>(rl);
            } else {
                // FP32 panel staged after the FP64 scratch when both fit the front region
                vb = reinterpret_cast<double*>(base);
                Ls = (nf > 1 || vneed + lp <= front_elems) ? base + vneed : nullptr;
            }
            wg_backsolve<D, NRHS, T>(c, e[k], Ls, vb, x, tid - g * GT, GT, wave - g * NW);
        }
    }
    // small subtrees: one front per wave, parents (greater height) first
    for (int h = pl.nwave_h - 1; h >= 0; --h) {
        T* S = F + (int64_t)wave * wave_slice;
        for (int k = pl.wave_hbeg[h] + wave; k < pl.wave_hbeg[h + 1]; k += NWAVE)
            backsolve_wave_front<D, NRHS, T>(c, pl.wave_list[k], S, x);
        __syncthreads();
    }
}

// forward substitution L y = b for a new rhs b (node-major [dof][NRHS], FP64,
// overwritten): fronts in elimination order; per front the pivot rows are
// solved in 16-pivot blocks (readlane chain in wave 0) and folded into the rows
// below; the update rows are scattered back into b; the pivot part is stored as
// the front's forward-substituted rhs for backsolve_lds.
template <int D, int NRHS, typename T>
__device__ __noinline__ void forward_lds(const RveCtx& c, Smem& sm, T* F, double* b, int front_elems) {
    const DevPlan& pl = *c.plan;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* vb = reinterpret_cast<double*>(F);  // [NRHS][m] front rows of b
    for (int s = 0; s < pl.nfront; ++s) {
        const DevFront fr = pl.fronts[s];
        const int m = fr.m, p = fr.p;
        const int32_t* rows = pl.rows + fr.rows_off;
        const T* Lp = reinterpret_cast<const T*>(c.L + fr.L_off);
        {
            // stage the panel after the FP64 rows of b when both fit
            const int vneed = (int)((sizeof(double) / sizeof(T)) * m * NRHS);
            const int lp = cpk(p, m);
            if (vneed + lp <= front_elems) {
                T* Ls = F + vneed;
                copy_in(Ls, Lp, lp, tid, NT);
                Lp = Ls;
            }
        }
        double* yg = c.L + fr.y_off;
        for (int t = tid; t < m * NRHS; t += NT) {
            const int i = t % m, q = t / m;
            vb[t] = (i < p) ? b[(int64_t)rows[i] * NRHS + q] : 0.0;
        }
        __syncthreads();
        if (p <= 64) {
            // the pivot triangle by wave 0 alone (lane = pivot row, readlane
            // broadcasts of the finished values), then every row below folds in
            // all p pivots in one pass
            if (wave == 0) {
                double vv[NRHS];
#pragma unroll
                for (int q = 0; q < NRHS; ++q) vv[q] = lane < p ? vb[q * m + lane] : 0.0;
                // four pivots per pass, read ahead of the updates (row
                // max(min(lane, m - 1), j + 1) of column j, inside the panel for
                // every lane; masked values)
                for (int j0 = 0; j0 < p - 1; j0 += 4) {
                    double l[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int j = min(j0 + u, p - 2);
                        const int row = max(min(lane, m - 1), j + 1);
                        l[u] = (double)Lp[cpk(j, m) + row - j] *
                               ((j0 + u < p - 1 && lane > j && lane < p) ? 1.0 : 0.0);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int q = 0; q < NRHS; ++q) vv[q] -= l[u] * readlane_d(vv[q], min(j0 + u, p - 2));
                }
#pragma unroll
                for (int q = 0; q < NRHS; ++q)
                    if (lane < p) vb[q * m + lane] = vv[q];
            }
            __syncthreads();
            for (int i = p + tid; i < m; i += NT) {
                double acc[NRHS];
#pragma unroll
                for (int q = 0; q < NRHS; ++q) acc[q] = vb[q * m + i];
#pragma unroll 4
                for (int j = 0; j < p; ++j) {
                    const double l = (double)Lp[cpk(j, m) + i - j];
#pragma unroll
                    for (int q = 0; q < NRHS; ++q) acc[q] -= l * vb[q * m + j];
                }
#pragma unroll
                for (int q = 0; q < NRHS; ++q) vb[q * m + i] = acc[q];
            }
            __syncthreads();
        }
        for (int K = 0; K < (p <= 64 ? 0 : p); K += 16) {
            const int kb = min(16, p - K);
            if (wave == 0) {
                const bool own = lane < kb;
                double Lr[16];
#pragma unroll
                for (int cc = 0; cc < 16; ++cc)
                    Lr[cc] = (own && cc < kb && cc < lane) ? (double)Lp[cpk(K + cc, m) + lane - cc] : 0.0;
#pragma unroll
                for (int q = 0; q < NRHS; ++q) {
                    double vv = own ? vb[q * m + K + lane] : 0.0;
#pragma unroll
                    for (int cc = 0; cc < 16; ++cc) {
                        if (cc < kb) {
                            const double yc = readlane_d(vv, cc);
                            if (lane > cc) vv -= Lr[cc] * yc;
                        }
                    }
                    if (own) vb[q * m + K + lane] = vv;
                }
            }
            __syncthreads();
            for (int i = K + kb + tid; i < m; i += NT) {
                double lk[16];
#pragma unroll
                for (int cc = 0; cc < 16; ++cc) lk[cc] = (cc < kb) ? (double)Lp[cpk(K + cc, m) + i - K - cc] : 0.0;
#pragma unroll
                for (int q = 0; q < NRHS; ++q) {
                    double acc = vb[q * m + i];
#pragma unroll
                    for (int cc = 0; cc < 16; ++cc)
                        if (cc < kb) acc -= lk[cc] * vb[q * m + K + cc];
                    vb[q * m + i] = acc;
                }
            }
            __syncthreads();
        }
        for (int t = tid; t < p * NRHS; t += NT) {
            const int j = t % p, q = t / p;
            yg[(int64_t)q * p + j] = vb[q * m + j];
        }
        for (int t = tid; t < (m - p) * NRHS; t += NT) {
            const int i = t % (m - p), q = t / (m - p);
            b[(int64_t)rows[p + i] * NRHS + q] += vb[q * m + p + i];  // rows[p+i] holds b; add the update
        }
        __syncthreads();
    }
}

// out = b - K x with the FP64 element tangents (matrix-free), free rows only;
// node-major [dof][NRHS]
template <int D, int NRHS>
__device__ void residual_ke(const RveCtx& c, const double* b, const double* x, double* out) {
    constexpr int NEN = 1 << D, ND = NEN * D;
    const int tot = c.nn * D;
    for (int vi = threadIdx.x; vi < tot; vi += NT) {
        const int v = vi / D, i = vi % D;
        double acc[NRHS];
#pragma unroll
        for (int q = 0; q < NRHS; ++q) acc[q] = 0.0;
        const bool pin = is_pinned(*c.plan, v);
        if (!pin) {
#pragma unroll
            for (int a = 0; a < NEN; ++a) {
                const int e = element_of_node(D, c.n, v, a);
                int nodes[NEN];
                element_nodes(D, c.n, e, nodes);
                const double* kr = c.ke + ((int64_t)e * ND + a * D + i) * ND;
#pragma unroll
                for (int bb = 0; bb < NEN; ++bb)
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const double kv = kr[bb * D + k];
                        const double* xr = x + ((int64_t)nodes[bb] * D + k) * NRHS;
#pragma unroll
                        for (int q = 0; q < NRHS; ++q) acc[q] += kv * xr[q];
                    }
            }
        }
#pragma unroll
        for (int q = 0; q < NRHS; ++q) out[(int64_t)vi * NRHS + q] = pin ? 0.0 : b[(int64_t)vi * NRHS + q] - acc[q];
    }
}

template <int D>
__device__ double free_norm2(const RveCtx& c, Smem& sm, const double* R) {
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < c.nn * D; t += NT)
        if (!is_pinned(*c.plan, t / D)) v[0] += R[t] * R[t];
    block_sum<1>(v, sm);
    return sm.outv[0];
}

// per-RVE context (plan, phases, Lame table, slot regions) and the uniform-grid
// constants in LDS: grad N at the Gauss points, w|J|, Fbar, the tolerance
template <int D>
__device__ inline void rve_setup(const SolveArgs& a, int rve, double* base, RveCtx& c, Smem& sm) {
    constexpr int NEN = 1 << D, ND = NEN * D, D2 = D * D;
    c.plan = &a.plans[a.rve_plan[rve]];
    c.d = D;
    c.n = c.plan->n;
    c.ne = c.plan->nelem;
    c.nn = c.plan->nnode;
    c.nen = NEN;
    c.nd = ND;
    c.phase = a.phase_pool + a.rve_phase[rve];
    c.lame = a.lame_pool + a.rve_lame[rve];
    const int kind = a.rve_kind ? a.rve_kind[rve] : 0;
    c.law = kind & 0xff;
    c.elem = (kind >> 8) & 0xff;
    c.ke32 = 0;
    c.w = base + a.lay.w;
    c.wt = base + a.lay.wt;
    c.R = base + a.lay.R;
    c.rhs = base + a.lay.rhs;
    c.x = base + a.lay.x;
    c.fe = base + a.lay.fe;
    c.ke = base + a.lay.ke;
    c.re = base + a.lay.re;
    c.L = base + a.lay.L;
    c.U = base + a.lay.U;
    c.S = base + a.lay.S;
    // constants of the uniform grid: grad N at the integration points, w|J|.
    // P1: point p is the Kuhn simplex of axis order perm(p), vertices 0,
    // e_s0, e_s0 + e_s1, ..., 1; a cell corner o is its vertex j when o holds j
    // ones, at s0 .. s(j-1); barycentric gradients -e_s0, e_s(j-1) - e_sj,
    // e_s(d-1) (over h), zero at the corners the simplex misses
    if (c.elem == 1 && threadIdx.x < 8 * NEN) {
        const int p = threadIdx.x / NEN, an = threadIdx.x % NEN;
        // the d! axis orders (p < D!: 2 in 2D, 6 in 3D), lexicographic
        const int perm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        const int perm2[2][3] = {{0, 1, 2}, {1, 0, 2}};
        const int npt = D == 2 ? 2 : 6;
        int oa[3] = {0, 0, 0};
        local_offset(D, an, oa);
        double g[3] = {0.0, 0.0, 0.0};
        if (p < npt) {
            const int* pm = D == 2 ? perm2[p] : perm3[p];
            int ones = 0;
            for (int k = 0; k < D; ++k) ones += oa[k];
            bool vert = true;
            for (int q = 0; q < ones; ++q) vert = vert && oa[pm[q]] == 1;
            if (vert) {
                const double ih = (double)c.n;
                if (ones == 0) g[pm[0]] = -ih;
                else if (ones == D) g[pm[D - 1]] = ih;
                else { g[pm[ones - 1]] = ih; g[pm[ones]] = -ih; }
            }
        }
        for (int k = 0; k < 3; ++k) sm.dN[(p * 8 + an) * 3 + k] = g[k];
    } else if (c.elem == 0 && threadIdx.x < NEN * NEN) {
        const int gp = threadIdx.x / NEN, an = threadIdx.x % NEN;
        const double gq = 0.57735026918962576451, h = 1.0 / c.n;
        int og[3] = {0, 0, 0}, oa[3] = {0, 0, 0};
        local_offset(D, gp, og);
        local_offset(D, an, oa);
        for (int k = 0; k < D; ++k) {
            double v = 1.0;
            for (int q = 0; q < D; ++q) {
                const double sa = oa[q] ? 1.0 : -1.0, xi = og[q] ? gq : -gq;
                v *= (q == k) ? 0.5 * sa : 0.5 * (1.0 + sa * xi);
            }
            sm.dN[(gp * 8 + an) * 3 + k] = v * 2.0 / h;
        }
    }
    if (threadIdx.x < D2) sm.Fbar[threadIdx.x] = a.F[(int64_t)rve * D2 + threadIdx.x];
    if (threadIdx.x == 0) {
        double h = 1.0 / c.n, wj = 1.0;
        for (int k = 0; k < D; ++k) wj *= (c.elem == 1 ? h : 0.5 * h);
        if (c.elem == 1) wj /= (D == 2 ? 2.0 : 6.0);  // simplex volume h^d / d!
        sm.wJ = wj;
        sm.flag = 0;
        sm.atol = a.atol >= 0 ? a.atol : a.rve_atol[rve];
    }
    __syncthreads();
}

template <int D, typename T>
__global__ __launch_bounds__(NT, 512 / NT) void rve_solve_kernel(SolveArgs a) {
    __shared__ Smem sm;
    extern __shared__ double dynRaw[];
    T* dynF = reinterpret_cast<T*>(dynRaw);
    constexpr bool IR = sizeof(T) < sizeof(double);  // FP32 factors + FP64 refinement
    constexpr int NEN = 1 << D, ND = NEN * D, D2 = D * D;
    const int64_t slot = blockIdx.x;
    double* base = a.ws + slot * a.lay.stride;
    for (;;) {
        if (threadIdx.x == 0) {
            // queue length: the whole batch, or a device-side count of a subset
            // list (entries outside [0, B) are skipped)
            const unsigned int nq =
                a.count_dev ? (unsigned int)min((int64_t)max(*a.count_dev, 0), a.B) : (unsigned int)a.B;
            int r = -1;
            for (;;) {
                if (a.skip && *a.skip) break;
                const unsigned int idx = atomicAdd(a.counter, 1u);
                if (idx >= nq) break;
                const int cand = a.order[idx];
                if (cand >= 0 && (int64_t)cand < a.B) {
                    r = cand;
                    break;
                }
            }
            sm.rve = r;
        }
        __syncthreads();
        const int rve = sm.rve;
        if (rve < 0) return;
        RveCtx c;
        rve_setup<D>(a, rve, base, c, sm);
        c.ke32 = IR ? 1 : 0;
        double* ir1 = base + a.lay.ir1;
        double* ir2 = base + a.lay.ir2;
        const int ndof = c.nn * D;
        // input checks and initial guess
        bool finite_in = true;
#pragma unroll
        for (int q = 0; q < D2; ++q) finite_in = finite_in && isfinite(sm.Fbar[q]);
        double* wst = a.wstate ? a.wstate + a.state_off[rve] : nullptr;
        for (int t = threadIdx.x; t < ndof; t += NT) c.w[t] = (wst && !is_pinned(*c.plan, t / D)) ? wst[t] : 0.0;
        __syncthreads();
        int status = 0, it = 0;
        bool capped = false, restarted = false;
        if (!finite_in) status = 4;
        double r0 = 0.0, rprev = 0.0;
        // tangent from the last Newton factorization (LDS plans in 2D, global-
        // front plans in either dimension): when the
        // quadratic model r_next ~ r^3 / r_prev^2 puts the next residual within
        // the tolerance, the factorization also forward-substitutes the d^2
        // columns Y of the current state (rhs [dof][1 + d^2], R first); if the
        // next state converges, X ~ K^-1 Y is one backward substitution away
        constexpr int NSPEC = D2 + 1;
        const bool spec_on = NSPEC <= kMaxNrhs && a.reuse_tan && (D == 2 || !c.plan->lds_ok);
        bool spec = false;  // the last factorization carries the Y columns
        PROF_T0();
        while (status == 0) {
            PROF_RESET();
            element_pass<D>(c, sm, c.w, 0, nullptr, nullptr);
            __syncthreads();
            PROF_MARK(PH_ELEM);
            if (sm.flag) {
                if (it == 0 && wst && !restarted) {
                    // a stored fluctuation that folds an element under the new
                    // Fbar is discarded: restart from w = 0 (J = det Fbar > 0)
                    restarted = true;
                    for (int t = threadIdx.x; t < ndof; t += NT) c.w[t] = 0.0;
                    __syncthreads();
                    if (threadIdx.x == 0) sm.flag = 0;
                    __syncthreads();
                    continue;
                }
                status = 2;
                break;
            }
            node_gather<D>(c, c.fe, 1, c.R, 1.0);
            __syncthreads();
            const double rn = sqrt(free_norm2<D>(c, sm, c.R));
            PROF_MARK(PH_GATHER);
            if (!isfinite(rn)) { status = 4; break; }
            if (it == 0) r0 = rn;
            if (rn <= a.rtol * r0 + sm.atol) break;
            if (it == a.max_iter) {
                if (a.flags & 1) capped = true;  // outputs at the last state, reported as NOCONV
                else status = 1;
                break;
            }
            spec = spec_on && it >= 1 && rn * rn * rn <= (a.rtol * r0 + sm.atol) * rprev * rprev;
            rprev = rn;
            if constexpr (NSPEC <= kMaxNrhs) {
                if (spec) {
                    // Y rows of this state: element pass mode 2 with the FP64
                    // tangent rows off (the factor-type tangents stay in place)
                    RveCtx cy = c;
                    cy.ke32 = 0;
                    double dP[D2], dA[D2 * D2];
#pragma unroll
                    for (int q = 0; q < D2; ++q) dP[q] = 0;
#pragma unroll
                    for (int q = 0; q < D2 * D2; ++q) dA[q] = 0;
                    element_pass<D>(cy, sm, c.w, 2, dP, dA);
                    __syncthreads();
                    node_gather<D>(c, c.re, D2, c.rhs, 1.0, NSPEC, 1);
                    for (int t = threadIdx.x; t < ndof; t += NT) c.rhs[(int64_t)t * NSPEC] = -c.R[t];
                    __syncthreads();
                    if (!c.plan->lds_ok) factorize_glb<D, T>(c, sm, NSPEC, dynF);
                    else if constexpr (D == 2) factorize_lds<D, NSPEC, T>(c, sm, dynF, dynF + a.lds_front, a.wave_slice);
                }
            }
            if (!spec) {
                for (int t = threadIdx.x; t < ndof; t += NT) c.rhs[t] = -c.R[t];
                __syncthreads();
                if (c.plan->lds_ok) factorize_lds<D, 1, T>(c, sm, dynF, dynF + a.lds_front, a.wave_slice);
                else factorize_glb<D, T>(c, sm, 1, dynF);
            }
            if (sm.flag) { status = 3; break; }
            PROF_RESET();
            if constexpr (NSPEC <= kMaxNrhs) {
                if (spec) {
                    // every column in one backward sweep, into the rhs buffer
                    // ([dof][1 + d^2]): the Newton step, then X' = K'^-1 Y', which
                    // stays there for the condensation if the next state converges
                    if (!c.plan->lds_ok) backsolve_glb<D, NSPEC, T>(c, sm, c.rhs);
                    else if constexpr (D == 2)
                        backsolve_lds<D, NSPEC, T>(c, sm, dynF, dynF + a.lds_front, c.rhs, a.lds_front, a.wave_slice);
                    for (int t = threadIdx.x; t < ndof; t += NT) c.x[t] = c.rhs[(int64_t)t * NSPEC];
                    __syncthreads();
                }
            }
            if (!spec) {
                if (c.plan->lds_ok) backsolve_lds<D, 1, T>(c, sm, dynF, dynF + a.lds_front, c.x, a.lds_front, a.wave_slice);
                else backsolve_glb<D, 1, T>(c, sm, c.x);
            }
            PROF_MARK(PH_BACK);
            if constexpr (IR) {
                // refinement against the FP64 tangent: dx = K32^-1 (b - K64 x), with
                // K64 x computed matrix-free by the element pass in FP64
                for (int ref = 0; ref < a.ir_max; ++ref) {
                    element_pass<D>(c, sm, c.w, 3, nullptr, nullptr, c.x);
                    __syncthreads();
                    residual_act<D>(c, c.R, -1.0, ir1);  // b = -R
                    __syncthreads();
                    const double rl2 = sqrt(free_norm2<D>(c, sm, ir1));
                    if (!(rl2 > a.ir_eta * rn)) break;
                    if (c.plan->lds_ok) {
                        forward_lds<D, 1, T>(c, sm, dynF, ir1, a.lds_front);
                        backsolve_lds<D, 1, T>(c, sm, dynF, dynF + a.lds_front, ir2, a.lds_front, a.wave_slice);
                    } else {
                        forward_glb<D, 1, T>(c, sm, ir1);
                        backsolve_glb<D, 1, T>(c, sm, ir2);
                    }
                    for (int t = threadIdx.x; t < ndof; t += NT) c.x[t] += ir2[t];
                    __syncthreads();
                }
            }
            // step with det F backtracking
            double alpha = 1.0;
            bool ok = false;
            for (int bt = 0; bt <= a.backtrack; ++bt) {
                for (int t = threadIdx.x; t < ndof; t += NT) c.wt[t] = c.w[t] + alpha * c.x[t];
                if (threadIdx.x == 0) sm.flag = 0;
                __syncthreads();
                element_pass<D>(c, sm, c.wt, 1, nullptr, nullptr);
                __syncthreads();
                const int bad = sm.flag;
                __syncthreads();
                if (!bad) { ok = true; break; }
                alpha *= 0.5;
            }
            if (threadIdx.x == 0) sm.flag = 0;
            PROF_MARK(PH_LINE);
            if (!ok) { status = 2; break; }
            for (int t = threadIdx.x; t < ndof; t += NT) c.w[t] = c.wt[t];
            __syncthreads();
            ++it;
        }
        __syncthreads();
        PROF_RESET();
        double* Pout = a.P + (int64_t)rve * D2;
        double* Aout = a.A ? a.A + (int64_t)rve * D2 * D2 : nullptr;
        if (status == 0) {
            // the condensation from X = K'^-1 Y', solved with the last Newton step
            // (still in the rhs buffer, columns 1..d^2): used where the last
            // factorized residual was within 1e-4 of the initial one, so the
            // stationary form's error (second order in that step) stays far
            // below the tangent's tolerance; in 2D the element pass adds it to
            // the average tangent itself (mode 4)
            const bool stale = Aout && spec && !capped && rprev <= 1e-4 * r0;
            const bool stale2 = stale && D == 2;
            double accP[D2], accA[D2 * D2];
#pragma unroll
            for (int q = 0; q < D2; ++q) accP[q] = 0;
#pragma unroll
            for (int q = 0; q < D2 * D2; ++q) accA[q] = 0;
            element_pass<D>(c, sm, c.w, stale2 ? 4 : 2, accP, accA, stale2 ? c.rhs + 1 : nullptr, NSPEC);
            __syncthreads();
            block_sum<D2>(accP, sm);
            if (threadIdx.x < D2) Pout[threadIdx.x] = sm.outv[threadIdx.x];
            __syncthreads();
            if (Aout && stale2) {
                block_sum<D2 * D2>(accA, sm);
                if (threadIdx.x < D2 * D2) Aout[threadIdx.x] = sm.outv[threadIdx.x];
                __syncthreads();
            } else if (Aout) {
                block_sum<D2 * D2>(accA, sm);
                double Aavg = threadIdx.x < D2 * D2 ? sm.outv[threadIdx.x] : 0.0;
                __syncthreads();
                // otherwise (3D) the stationary form assembled below, refined
                // while ||Y - K X||_F > 1e-4 ||Y||_F (at most twice), or a
                // factorization at w: FP64 (direct Schur form below, no
                // refinement) for global-front plans and for LDS plans whose
                // FP64 front region keeps the occupancy, else in the factor type
                const bool tan64 = !stale && (!IR || !c.plan->lds_ok || a.tan64);
                // Y of w: into the rhs buffer for a factorization at w, else
                // beside X (ir2), X then moved into the element-Y slots
                double* const Y = stale ? ir2 : c.rhs;
                double* const X = c.re;  // [dof][D2] once the element Y rows are gathered
                node_gather<D>(c, c.re, D2, Y, 1.0);
                __syncthreads();
                if constexpr (NSPEC <= kMaxNrhs) {
                    if (stale) {
                        for (int t = threadIdx.x; t < ndof * D2; t += NT)
                            X[t] = c.rhs[(int64_t)(t / D2) * NSPEC + 1 + t % D2];
                        __syncthreads();
                    }
                }
                if (stale)
                    ;
                else if (!c.plan->lds_ok)
                    factorize_glb<D, double>(c, sm, D2, dynRaw);
                else if (IR && a.tan64)
                    factorize_lds<D, D2, double>(c, sm, dynRaw, dynRaw + a.lds_front64, a.wave_slice);
                else
                    factorize_lds<D, D2, T>(c, sm, dynF, dynF + a.lds_front, a.wave_slice);
                if (sm.flag) {
                    status = 3;
                } else if (!tan64) {
                    // X ~ K^-1 Y from the factors (FP32, or of the previous state),
                    // refined against the FP64 tangent of w; then the stationary
                    // (second-order) form
                    //   Abar = <A> - Y^T X - X^T r,  r = Y - K X,
                    // whose error is (X - X*)^T K (X - X*) (energy-norm error squared)
                    if (!stale) backsolve_lds<D, D2, T>(c, sm, dynF, dynF + a.lds_front, X, a.lds_front, a.wave_slice);
                    // refinement corrections: ir2 unless it holds Y
                    double* const corr = stale ? c.rhs : ir2;
                    const int max_ref = stale ? 2 : a.ir_max_tan;
                    for (int ref = 0;; ++ref) {
                        residual_ke<D, D2>(c, Y, X, ir1);
                        __syncthreads();
                        if (ref == max_ref) break;
                        if (stale) {
                            double nr[2] = {0.0, 0.0};
                            for (int t = threadIdx.x; t < ndof * D2; t += NT) {
                                if (is_pinned(*c.plan, t / D2 / D)) continue;
                                nr[0] += ir1[t] * ir1[t];
                                nr[1] += Y[t] * Y[t];
                            }
                            block_sum<2>(nr, sm);
                            const bool done = !(sm.outv[0] > 1e-8 * sm.outv[1]);
                            __syncthreads();
                            if (done) break;
                        }
                        if (c.plan->lds_ok) {
                            forward_lds<D, D2, T>(c, sm, dynF, ir1, a.lds_front);
                            backsolve_lds<D, D2, T>(c, sm, dynF, dynF + a.lds_front, corr, a.lds_front, a.wave_slice);
                        } else {
                            forward_glb<D, D2, T>(c, sm, ir1);
                            backsolve_glb<D, D2, T>(c, sm, corr);
                        }
                        for (int t = threadIdx.x; t < ndof * D2; t += NT) X[t] += corr[t];
                        __syncthreads();
                    }
                    double acc[D2 * D2];
#pragma unroll
                    for (int q = 0; q < D2 * D2; ++q) acc[q] = 0;
                    for (int t = threadIdx.x; t < ndof; t += NT) {
                        if (is_pinned(*c.plan, t / D)) continue;
#pragma unroll
                        for (int g = 0; g < D2; ++g)
#pragma unroll
                            for (int h2 = 0; h2 < D2; ++h2)
                                acc[g * D2 + h2] += Y[t * D2 + g] * X[t * D2 + h2] + X[t * D2 + g] * ir1[t * D2 + h2];
                    }
                    block_sum<D2 * D2>(acc, sm);
                    if (threadIdx.x < D2 * D2) Aout[threadIdx.x] = Aavg - sm.outv[threadIdx.x];
                    __syncthreads();
                } else {
                    // Z^T D^-1 Z over every pivot of every front
                    double acc[D2 * D2];
#pragma unroll
                    for (int q = 0; q < D2 * D2; ++q) acc[q] = 0;
                    const DevPlan& pl = *c.plan;
                    for (int s = 0; s < pl.nfront; ++s) {
                        const DevFront fr = pl.fronts[s];
                        const double* Dg = c.L + fr.D_off;
                        const double* y = c.L + fr.y_off;
                        for (int j = threadIdx.x; j < fr.p; j += NT) {
                            const double rd = 1.0 / Dg[j];
                            double z[D2];
#pragma unroll
                            for (int g = 0; g < D2; ++g) z[g] = y[(int64_t)g * fr.p + j];
#pragma unroll
                            for (int g = 0; g < D2; ++g)
#pragma unroll
                                for (int h2 = 0; h2 < D2; ++h2) acc[g * D2 + h2] += z[g] * z[h2] * rd;
                        }
                    }
                    block_sum<D2 * D2>(acc, sm);
                    if (threadIdx.x < D2 * D2) Aout[threadIdx.x] = Aavg - sm.outv[threadIdx.x];
                    __syncthreads();
                }
            }
            if (status == 0 && wst)
                for (int t = threadIdx.x; t < ndof; t += NT) wst[t] = c.w[t];
        }
        if (status != 0) {
            const double qnan = __builtin_nan("");
            if (threadIdx.x < D2) Pout[threadIdx.x] = qnan;
            if (Aout && threadIdx.x < D2 * D2) Aout[threadIdx.x] = qnan;
        }
        PROF_MARK(PH_FINAL);
        if (threadIdx.x == 0) {
            if (a.status) a.status[rve] = (status == 0 && capped) ? 1 : status;
            if (a.iters) a.iters[rve] = it;
            sm.flag = 0;
        }
        __syncthreads();
    }
}

// The Newton residual and the element tangents of every RVE at its stored (or
// zero) fluctuation, alone: one element pass and the node gather of R per RVE
// (the assembly phase of a Newton iteration, timed on its own by
// rve_assemble_batch).  status[r] = 2 where some J <= 0, else 0.
template <int D>
__global__ __launch_bounds__(NT, 512 / NT) void rve_assembly_kernel(SolveArgs a) {
    __shared__ Smem sm;
    double* base = a.ws + (int64_t)blockIdx.x * a.lay.stride;
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned int idx = atomicAdd(a.counter, 1u);
            sm.rve = idx < (unsigned int)a.B ? a.order[idx] : -1;
        }
        __syncthreads();
        const int rve = sm.rve;
        if (rve < 0) return;
        RveCtx c;
        rve_setup<D>(a, rve, base, c, sm);
        const int ndof = c.nn * D;
        const double* wst = a.wstate ? a.wstate + a.state_off[rve] : nullptr;
        for (int t = threadIdx.x; t < ndof; t += NT) c.w[t] = (wst && !is_pinned(*c.plan, t / D)) ? wst[t] : 0.0;
        __syncthreads();
        element_pass<D>(c, sm, c.w, 0, nullptr, nullptr);
        __syncthreads();
        node_gather<D>(c, c.fe, 1, c.R, 1.0);
        if (threadIdx.x == 0 && a.status) a.status[rve] = sm.flag ? 2 : 0;
        __syncthreads();
    }
}

__global__ void reset_counter_kernel(unsigned int* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

int lds_static_bytes() { return (int)sizeof(Smem); }

// dynamic LDS limits are raised once per process, outside any stream capture
hipError_t prepare_rve_solve() {
    const void* ks[4] = {(const void*)rve_solve_kernel<2, double>, (const void*)rve_solve_kernel<2, float>,
                         (const void*)rve_solve_kernel<3, double>, (const void*)rve_solve_kernel<3, float>};
    for (const void* k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           kLdsBytesMax - (int)sizeof(Smem));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_rve_assembly(const SolveArgs& a, int nslots, hipStream_t stream) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, stream, a.counter);
    if (a.dim == 2)
        hipLaunchKernelGGL((rve_assembly_kernel<2>), dim3(nslots), dim3(NT), 0, stream, a);
    else
        hipLaunchKernelGGL((rve_assembly_kernel<3>), dim3(nslots), dim3(NT), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_rve_solve(const SolveArgs& a, int nslots, size_t dyn_bytes, bool fp32, hipStream_t stream) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, stream, a.counter);
    if (a.dim == 2 && fp32)
        hipLaunchKernelGGL((rve_solve_kernel<2, float>), dim3(nslots), dim3(NT), dyn_bytes, stream, a);
    else if (a.dim == 2)
        hipLaunchKernelGGL((rve_solve_kernel<2, double>), dim3(nslots), dim3(NT), dyn_bytes, stream, a);
    else if (fp32)
        hipLaunchKernelGGL((rve_solve_kernel<3, float>), dim3(nslots), dim3(NT), dyn_bytes, stream, a);
    else
        hipLaunchKernelGGL((rve_solve_kernel<3, double>), dim3(nslots), dim3(NT), dyn_bytes, stream, a);
    return hipGetLastError();
}

}  // namespace FEHMM_VARIANT
}  // namespace fehmm

#if FEHMM_PHASE_PROF
#define FEHMM_CAT2(a, b) a##_##b
#define FEHMM_CAT(a, b) FEHMM_CAT2(a, b)
extern "C" int FEHMM_CAT(rve_debug_phase_clocks, FEHMM_VARIANT)(unsigned long long* out, int reset) {
    namespace V = fehmm::FEHMM_VARIANT;
    if (hipMemcpyFromSymbol(out, HIP_SYMBOL(V::g_phase), sizeof(unsigned long long) * V::PH_N) != hipSuccess)
        return -3;
    if (reset) {
        unsigned long long z[V::PH_N] = {0};
        if (hipMemcpyToSymbol(HIP_SYMBOL(V::g_phase), z, sizeof(z)) != hipSuccess) return -3;
    }
    return 0;
}
#if FEHMM_NT == 256
// the phase clocks of both workgroup sizes, summed
extern "C" int rve_debug_phase_clocks_nt512(unsigned long long* out, int reset);
extern "C" int rve_debug_phase_clocks(unsigned long long* out, int reset) {
    unsigned long long b[fehmm::nt256::PH_N];
    if (rve_debug_phase_clocks_nt256(out, reset) || rve_debug_phase_clocks_nt512(b, reset)) return -3;
    for (int i = 0; i < fehmm::nt256::PH_N; ++i) out[i] += b[i];
    return 0;
}
#endif
#endif
