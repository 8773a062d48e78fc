// rve_solve.hip -- persistent batched periodic-RVE solver for gfx950.
//
// One workgroup (256 threads, four wave64) owns one workspace slot and pulls
// RVE ids from a device queue until the batch is exhausted.  Per RVE it runs the
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
// G_IK, S_IK) written with P and A = dP/dF.
//
// The linear solve is a multifrontal LDL^T (no pivoting: the tangent can be
// indefinite at the initial guess past a micro-instability of a stiff inclusion)
// driven by the (d, n) plan: element matrices are gathered straight into the
// dense fronts, children's update matrices are extended-added from a stack, the
// forward substitution is fused into the factorization, and the backward
// substitution walks the fronts in reverse.
#include <hip/hip_runtime.h>

#include "mesh_common.h"
#include "solver_dev.h"

namespace fehmm {

constexpr int NT = 256;
constexpr int NWAVE = NT / 64;

struct Smem {
    double red[NWAVE * 96];
    double dN[8 * 8 * 3];    // [gp][a][k]
    double dd[8 * 8 * 8];    // [gp][a][b] grad N_a . grad N_b
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

// Element pass.  mode 0: residual + tangent rows (Newton); mode 1: J > 0 check
// only (on w); mode 2: final outputs (Pbar, <A>, Y rows).  Work item = (e, a)
// in 2D (rows i = 0,1), (e, a, i) in 3D.
template <int D>
__device__ void element_pass(const RveCtx& c, Smem& sm, const double* w, int mode, double* accP, double* accA) {
    constexpr int NEN = 1 << D, ND = NEN * D, RPI = (D == 2) ? 2 : 1;
    const int nitems = c.ne * NEN * (D / RPI);
    const double wJ = sm.wJ;
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
        for (int gp = 0; gp < NEN; ++gp) {
            double F[D * D], Fi[D * D], J;
            gp_F<D>(c, sm, wl, gp, F);
            inv_det<D>(F, Fi, J);
            if (!(J > 0.0)) { sm.flag = 1; continue; }
            if (mode == 1) continue;
            const double c1 = mu - 0.5 * lam * (J * J - 1.0), c2 = lam * J * J;
            if (mode == 2 && a == 0 && i0 == 0) {
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
#pragma unroll
                    for (int b = 0; b < NEN; ++b) {
                        const double dab = sm.dd[(gp * 8 + a) * 8 + b];
#pragma unroll
                        for (int k = 0; k < D; ++k)
                            kr[r][b * D + k] += ((i == k ? mu * dab : 0.0) + c1 * ga[k] * g[b][i] + c2 * ga[i] * g[b][k]) * wJ;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < D; ++k)
#pragma unroll
                        for (int L = 0; L < D; ++L)
                            yr[r][k * D + L] += ((i == k ? mu * dNa[L] : 0.0) + c1 * ga[k] * Fi[L * D + i] +
                                                 c2 * ga[i] * Fi[L * D + k]) * wJ;
                }
            }
        }
        if (mode == 0) {
#pragma unroll
            for (int r = 0; r < RPI; ++r) {
                const int row = a * D + i0 + r;
                c.fe[(int64_t)e * ND + row] = fr[r];
                double* kd = c.ke + ((int64_t)e * ND + row) * ND;
#pragma unroll
                for (int q = 0; q < ND; ++q) kd[q] = kr[r][q];
            }
        } else if (mode == 2) {
#pragma unroll
            for (int r = 0; r < RPI; ++r) {
                const int row = a * D + i0 + r;
                double* yd = c.re + ((int64_t)e * ND + row) * (D * D);
#pragma unroll
                for (int q = 0; q < D * D; ++q) yd[q] = yr[r][q];
            }
        }
    }
}

// node gather of element vectors: out[(v*D+i)*nc + col] = sum_a src[e_a(v)][(a*D+i)*nc + col]
template <int D>
__device__ void node_gather(const RveCtx& c, const double* src, int nc, double* out, double sign) {
    constexpr int NEN = 1 << D, ND = NEN * D;
    const int tot = c.nn * D * nc;
    for (int t = threadIdx.x; t < tot; t += NT) {
        int col = t % nc, vi = t / nc, v = vi / D, i = vi % D;
        double s = 0;
#pragma unroll
        for (int a = 0; a < NEN; ++a) {
            int e = element_of_node(D, c.n, v, a);
            s += src[((int64_t)e * ND + a * D + i) * nc + col];
        }
        out[t] = sign * s;
    }
}

// Multifrontal LDL^T of K_ff with nrhs right-hand sides in c.rhs (node-major
// [dof][nrhs]); forward substitution fused.  Returns via sm.flag = 2 on a
// vanishing pivot.
template <int D>
__device__ void factorize(const RveCtx& c, Smem& sm, int nrhs) {
    constexpr int NEN = 1 << D, ND = NEN * D;
    const DevPlan& pl = *c.plan;
    for (int s = 0; s < pl.nfront; ++s) {
        const DevFront fr = pl.fronts[s];
        const int m = fr.m, p = fr.p, mu = m - p;
        const int32_t* rows = pl.rows + fr.rows_off;
        double* Fp = c.L + fr.L_off;
        double* Dg = c.L + fr.D_off;
        double* y = c.L + fr.y_off;
        double* Us = c.S;
        double* rus = c.S + (int64_t)mu * mu;
        // 1. zero the panel and the scratch update matrix, load the pivot rhs
        for (int t = threadIdx.x; t < m * p; t += NT) Fp[t] = 0.0;
        for (int t = threadIdx.x; t < mu * mu + mu * nrhs; t += NT) Us[t] = 0.0;
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
            double v = 0;
            for (int q = 0; q < kp.c_count; ++q) {
                const KContrib cb = pl.kcontrib[kp.c_begin + q];
                v += c.ke[((int64_t)cb.elem * ND + cb.lb * D + k) * ND + cb.la * D + l];
            }
            Fp[(int64_t)col * m + r] = v;
            if (r == col) Dg[col] = v;
        }
        __syncthreads();
        // 3. extend-add of the children's update matrices and rhs updates
        for (int q = fr.child_begin; q < fr.child_end; ++q) {
            const DevFront ch = pl.fronts[pl.children[q]];
            const int mc = ch.m - ch.p;
            const int32_t* rel = pl.relind + ch.relind_off;
            const double* Uc = c.U + ch.U_off;
            const double* ruc = Uc + (int64_t)mc * mc;
            for (int t = threadIdx.x; t < mc * mc; t += NT) {
                const int i = t % mc, k = t / mc;
                if (i < k) continue;
                const int R = rel[i], C = rel[k];
                const double v = Uc[t];
                if (C < p) Fp[(int64_t)C * m + R] += v;
                else Us[(int64_t)(C - p) * mu + (R - p)] += v;
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
        // 4. LDL^T of the m x p panel (right-looking, unblocked), forward rhs
        for (int j = 0; j < p; ++j) {
            const double piv = Fp[(int64_t)j * m + j];
            if (!(fabs(piv) > 1e-14 * fabs(Dg[j])) || !isfinite(piv)) {
                if (threadIdx.x == 0) sm.flag = 2;
            }
            const double rp = 1.0 / piv;
            const double* colj = Fp + (int64_t)j * m;
            // trailing panel columns k in (j, p), rows i >= k
            const int w = m - j - 1;
            const int ncol = p - j - 1;
            for (int t = threadIdx.x; t < w * ncol; t += NT) {
                const int i = j + 1 + t % w, k = j + 1 + t / w;
                if (i < k) continue;
                Fp[(int64_t)k * m + i] -= colj[i] * colj[k] * rp;
            }
            for (int t = threadIdx.x; t < w * nrhs; t += NT) {
                const int i = j + 1 + t % w, col = t / w;
                const double l = colj[i] * rp;
                const double yj = y[(int64_t)col * p + j];
                if (i < p) y[(int64_t)col * p + i] -= l * yj;
                else rus[(int64_t)col * mu + (i - p)] -= l * yj;
            }
            __syncthreads();
            for (int t = threadIdx.x; t < w; t += NT) Fp[(int64_t)j * m + j + 1 + t] *= rp;
            if (threadIdx.x == 0) Dg[j] = piv;
            // no barrier needed: the next step reads column j+1 (finished above)
        }
        __syncthreads();
        // 5. Schur complement U_s -= L21 D L21^T
        for (int t = threadIdx.x; t < mu * mu; t += NT) {
            const int i = t % mu, k = t / mu;
            if (i < k) continue;
            double s = 0;
            for (int j = 0; j < p; ++j) {
                const double* cj = Fp + (int64_t)j * m + p;
                s += cj[i] * Dg[j] * cj[k];
            }
            Us[t] -= s;
        }
        __syncthreads();
        // 6. push U_s (and its rhs part) on the stack
        if (mu > 0) {
            double* dst = c.U + fr.U_off;
            for (int t = threadIdx.x; t < mu * mu + mu * nrhs; t += NT) dst[t] = Us[t];
        }
        __syncthreads();
    }
}

// backward substitution L^T x = D^-1 y (nrhs = 1); x in node-major dof order
template <int D>
__device__ void backsolve(const RveCtx& c, Smem& sm) {
    const DevPlan& pl = *c.plan;
    for (int t = threadIdx.x; t < D; t += NT) c.x[t] = 0.0;  // pinned node
    for (int s = pl.nfront - 1; s >= 0; --s) {
        const DevFront fr = pl.fronts[s];
        const int m = fr.m, p = fr.p;
        const int32_t* rows = pl.rows + fr.rows_off;
        const double* Fp = c.L + fr.L_off;
        const double* Dg = c.L + fr.D_off;
        double* y = c.L + fr.y_off;
        for (int j = threadIdx.x; j < p; j += NT) {
            double v = y[j] / Dg[j];
            const double* cj = Fp + (int64_t)j * m;
            for (int i = p; i < m; ++i) v -= cj[i] * c.x[rows[i]];
            y[j] = v;
        }
        __syncthreads();
        for (int jj = p - 1; jj > 0; --jj) {
            const double xj = y[jj];
            for (int j = threadIdx.x; j < jj; j += NT) y[j] -= Fp[(int64_t)j * m + jj] * xj;
            __syncthreads();
        }
        for (int j = threadIdx.x; j < p; j += NT) c.x[rows[j]] = y[j];
        __syncthreads();
    }
}

template <int D>
__device__ double free_norm2(const RveCtx& c, Smem& sm, const double* R) {
    double v[1] = {0.0};
    for (int t = D + threadIdx.x; t < c.nn * D; t += NT) v[0] += R[t] * R[t];
    block_sum<1>(v, sm);
    return sm.outv[0];
}

template <int D>
__global__ __launch_bounds__(NT) void rve_solve_kernel(SolveArgs a) {
    __shared__ Smem sm;
    constexpr int NEN = 1 << D, ND = NEN * D, D2 = D * D;
    const int64_t slot = blockIdx.x;
    double* base = a.ws + slot * a.lay.stride;
    for (;;) {
        if (threadIdx.x == 0) {
            unsigned int idx = atomicAdd(a.counter, 1u);
            sm.rve = (idx < (unsigned int)a.B) ? a.order[idx] : -1;
        }
        __syncthreads();
        const int rve = sm.rve;
        if (rve < 0) return;
        RveCtx c;
        c.plan = &a.plans[a.rve_plan[rve]];
        c.d = D;
        c.n = c.plan->n;
        c.ne = c.plan->nelem;
        c.nn = c.plan->nnode;
        c.nen = NEN;
        c.nd = ND;
        c.phase = a.phase_pool + a.rve_phase[rve];
        c.lame = a.lame_pool + a.rve_lame[rve];
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
        const int ndof = c.nn * D;
        // constants of the uniform grid: grad N at the Gauss points, w|J|
        if (threadIdx.x < NEN * NEN) {
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
            for (int k = 0; k < D; ++k) wj *= 0.5 * h;
            sm.wJ = wj;
            sm.flag = 0;
            sm.atol = a.atol >= 0 ? a.atol : a.rve_atol[rve];
        }
        __syncthreads();
        for (int t = threadIdx.x; t < NEN * NEN * NEN; t += NT) {
            const int gp = t / (NEN * NEN), an = (t / NEN) % NEN, bn = t % NEN;
            double s = 0;
            for (int k = 0; k < D; ++k) s += sm.dN[(gp * 8 + an) * 3 + k] * sm.dN[(gp * 8 + bn) * 3 + k];
            sm.dd[(gp * 8 + an) * 8 + bn] = s;
        }
        // input checks and initial guess
        bool finite_in = true;
        for (int q = 0; q < D2; ++q) finite_in = finite_in && isfinite(sm.Fbar[q]);
        double* wst = a.wstate ? a.wstate + a.state_off[rve] : nullptr;
        for (int t = threadIdx.x; t < ndof; t += NT) c.w[t] = (wst && t >= D) ? wst[t] : 0.0;
        __syncthreads();
        int status = 0, it = 0;
        if (!finite_in) status = 4;
        double r0 = 0.0;
        while (status == 0) {
            element_pass<D>(c, sm, c.w, 0, nullptr, nullptr);
            __syncthreads();
            if (sm.flag) { status = 2; break; }
            node_gather<D>(c, c.fe, 1, c.R, 1.0);
            __syncthreads();
            const double rn = sqrt(free_norm2<D>(c, sm, c.R));
            if (!isfinite(rn)) { status = 4; break; }
            if (it == 0) r0 = rn;
            if (rn <= a.rtol * r0 + sm.atol) break;
            if (it == a.max_iter) { status = 1; break; }
            for (int t = threadIdx.x; t < ndof; t += NT) c.rhs[t] = -c.R[t];
            __syncthreads();
            factorize<D>(c, sm, 1);
            if (sm.flag) { status = 3; break; }
            backsolve<D>(c, sm);
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
            if (!ok) { status = 2; break; }
            for (int t = threadIdx.x; t < ndof; t += NT) c.w[t] = c.wt[t];
            __syncthreads();
            ++it;
        }
        __syncthreads();
        double* Pout = a.P + (int64_t)rve * D2;
        double* Aout = a.A ? a.A + (int64_t)rve * D2 * D2 : nullptr;
        if (status == 0) {
            double accP[D2], accA[D2 * D2];
            for (int q = 0; q < D2; ++q) accP[q] = 0;
            for (int q = 0; q < D2 * D2; ++q) accA[q] = 0;
            element_pass<D>(c, sm, c.w, 2, accP, accA);
            __syncthreads();
            block_sum<D2>(accP, sm);
            if (threadIdx.x < D2) Pout[threadIdx.x] = sm.outv[threadIdx.x];
            __syncthreads();
            if (Aout) {
                block_sum<D2 * D2>(accA, sm);
                double Aavg = threadIdx.x < D2 * D2 ? sm.outv[threadIdx.x] : 0.0;
                __syncthreads();
                node_gather<D>(c, c.re, D2, c.rhs, 1.0);
                __syncthreads();
                factorize<D>(c, sm, D2);
                if (sm.flag) {
                    status = 3;
                } else {
                    // Z^T D^-1 Z over every pivot of every front
                    double acc[D2 * D2];
                    for (int q = 0; q < D2 * D2; ++q) acc[q] = 0;
                    const DevPlan& pl = *c.plan;
                    for (int s = 0; s < pl.nfront; ++s) {
                        const DevFront fr = pl.fronts[s];
                        const double* Dg = c.L + fr.D_off;
                        const double* y = c.L + fr.y_off;
                        for (int j = threadIdx.x; j < fr.p; j += NT) {
                            const double rd = 1.0 / Dg[j];
                            double z[D2];
                            for (int g = 0; g < D2; ++g) z[g] = y[(int64_t)g * fr.p + j];
                            for (int g = 0; g < D2; ++g)
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
        if (threadIdx.x == 0) {
            if (a.status) a.status[rve] = status;
            if (a.iters) a.iters[rve] = it;
            sm.flag = 0;
        }
        __syncthreads();
    }
}

__global__ void reset_counter_kernel(unsigned int* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

hipError_t launch_rve_solve(const SolveArgs& a, int nslots, hipStream_t stream) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, stream, a.counter);
    if (a.dim == 2)
        hipLaunchKernelGGL(rve_solve_kernel<2>, dim3(nslots), dim3(NT), 0, stream, a);
    else
        hipLaunchKernelGGL(rve_solve_kernel<3>, dim3(nslots), dim3(NT), 0, stream, a);
    return hipGetLastError();
}

}  // namespace fehmm
