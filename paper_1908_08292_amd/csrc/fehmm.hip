// fehmm.hip -- two-scale FE-HMM driver (include/fehmm.h): macro Q1 mesh, device
// gather of the quadrature-point deformation gradients, the batched RVE solves,
// deterministic colour-ordered assembly of the banded macro system, and a
// single-workgroup banded LDL^T solve; the macro Newton loop runs on the host
// with one device-to-host norm per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/fehmm.h"
#include "../../include/surrogate.h"

int rve_internal_set_error(int code, const std::string& msg);  // rve_abi.cpp
static inline int set_error(int code, const std::string& msg) { return rve_internal_set_error(code, msg); }

namespace {

constexpr int NTB = 1024;  // threads of the banded solver

struct MacroGeom {
    double dN[4][4][2];  // [point][node][dir]
    double wdet;         // weight of each point
    int npt;             // points per grid cell: 4 (Q1, 2x2 Gauss) or 2 (P1 triangles)
};

// F at every Gauss point: F = I + sum_a u_a (x) grad N_a
__global__ void macro_gather_F(const int* __restrict__ conn, int nelem, const double* __restrict__ u, MacroGeom g,
                               double* __restrict__ F, const int* __restrict__ done) {
    if (*done) return;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= g.npt * nelem) return;
    const int e = q / g.npt, gp = q % g.npt;
    double f[4] = {1.0, 0.0, 0.0, 1.0};
    for (int a = 0; a < 4; ++a) {
        const int v = conn[4 * e + a];
        for (int i = 0; i < 2; ++i)
            for (int J = 0; J < 2; ++J) f[i * 2 + J] += u[2 * v + i] * g.dN[gp][a][J];
    }
    for (int k = 0; k < 4; ++k) F[4 * q + k] = f[k];
}

// element residual (8) and tangent (8 x 8) from the transferred Pbar, Abar
__global__ void macro_element(int nelem, const double* __restrict__ P, const double* __restrict__ A, MacroGeom g,
                              double* __restrict__ ke, double* __restrict__ fe, const int* __restrict__ done) {
    if (*done) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nelem * 8) return;
    const int e = t >> 3, r = t & 7, a = r >> 1, i = r & 1;
    double fr = 0.0, kr[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int gp = 0; gp < g.npt; ++gp) {
        const double* Pq = P + 4 * (g.npt * e + gp);
        const double* Aq = A + 16 * (g.npt * e + gp);
        for (int J = 0; J < 2; ++J) fr += Pq[i * 2 + J] * g.dN[gp][a][J] * g.wdet;
        for (int b = 0; b < 4; ++b)
            for (int k = 0; k < 2; ++k) {
                double s = 0.0;
                for (int J = 0; J < 2; ++J)
                    for (int L = 0; L < 2; ++L) s += g.dN[gp][a][J] * Aq[(i * 2 + J) * 4 + k * 2 + L] * g.dN[gp][b][L];
                kr[b * 2 + k] += s * g.wdet;
            }
    }
    fe[8 * e + r] = fr;
    for (int c = 0; c < 8; ++c) ke[64 * e + 8 * r + c] = kr[c];
}

__global__ void macro_zero_int(int* __restrict__ x, int n) {
    if ((int)threadIdx.x < n) x[threadIdx.x] = 0;
}

// fallback set of a load step: a point joins when its indicator exceeds the
// threshold (or is NaN) and stays; flag reports a new member; ind is
// rewritten as +inf for members and 0 otherwise, for the compaction
__global__ void macro_merge_fallback(float* __restrict__ ind, int* __restrict__ mask, float thr, int n,
                                     int* __restrict__ grew, const int* __restrict__ done) {
    if (*done) return;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float v = ind[q];
    int m = mask[q];
    if (!m && !(v <= thr)) {
        m = 1;
        mask[q] = 1;
        *grew = 1;
    }
    ind[q] = m ? INFINITY : 0.0f;
}

__global__ void macro_zero_ints(int* __restrict__ x, int64_t n, const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = 0;
}

__global__ void macro_zero(double* __restrict__ x, int64_t n, const int* __restrict__ done) {
    if (*done) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = 0.0;
}

// add the elements of one colour (no two share a node) into the lower band
// K[i * (bw + 1) + (i - j)], i >= j, and into R
__global__ void macro_scatter(const int* __restrict__ elist, int nel, const int* __restrict__ conn,
                              const double* __restrict__ ke, const double* __restrict__ fe, int bw,
                              double* __restrict__ K, double* __restrict__ R, const int* __restrict__ done) {
    if (*done) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nel * 8) return;
    const int e = elist[t >> 3], r = t & 7;
    const int gi = 2 * conn[4 * e + (r >> 1)] + (r & 1);
    R[gi] += fe[8 * e + r];
    for (int c = 0; c < 8; ++c) {
        const int gj = 2 * conn[4 * e + (c >> 1)] + (c & 1);
        if (gj <= gi) K[(int64_t)gi * (bw + 1) + (gi - gj)] += ke[64 * e + 8 * r + c];
    }
}

// first macro iteration of a load step: the prescribed increment moves the free
// dofs through the coupling block, R_f += K_fd dud (K symmetric, lower band:
// K(i, j) for j <= i sits in row i, for j > i as K(j, i) in row j)
__global__ void macro_dirichlet_rhs(const double* __restrict__ K, const double* __restrict__ dud,
                                    const int* __restrict__ fixed, int ndof, int bw, double* __restrict__ R,
                                    const int* __restrict__ done) {
    if (*done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ndof || fixed[i]) return;
    double acc = 0.0;
    for (int k = 1; k <= bw; ++k) {
        const int jl = i - k, ju = i + k;
        if (jl >= 0) acc += K[(int64_t)i * (bw + 1) + k] * dud[jl];
        if (ju < ndof) acc += K[(int64_t)ju * (bw + 1) + k] * dud[ju];
    }
    R[i] += acc;
}

// Dirichlet dofs: identity row/column, zero residual (their increment is
// applied by macro_update)
__global__ void macro_bc(const int* __restrict__ fixed, int ndof, int bw, double* __restrict__ K,
                         double* __restrict__ R, const int* __restrict__ done) {
    if (*done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ndof) return;
    for (int k = 1; k <= bw; ++k) {
        const int j = i - k;
        if (j >= 0 && (fixed[i] || fixed[j])) K[(int64_t)i * (bw + 1) + k] = 0.0;
    }
    if (fixed[i]) {
        K[(int64_t)i * (bw + 1)] = 1.0;
        R[i] = 0.0;
    }
}

// Device-side state of one load step.  The macro Newton's decisions are taken
// on the device (macro_norm_step), and every later kernel of the step returns
// at once when `done` is set, so a whole load step -- with its data-dependent
// number of macro iterations -- can be replayed as one captured graph.
struct StepState {
    int step;       // load step (written by the host before the step)
    int done;       // converged, failed or out of iterations
    int it;         // macro Newton updates taken when done
    int status;     // FEHMM_STEP_*
    int failed;     // failed RVEs at the stopping iteration
    int grew;       // surrogate: the fallback set grew in this iteration
    int band_flag;  // zero or non-finite pivot in a macro solve
    int pad;
    double r0;
    long long micro, fallback, surrogate;
    double hist[FEHMM_MAX_HIST];
};

// start of a load step: the increment of the prescribed displacements
// (right-edge x dofs: the step's fraction of the stretch, other fixed dofs 0),
// dud = target - u on fixed dofs and 0 elsewhere; it enters the first macro
// Newton iteration through the linear solve (macro_dirichlet_rhs), and u takes
// it with that iteration's update.  Also resets the step state.
__global__ void macro_step_init(StepState* __restrict__ st, const double* __restrict__ u,
                                double* __restrict__ dud, const int* __restrict__ fixed,
                                const int* __restrict__ rightx, double ux_per_step, int ndof) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int step = st->step;
    if (i < ndof) dud[i] = fixed[i] ? (rightx[i] ? ux_per_step * step : 0.0) - u[i] : 0.0;
    if (i == 0) {
        st->done = 0;
        st->it = 0;
        st->status = FEHMM_STEP_CONVERGED;
        st->failed = 0;
        st->grew = 0;
        st->band_flag = 0;
        st->r0 = -1.0;
        st->micro = st->fallback = st->surrogate = 0;
    }
}

// one workgroup: ||R||, failed RVEs and micro iterations of this macro
// iteration; records the residual history and decides convergence
__global__ void macro_norm_step(const double* __restrict__ R, int ndof, const int* __restrict__ status,
                                const int* __restrict__ iters, int nqp, int tolerate_noconv,
                                const int* __restrict__ fallback_count, StepState* __restrict__ st, int it,
                                double rtol, int max_iter) {
    if (st->done) return;
    __shared__ double s[256];
    __shared__ int bad[256];
    __shared__ long long mi[256];
    double acc = 0.0;
    int nb = 0;
    long long m = 0;
    for (int i = threadIdx.x; i < ndof; i += 256) acc += R[i] * R[i];
    for (int q = threadIdx.x; q < nqp; q += 256) {
        const int sq = status[q];
        nb += (sq != 0 && !(tolerate_noconv && sq == 1)) ? 1 : 0;
        m += iters[q];
    }
    s[threadIdx.x] = acc;
    bad[threadIdx.x] = nb;
    mi[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s[threadIdx.x] += s[threadIdx.x + o];
            bad[threadIdx.x] += bad[threadIdx.x + o];
            mi[threadIdx.x] += mi[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    st->micro += mi[0];
    if (fallback_count) {
        const int nf = *fallback_count;
        st->fallback += nf;
        st->surrogate += nqp - nf;
    }
    const int grew = st->grew;
    st->grew = 0;
    if (bad[0] > 0) {
        st->status = FEHMM_STEP_RVE_FAILED;
        st->failed = bad[0];
        st->it = it;
        st->done = 1;
        return;
    }
    const double rn = sqrt(s[0]);
    if (st->r0 < 0) st->r0 = rn;
    const double r0 = st->r0;
    st->hist[it] = r0 > 0 ? rn / r0 : 0.0;
    if ((rn <= rtol * r0 || rn == 0.0) && !grew) {
        st->it = it;
        st->done = 1;
    } else if (it == max_iter) {
        st->status = FEHMM_STEP_NOCONV;
        st->it = it;
        st->done = 1;
    }
}

// banded LDL^T (lower band, bandwidth bw) and solve K du = -R in one workgroup
__global__ __launch_bounds__(NTB) void macro_band_solve(double* __restrict__ K, const double* __restrict__ R, int n,
                                                        int bw, double* __restrict__ du, int* __restrict__ flag,
                                                        const int* __restrict__ done) {
    if (*done) return;
    const int ld = bw + 1;
    for (int k = 0; k < n; ++k) {
        const double piv = K[(int64_t)k * ld];
        if (threadIdx.x == 0 && (!(fabs(piv) > 0.0) || !isfinite(piv))) *flag = 1;
        const int w = min(bw, n - 1 - k);
        // trailing band update with the unscaled column: K_ij -= K_ik K_jk / piv
        for (int t = threadIdx.x; t < w * w; t += NTB) {
            const int ii = t / w, jj = t % w;
            if (jj > ii) continue;
            const int i = k + 1 + ii, j = k + 1 + jj;
            K[(int64_t)i * ld + (i - j)] -= K[(int64_t)i * ld + (i - k)] * K[(int64_t)j * ld + (j - k)] / piv;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < w; t += NTB) {
            const int i = k + 1 + t;
            K[(int64_t)i * ld + (i - k)] /= piv;
        }
        __syncthreads();
    }
    // forward (unit L), diagonal, backward; one workgroup, dot products by wave 0
    for (int i = threadIdx.x; i < n; i += NTB) du[i] = -R[i];
    __syncthreads();
    __shared__ double red[64];
    for (int i = 0; i < n; ++i) {
        if (threadIdx.x < 64) {
            double s = 0.0;
            for (int j = max(0, i - bw) + threadIdx.x; j < i; j += 64) s += K[(int64_t)i * ld + (i - j)] * du[j];
            for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
            if (threadIdx.x == 0) du[i] -= s;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += NTB) du[i] /= K[(int64_t)i * ld];
    __syncthreads();
    for (int i = n - 1; i >= 0; --i) {
        const double xi = du[i];
        for (int t = threadIdx.x; t < bw; t += NTB) {
            const int j = i - 1 - t;
            if (j >= 0) du[j] -= K[(int64_t)i * ld + (i - j)] * xi;
        }
        __syncthreads();
    }
}

// Blocked banded LDL^T and solve K du = -R in one workgroup of 4 waves, for
// bandwidths past the windowed solver's (macro_band_factor_window below) up to
// kBandMaxBw; the unblocked macro_band_solve above takes wider bands.  The
// factor stays in global memory.  Per block of kPanel columns: wave 0 factors the
// panel (kPanel columns x up to kPanel + bw rows) in registers, one column
// after the other with the pivot row's values broadcast by readlane (no
// barrier inside a panel); then all waves apply the panel's rank-kPanel update
// to the trailing bw x bw triangle as 16 x 16 FP64 MFMA tiles.  The factor is
// also written transposed (Kt: row j holds column j of L), so both triangular
// solves read contiguous band rows: blocks of 64 rows are staged in LDS by the
// whole workgroup, the contributions of earlier (forward) or later (backward)
// blocks are dot products split over the waves, and the 64 x 64 diagonal
// triangle is a sweep in wave 0 (lane = row) with readlane broadcasts.
// Solution values of the last bw rows live in an LDS ring.  Global loads are
// issued unconditionally (clamped addresses) so that they pipeline.
constexpr int kPanel = 16;
constexpr int kPanelStride = kPanel + 1;                   // LDS row stride (doubles), bank spread
constexpr int kPanelSlotsMax = 4;                          // rows per lane in the panel
constexpr int kBandMaxBw = 64 * kPanelSlotsMax - kPanel;   // 240
constexpr int kBandNT = 256;
constexpr int kRing = 256;                                 // power of two > kBandMaxBw

typedef double band_dbl4 __attribute__((ext_vector_type(4)));

__device__ inline double rdlane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// dynamic LDS of the band solve (doubles): max(panel staging, 64 solve rows) + ring + partial sums
inline size_t band_lds_bytes(int bw) {
    const size_t panel = 2 * (size_t)(kPanel + kBandMaxBw) * kPanelStride;
    const size_t rows = 64 * (size_t)(bw + 1);
    return sizeof(double) * (std::max(panel, rows) + kRing + 4 * 64);
}

// Both triangular solves of K du = -R on a stored band factor (L below the
// diagonal and D on it in K's rows, the transposed copy in Kt), by one
// workgroup of kBandNT threads: forward (pass 0) L y = -R on K, backward (pass
// 1) x = D^-1 y - L^T x on Kt; blocks of 64 rows staged in LDS (band_lds, of
// band_lds_bytes(bw) bytes).
__device__ void band_solves(const double* __restrict__ K, const double* __restrict__ Kt, const double* __restrict__ R,
                            int n, int bw, double* __restrict__ du, double* band_lds) {
    const int ld = bw + 1, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const size_t big = std::max<size_t>(2 * (size_t)(kPanel + kBandMaxBw) * kPanelStride, 64 * (size_t)ld);
    double* Kb = band_lds;
    double* ring = band_lds + big;
    double* red = ring + kRing;
    for (int pass = 0; pass < 2; ++pass) {
        const double* Src = pass == 0 ? K : Kt;
        const int nblk64 = (n + 63) / 64;
        for (int bi = 0; bi < nblk64; ++bi) {
            const int i0 = (pass == 0 ? bi : nblk64 - 1 - bi) * 64;
            const int rows = min(64, n - i0);
            const int64_t base = (int64_t)i0 * ld;
            const int cnt = rows * ld;
            for (int e = tid; e < cnt; e += kBandNT) Kb[e] = Src[base + e];
            __syncthreads();
            // contributions of rows outside the block, split over the waves
            const int i = i0 + lane;
            double sdot = 0.0;
            if (lane < rows) {
                if (pass == 0) {
                    // t = i - j with j < i0
                    const int tmax = min(i, bw);
                    for (int t = lane + 1 + wave; t <= tmax; t += 4)
                        sdot += Kb[lane * ld + t] * ring[(i - t) & (kRing - 1)];
                } else {
                    // t = j - i with j >= i0 + 64
                    const int tmax = min(n - 1 - i, bw);
                    for (int t = 64 - lane + wave; t <= tmax; t += 4)
                        sdot += Kb[lane * ld + t] * ring[(i + t) & (kRing - 1)];
                }
            }
            red[wave * 64 + lane] = sdot;
            __syncthreads();
            if (wave == 0) {
                double acc = 0.0;
                if (lane < rows) {
                    const double s4 = red[lane] + red[64 + lane] + red[128 + lane] + red[192 + lane];
                    acc = pass == 0 ? -R[i] - s4 : du[i] / Kb[lane * ld] - s4;  // du[i]: stored by this lane
                }
                if (pass == 0) {
                    for (int k = 0; k < rows; ++k) {
                        const double yk = rdlane(acc, k);
                        const int off = lane - k;
                        const double l = Kb[lane * ld + ((off > 0 && off <= bw && lane < rows) ? off : 0)];
                        if (off > 0 && off <= bw && lane < rows) acc -= l * yk;
                    }
                } else {
                    for (int k = rows - 1; k >= 0; --k) {
                        const double xk = rdlane(acc, k);
                        const int off = k - lane;
                        const double l = Kb[lane * ld + ((off > 0 && off <= bw) ? off : 0)];
                        if (off > 0 && off <= bw) acc -= l * xk;
                    }
                }
                if (lane < rows) {
                    ring[i & (kRing - 1)] = acc;
                    du[i] = acc;
                }
            }
            __syncthreads();
        }
    }
}

template <int SLOTS>
__global__ __launch_bounds__(kBandNT) void macro_band_solve_blocked(double* __restrict__ K, double* __restrict__ Kt,
                                                                    const double* __restrict__ R, int n, int bw,
                                                                    double* __restrict__ du, int* __restrict__ flag,
                                                                    const int* __restrict__ done) {
    if (*done) return;
    extern __shared__ double band_lds[];
    const int ld = bw + 1, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const size_t big = std::max<size_t>(2 * (size_t)(kPanel + kBandMaxBw) * kPanelStride, 64 * (size_t)ld);
    double* Ls = band_lds;                                          // scaled panel columns L[r][c]
    double* Ws = band_lds + (kPanel + kBandMaxBw) * kPanelStride;   // L[r][c] * D[c]
    (void)big;
    for (int k0 = 0; k0 < n; k0 += kPanel) {
        const int nb = min(kPanel, n - k0);
        const int m = min(n - k0, nb + bw);  // rows touched by the panel
        if (wave == 0) {
            double pv[SLOTS][kPanel];
#pragma clang loop unroll(full)
            for (int s = 0; s < SLOTS; ++s) {
                const int rr = lane + 64 * s, r = k0 + rr;
#pragma clang loop unroll(full)
                for (int c = 0; c < kPanel; ++c) {
                    const int off = rr - c;  // r - (k0 + c)
                    const bool in = c < nb && rr < m && off >= 0 && off <= bw;
                    const double v = K[in ? (int64_t)r * ld + off : 0];
                    pv[s][c] = in ? v : 0.0;
                }
            }
#pragma clang loop unroll(full)
            for (int c = 0; c < kPanel; ++c) {
                if (c < nb) {
                    const double piv = rdlane(pv[0][c], c);
                    if (lane == 0 && (!(fabs(piv) > 0.0) || !isfinite(piv))) *flag = 1;
                    const double inv = 1.0 / piv;
                    double colv[kPanel];
#pragma clang loop unroll(full)
                    for (int j = 0; j < kPanel; ++j) colv[j] = (j > c) ? rdlane(pv[0][c], j) : 0.0;
                    // rows at or above the pivot get l = 0 (predicated, no branch)
#pragma clang loop unroll(full)
                    for (int s = 0; s < SLOTS; ++s) {
                        const int rr = lane + 64 * s;
                        const double l = (rr > c) ? pv[s][c] * inv : 0.0;
#pragma clang loop unroll(full)
                        for (int j = c + 1; j < kPanel; ++j) pv[s][j] -= (rr >= j) ? l * colv[j] : 0.0;
                        pv[s][c] = (rr > c) ? l : pv[s][c];
                    }
                }
            }
            // write back (L below the diagonal, D on it; transposed copy in Kt) and
            // stage L, L*D for the update
            double dcol[kPanel];
#pragma clang loop unroll(full)
            for (int c = 0; c < kPanel; ++c) dcol[c] = rdlane(pv[0][c], c);
#pragma clang loop unroll(full)
            for (int s = 0; s < SLOTS; ++s) {
                const int rr = lane + 64 * s, r = k0 + rr;
                if (rr < m) {
#pragma clang loop unroll(full)
                    for (int c = 0; c < kPanel; ++c) {
                        const int off = rr - c;
                        const bool in = c < nb && off >= 0 && off <= bw;
                        if (in) {
                            K[(int64_t)r * ld + off] = pv[s][c];
                            Kt[(int64_t)(k0 + c) * ld + off] = pv[s][c];
                        }
                        const double l = (in && off > 0) ? pv[s][c] : 0.0;
                        Ls[rr * kPanelStride + c] = l;
                        Ws[rr * kPanelStride + c] = l * dcol[c];
                    }
                }
            }
        }
        __syncthreads();
        // trailing update: K[i][j] -= sum_c L[i][c] D[c] L[j][c] for nb <= j <= i < m
        // trailing update on FP64 MFMA: 16 x 16 lower-triangle tiles of the
        // (T x 16)(16 x T) product, two tiles per wave and pass (their old values
        // are loaded before the MFMAs)
        {
            const int T = m - nb;
            const int n16 = (T + 15) >> 4;
            const int ntile = n16 * (n16 + 1) / 2;
            for (int tt = 2 * wave; tt < ntile; tt += 8) {
                int Ii[2], Jj[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int t = tt + u;
                    int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
                    if ((r + 1) * (r + 2) / 2 <= t) ++r;
                    if (r * (r + 1) / 2 > t) --r;
                    Ii[u] = r;
                    Jj[u] = t - r * (r + 1) / 2;
                }
                double old[2][4];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 16 * Ii[u] + (lane >> 4) + 4 * v, col = 16 * Jj[u] + (lane & 15);
                        const bool in = tt + u < ntile && row < T && col <= row;
                        old[u][v] = K[in ? (int64_t)(k0 + nb + row) * ld + (row - col) : 0];
                    }
                band_dbl4 acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int kk = 4 * ks + (lane >> 4);
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int ra = nb + 16 * Ii[u] + (lane & 15), rb = nb + 16 * Jj[u] + (lane & 15);
                        const double av = Ls[(ra < m ? ra : 0) * kPanelStride + kk];
                        const double bv = Ws[(rb < m ? rb : 0) * kPanelStride + kk];
                        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra < m ? av : 0.0, rb < m ? bv : 0.0, acc[u],
                                                                     0, 0, 0);
                    }
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 16 * Ii[u] + (lane >> 4) + 4 * v, col = 16 * Jj[u] + (lane & 15);
                        if (tt + u < ntile && row < T && col <= row)
                            K[(int64_t)(k0 + nb + row) * ld + (row - col)] = old[u][v] - acc[u][v];
                    }
            }
        }
        __syncthreads();
    }
    band_solves(K, Kt, R, n, bw, du, band_lds);
}

// Banded LDL^T with the active window held in LDS, for bandwidths whose window
// spans at most kWinMax tile rows.  The band is cut into 16 x 16 tiles.  The
// part that later panels still update -- below panel kt, tile rows kt .. kt +
// ntw - 1 (ntw = (bw + 15) / 16 + 1), lower triangle, at most 55 tiles -- stays
// in LDS for the whole factorization: diagonal d = I - J keeps its ntw - d tiles
// of the window in a ring, tile (I, J) at slot base(d) + J mod (ntw - d), so the
// row that enters when the window moves on takes exactly the slots of the
// retired panel column.  Per panel (tile column kt), one workgroup of four
// waves: wave 0 factors the diagonal tile (lane = row, readlane broadcasts) and
// forms W = L11^-T D^-1; the tiles below become L = A W on MFMA (in place); the
// factor goes out to K and Kt (band entries only); the trailing tiles take -L(I)
// D L(J)^T on MFMA; the entering tile row, read from K while the panel is
// processed (no earlier panel reaches it), is stored.  The matrix is read once
// and the factor written once, and no global round trip sits on the panel
// chain.  Rows and columns past n are padded with the identity.
constexpr int kWinMax = 10;                                  // tile rows of the window (bw <= 144)
constexpr int kWinSlots = kWinMax * (kWinMax + 1) / 2;       // window tiles
constexpr int kWinWaves = 4;
constexpr int kWinNT = 64 * kWinWaves;
constexpr int kWinStride = 17;                               // LDS row stride of a tile (doubles)
constexpr int kWinTile = 16 * kWinStride;
inline size_t band_win_lds_bytes() {
    return sizeof(double) * ((size_t)(kWinSlots + kWinMax) * kWinTile + 256 + 16) +
           sizeof(int) * (2 * kWinMax * kWinMax);
}
inline bool band_win_fits(int bw) { return (bw + 15) / 16 + 1 <= kWinMax; }

__device__ inline int win_slot(int I, int J, int ntw) {
    const int d = I - J;
    return d * ntw - ((d * (d - 1)) >> 1) + J % (ntw - d);
}

// entry (r, c) of the band matrix (lower band from K, identity past n); the
// read is unconditional, at a clamped address, and its value enters through a
// 0/1 factor (a select would let the compiler move the read under a branch and
// wait for it there)
__device__ inline double band_at(const double* __restrict__ K, int n, int bw, int r, int c) {
    const int off = r - c;
    const bool in = (r < n) & (c < n) & (off >= 0) & (off <= bw);
    const double x = K[in ? (int64_t)r * (bw + 1) + off : 0];
    return fma(x, in ? 1.0 : 0.0, ((r == c) & (r >= n)) ? 1.0 : 0.0);
}

__device__ inline double recip_nr64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// B. by one wave: LDL^T of the diagonal tile T of panel kt (lane = row, readlane
// broadcasts), W = L11^-T D^-1 from the rows of L11^-1 into Wm, the pivots into
// Dv, the tile's factor rows out to K and Kt
__device__ __forceinline__ void win_diag(const double* T, double* Wm, double* Dv, int kt, int n, int bw,
                                         double* __restrict__ K, double* __restrict__ Kt, int* __restrict__ flag,
                                         int lane) {
    const int ld = bw + 1;
    const bool own = lane < 16;
    double a[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) a[c] = (own && c <= lane) ? T[(lane & 15) * kWinStride + c] : 0.0;
    double dpiv = 1.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const double piv = rdlane(a[j], j);
        if (lane == j) {
            dpiv = piv;
            if (!(fabs(piv) > 0.0) || !isfinite(piv)) *flag = 1;
        }
        const double l = (own && lane > j) ? a[j] * recip_nr64(piv) : 0.0;
        const double lp = l * piv;
#pragma unroll
        for (int cc = j + 1; cc < 16; ++cc) a[cc] -= lp * rdlane(l, cc);
        if (lane > j) a[j] = l;
    }
    // row `lane` of L11^-1 (unit lower), by forward substitution
    double li[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) li[cc] = (cc == lane) ? 1.0 : 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const double le = (own && lane > e) ? a[e] : 0.0;
#pragma unroll
        for (int cc = 0; cc <= e; ++cc) li[cc] -= le * rdlane(li[cc], e);
    }
    if (own) {
        const double rd = recip_nr64(dpiv);
#pragma unroll
        for (int k = 0; k < 16; ++k) Wm[k * 16 + lane] = li[k] * rd;
        Dv[lane] = dpiv;
        const int r = 16 * kt + lane;
        if (r < n) {
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int off = lane - c;
                if (off >= 0 && off <= bw) {
                    const double v = off == 0 ? dpiv : a[c];
                    K[(int64_t)r * ld + off] = v;
                    Kt[(int64_t)(16 * kt + c) * ld + off] = v;
                }
            }
        }
    }
}

// C. the panel tiles below the diagonal owned by wave W (o = W + 1, W + 5, ...):
// L = A W on MFMA, in place, L D to LDp, the factor out to K and Kt
template <int W>
__device__ __forceinline__ void win_panel(double* Wn, double* LDp, const double* Wm, const double* Dv,
                                          const int* slot, int rows_w, int kt, int n, int bw,
                                          double* __restrict__ K, double* __restrict__ Kt, int lane) {
    constexpr int NO = (kWinMax - 1 - W + kWinWaves - 1) / kWinWaves;  // tiles of this wave
    const int ld = bw + 1, c = lane & 15, gc = 16 * kt + c;
    double av[NO > 0 ? NO : 1][4];
    double* T[NO > 0 ? NO : 1];
    double wv[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) wv[ks] = Wm[(4 * ks + (lane >> 4)) * 16 + c];
#pragma unroll
    for (int q = 0; q < NO; ++q) {
        const int o = W + 1 + kWinWaves * q;
        T[q] = Wn + slot[min(o, rows_w - 1) * kWinMax] * kWinTile;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) av[q][ks] = T[q][c * kWinStride + 4 * ks + (lane >> 4)];
    }
    const double dc = Dv[c];
#pragma unroll
    for (int q = 0; q < NO; ++q) {
        const int o = W + 1 + kWinWaves * q;
        if (o < rows_w) {
            band_dbl4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) t = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q][ks], wv[ks], t, 0, 0, 0);
            double* LDt = LDp + o * kWinTile;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = (lane >> 4) + 4 * v, r = 16 * (kt + o) + rr, off = r - gc;
                T[q][rr * kWinStride + c] = t[v];
                LDt[rr * kWinStride + c] = t[v] * dc;
                if (r < n && off <= bw) {
                    K[(int64_t)r * ld + off] = t[v];
                    Kt[(int64_t)gc * ld + off] = t[v];
                }
            }
        }
    }
}

// D. the trailing tiles owned by wave W: tile (kt + oi, kt + oj), 1 <= oj <= oi,
// numbered t = (oi - 1) oi / 2 + oj - 1; wave 0 takes t = 0 (the next diagonal
// tile, which it factors right after), waves 1 .. 3 the others in turn.  Every
// operand is read first, then the MFMAs run, then the tiles are stored.
__device__ constexpr bool win_owns(int W, int t) { return W == 0 ? t == 0 : (t > 0 && (t - 1) % (kWinWaves - 1) == W - 1); }

template <int W>
__device__ __forceinline__ void win_trailing(double* Wn, const double* LDp, const int* slot, int rows_w, int lane) {
    const int c = lane & 15, kq = lane >> 4;
    double aI[kWinMax][4], bJ[kWinMax][4];
#pragma unroll
    for (int o = 1; o < (W == 0 ? 2 : kWinMax); ++o) {
        const double* LDt = LDp + min(o, rows_w - 1) * kWinTile;
        const double* Lt = Wn + slot[min(o, rows_w - 1) * kWinMax] * kWinTile;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            aI[o][ks] = -LDt[c * kWinStride + 4 * ks + kq];
            bJ[o][ks] = Lt[c * kWinStride + 4 * ks + kq];
        }
    }
    constexpr int NTT = (kWinMax - 1) * kWinMax / 2;
    constexpr int NT = W == 0 ? 1 : (NTT - 1 - (W - 1) + kWinWaves - 2) / (kWinWaves - 1);
    band_dbl4 acc[NT];
    double* C[NT];
    {
        int q = 0;
#pragma unroll
        for (int oi = 1; oi < kWinMax; ++oi)
#pragma unroll
            for (int oj = 1; oj <= oi; ++oj)
                if (win_owns(W, (oi - 1) * oi / 2 + oj - 1)) {
                    C[q] = Wn + slot[min(oi, rows_w - 1) * kWinMax + min(oj, rows_w - 1)] * kWinTile;
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[q][v] = C[q][(kq + 4 * v) * kWinStride + c];
                    ++q;
                }
    }
    {
        int q = 0;
#pragma unroll
        for (int oi = 1; oi < kWinMax; ++oi)
#pragma unroll
            for (int oj = 1; oj <= oi; ++oj)
                if (win_owns(W, (oi - 1) * oi / 2 + oj - 1)) {
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks)
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(aI[oi][ks], bJ[oj][ks], acc[q], 0, 0, 0);
                    ++q;
                }
    }
    {
        int q = 0;
#pragma unroll
        for (int oi = 1; oi < kWinMax; ++oi)
#pragma unroll
            for (int oj = 1; oj <= oi; ++oj)
                if (win_owns(W, (oi - 1) * oi / 2 + oj - 1)) {
                    if (oi < rows_w) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) C[q][(kq + 4 * v) * kWinStride + c] = acc[q][v];
                    }
                    ++q;
                }
    }
}

__global__ __launch_bounds__(kWinNT) void macro_band_factor_window(double* __restrict__ K, double* __restrict__ Kt,
                                                                  int n, int bw, int* __restrict__ flag,
                                                                  const int* __restrict__ done) {
    if (*done) return;
    extern __shared__ double win_lds[];
    double* Wn = win_lds;                        // window tiles, [kWinSlots][16][kWinStride]
    double* LDp = Wn + kWinSlots * kWinTile;     // the panel's L tiles with column c scaled by D[c]
    double* Wm = LDp + kWinMax * kWinTile;       // W[k * 16 + c]
    double* Dv = Wm + 256;                       // the panel's pivots
    int* slots = reinterpret_cast<int*>(Dv + 16);  // two buffers of the panel's window-tile slots
    const int ld = bw + 1, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ntw = (bw + 15) / 16 + 1, nt = (n + 15) / 16;
    const int pr = tid >> 4, pc = tid & 15;      // this thread's element of a staged tile
    for (int I = 0; I < min(ntw, nt); ++I)
        for (int J = 0; J <= I; ++J)
            Wn[win_slot(I, J, ntw) * kWinTile + pr * kWinStride + pc] = band_at(K, n, bw, 16 * I + pr, 16 * J + pc);
    // slots of panel kt's window tiles: slot[oi * kWinMax + oj] holds tile (kt +
    // oi, kt + oj); two buffers (a panel's E still reads its own while the next
    // table is written)
    auto fill_slots = [&](int kt) {
        int* slot = slots + (kt & 1) * kWinMax * kWinMax;
        if (tid < kWinMax * kWinMax) {
            const int oi = tid / kWinMax, oj = tid - oi * kWinMax;
            if (oj <= oi && oi < ntw) slot[tid] = win_slot(kt + oi, kt + oj, ntw);
        }
    };
    fill_slots(0);
    __syncthreads();
    if (wave == 0) win_diag(Wn + slots[0] * kWinTile, Wm, Dv, 0, n, bw, K, Kt, flag, lane);
    __syncthreads();
    // per panel kt (its diagonal tile already factored): C, then D with the next
    // panel's diagonal tile updated and factored by wave 0 while the other waves
    // update the rest of the window, then E
    for (int kt = 0; kt < nt; ++kt) {
        const int rows_w = min(ntw, nt - kt);
        const int* slot = slots + (kt & 1) * kWinMax * kWinMax;
        // the tile row that enters after this panel: tiles (In, In - d), d < ntw;
        // it takes the slots of the retired panel tiles (kt + d, kt)
        const int In = kt + ntw;
        const bool enter = In < nt;
        double pf[kWinMax];
#pragma unroll
        for (int d = 0; d < kWinMax; ++d) pf[d] = band_at(K, enter ? n : 0, bw, 16 * In + pr, 16 * (In - d) + pc);
        // C. the tiles below the diagonal: L = A W, in place
        switch (wave) {
            case 0: win_panel<0>(Wn, LDp, Wm, Dv, slot, rows_w, kt, n, bw, K, Kt, lane); break;
            case 1: win_panel<1>(Wn, LDp, Wm, Dv, slot, rows_w, kt, n, bw, K, Kt, lane); break;
            case 2: win_panel<2>(Wn, LDp, Wm, Dv, slot, rows_w, kt, n, bw, K, Kt, lane); break;
            default: win_panel<3>(Wn, LDp, Wm, Dv, slot, rows_w, kt, n, bw, K, Kt, lane); break;
        }
        __syncthreads();
        // D. the trailing tiles; wave 0 then factors panel kt + 1's diagonal tile
        //    (Wm and Dv are free: C has read them)
        switch (wave) {
            case 0:
                win_trailing<0>(Wn, LDp, slot, rows_w, lane);
                if (kt + 1 < nt) {
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    win_diag(Wn + slot[kWinMax + 1] * kWinTile, Wm, Dv, kt + 1, n, bw, K, Kt, flag, lane);
                }
                break;
            case 1: win_trailing<1>(Wn, LDp, slot, rows_w, lane); break;
            case 2: win_trailing<2>(Wn, LDp, slot, rows_w, lane); break;
            default: win_trailing<3>(Wn, LDp, slot, rows_w, lane); break;
        }
        __syncthreads();
        // E. the entering tile row into the retired panel tiles' slots; the next
        //    panel's slot table
        if (enter) {
#pragma unroll
            for (int d = 0; d < kWinMax; ++d)
                if (d < ntw) Wn[slot[d * kWinMax] * kWinTile + pr * kWinStride + pc] = pf[d];
        }
        fill_slots(kt + 1);
        __syncthreads();
    }
}

// Both triangular solves of K du = -R on the band factor of
// macro_band_factor_window (bw <= 144), one workgroup: forward L y = -R on K,
// then x = D^-1 y - L^T x on Kt (row j of Kt holds column j of L), in blocks of
// 64 rows.  Each block is staged in LDS while the previous one is solved
// (double buffer; the next block's rows are read into registers first).  The
// contributions of earlier (forward) or later (backward) rows are dot products
// over the LDS ring of solved values, split over the four waves; the block's
// own 64 x 64 triangle is a sweep in wave 0 (lane = row, readlane broadcasts)
// with every factor entry of the lane's row read before the sweep.
constexpr int kSolveBlk = 64;
constexpr int kSolvePer = (kSolveBlk * (16 * kWinMax - 15) + kBandNT - 1) / kBandNT;  // staged doubles per thread
inline size_t band_solve_win_lds_bytes(int bw) {
    return sizeof(double) * (2 * (size_t)kSolveBlk * (bw + 1) + kRing + 4 * 64);
}

__global__ __launch_bounds__(kBandNT) void macro_band_solves_win(const double* __restrict__ K,
                                                                const double* __restrict__ Kt,
                                                                const double* __restrict__ R, int n, int bw,
                                                                double* __restrict__ du,
                                                                const int* __restrict__ done) {
    if (*done) return;
    extern __shared__ double sv_lds[];
    const int ld = bw + 1, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int bsz = kSolveBlk * ld;
    double* ring = sv_lds + 2 * bsz;
    double* red = ring + kRing;
    const int nb = (n + kSolveBlk - 1) / kSolveBlk;
    double pre[kSolvePer];
    for (int pass = 0; pass < 2; ++pass) {
        const double* Src = pass == 0 ? K : Kt;
        // the rows of block bi: forward in increasing, backward in decreasing order
        auto row0 = [&](int bi) { return (pass == 0 ? bi : nb - 1 - bi) * kSolveBlk; };
        auto fetch = [&](int bi) {
            const int r0 = row0(bi), cnt = min(kSolveBlk, n - r0) * ld;
            const double* src = Src + (int64_t)r0 * ld;
#pragma unroll
            for (int q = 0; q < kSolvePer; ++q) {
                const int e = tid + kBandNT * q;
                pre[q] = src[e < cnt ? e : 0];
            }
        };
        auto stage = [&](int bi) {
            const int r0 = row0(bi), cnt = min(kSolveBlk, n - r0) * ld;
            double* dst = sv_lds + (bi & 1) * bsz;
#pragma unroll
            for (int q = 0; q < kSolvePer; ++q) {
                const int e = tid + kBandNT * q;
                if (e < cnt) dst[e] = pre[q];
            }
        };
        fetch(0);
        stage(0);
        __syncthreads();
        for (int bi = 0; bi < nb; ++bi) {
            const double* Kb = sv_lds + (bi & 1) * bsz;
            const int i0 = row0(bi), rows = min(kSolveBlk, n - i0), i = i0 + lane;
            if (bi + 1 < nb) fetch(bi + 1);
            // contributions of rows outside the block
            double s0 = 0.0, s1 = 0.0;
            if (lane < rows) {
                if (pass == 0) {
                    const int tmax = min(i, bw);  // t = i - j, j < i0
                    int t = lane + 1 + wave;
                    for (; t + 4 <= tmax; t += 8) {
                        s0 += Kb[lane * ld + t] * ring[(i - t) & (kRing - 1)];
                        s1 += Kb[lane * ld + t + 4] * ring[(i - t - 4) & (kRing - 1)];
                    }
                    if (t <= tmax) s0 += Kb[lane * ld + t] * ring[(i - t) & (kRing - 1)];
                } else {
                    const int tmax = min(n - 1 - i, bw);  // t = j - i, j >= i0 + 64
                    int t = kSolveBlk - lane + wave;
                    for (; t + 4 <= tmax; t += 8) {
                        s0 += Kb[lane * ld + t] * ring[(i + t) & (kRing - 1)];
                        s1 += Kb[lane * ld + t + 4] * ring[(i + t + 4) & (kRing - 1)];
                    }
                    if (t <= tmax) s0 += Kb[lane * ld + t] * ring[(i + t) & (kRing - 1)];
                }
            }
            red[wave * 64 + lane] = s0 + s1;
            __syncthreads();
            if (wave == 0) {
                double acc = 0.0;
                if (lane < rows) {
                    const double s4 = red[lane] + red[64 + lane] + red[128 + lane] + red[192 + lane];
                    acc = pass == 0 ? -R[i] - s4 : du[i] / Kb[lane * ld] - s4;  // du[i]: stored by this lane
                }
                const int lr = min(lane, rows - 1);
                if (pass == 0) {
                    double l[kSolveBlk];
#pragma unroll
                    for (int k = 0; k < kSolveBlk; ++k) {
                        const int off = lane - k;
                        l[k] = ((off > 0) & (off <= bw)) ? Kb[lr * ld + (off > 0 && off <= bw ? off : 0)] : 0.0;
                    }
#pragma unroll
                    for (int k = 0; k < kSolveBlk; ++k) acc -= l[k] * rdlane(acc, k);
                } else {
                    double l[kSolveBlk];
#pragma unroll
                    for (int k = 0; k < kSolveBlk; ++k) {
                        const int off = k - lane;
                        l[k] = ((off > 0) & (off <= bw)) ? Kb[lr * ld + (off > 0 && off <= bw ? off : 0)] : 0.0;
                    }
#pragma unroll
                    for (int k = kSolveBlk - 1; k >= 0; --k) acc -= l[k] * rdlane(acc, k);
                }
                if (lane < rows) {
                    ring[i & (kRing - 1)] = acc;
                    du[i] = acc;
                }
            }
            if (bi + 1 < nb) stage(bi + 1);
            __syncthreads();
        }
    }
}

// u += du on free dofs; in the first iteration of a step (dud non-null) the
// fixed dofs take the prescribed increment
__global__ void macro_update(double* __restrict__ u, const double* __restrict__ du, const int* __restrict__ fixed,
                             const double* __restrict__ dud, int ndof, const int* __restrict__ done) {
    if (*done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ndof) return;
    if (!fixed[i]) u[i] += du[i];
    else if (dud) u[i] += dud[i];
}

inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

struct fehmm_s {
    fehmm_desc desc{};
    int nnode = 0, nelem = 0, ndof = 0, nqp = 0, bw = 0;
    std::vector<double> xy;
    std::vector<int> conn, fixed;
    std::vector<std::vector<int>> colour;
    MacroGeom geom{};
    rve_batch batch = nullptr;
    int64_t state_doubles = 0;
    hipStream_t stream = nullptr;
    // device
    int *d_conn = nullptr, *d_fixed = nullptr, *d_col[4] = {nullptr, nullptr, nullptr, nullptr};
    int *d_status = nullptr, *d_iters = nullptr, *d_rightx = nullptr;
    StepState* d_state = nullptr;
    double *d_u = nullptr, *d_du = nullptr, *d_F = nullptr, *d_P = nullptr, *d_A = nullptr;
    double* d_dud = nullptr;  // prescribed increment of the load step (0 on free dofs)
    double *d_w = nullptr, *d_ke = nullptr, *d_fe = nullptr, *d_K = nullptr, *d_R = nullptr, *d_norm = nullptr;
    double* d_Kt = nullptr;  // transposed copy of the band factor (blocked band solve)
    // surrogate replacement of micro solves
    rve_surrogate surr = nullptr;
    float surr_thr = 0.f;
    int surr_prec = RVE_SURR_BF16X3;
    double surr_rtol = 1e-4;
    float* d_ind = nullptr;
    int32_t *d_sidx = nullptr, *d_scnt = nullptr, *d_smask = nullptr;
    // a whole load step captured as one graph (fehmm_set_graph)
    bool graph_on = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool alive = true;
};

#define FH_HIP(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return set_error(RVE_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

static void fehmm_free(fehmm_s* h) {
    int* ip[] = {h->d_conn, h->d_fixed, h->d_col[0], h->d_col[1], h->d_col[2], h->d_col[3], h->d_status,
                 h->d_iters, h->d_rightx};
    for (int* p : ip) (void)hipFree(p);
    (void)hipFree(h->d_state);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
    double* dp[] = {h->d_Kt, h->d_u, h->d_du, h->d_dud, h->d_F, h->d_P, h->d_A, h->d_w, h->d_ke, h->d_fe, h->d_K,
                    h->d_R, h->d_norm};
    for (double* p : dp) (void)hipFree(p);
    (void)hipFree(h->d_ind);
    (void)hipFree(h->d_sidx);
    (void)hipFree(h->d_scnt);
    (void)hipFree(h->d_smask);
    if (h->batch) rve_batch_destroy(h->batch);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    h->batch = nullptr;
}

extern "C" {

int fehmm_create(const fehmm_desc* d, fehmm* out) {
    if (!d || !out) return set_error(RVE_EINVAL, "fehmm_create: NULL argument");
    *out = nullptr;
    if (d->nx < 1 || d->ny < 1 || d->nx > 4096 || d->ny > 4096 || !(d->Lx > 0) || !(d->Ly > 0))
        return set_error(RVE_EINVAL, "fehmm_create: bad macro grid");
    if (d->bc != FEHMM_BC_CLAMPED_PULL && d->bc != FEHMM_BC_UNIAXIAL)
        return set_error(RVE_EINVAL, "fehmm_create: unknown boundary condition");
    if (d->elem != FEHMM_ELEM_Q1 && d->elem != FEHMM_ELEM_P1)
        return set_error(RVE_EINVAL, "fehmm_create: unknown macro element kind");
    if (d->scheme != FEHMM_NESTED && d->scheme != FEHMM_ALTERNATING)
        return set_error(RVE_EINVAL, "fehmm_create: unknown scheme");
    if (d->nsteps < 1 || !(d->rtol_macro > 0) || d->max_macro_iter < 1 || d->max_macro_iter > FEHMM_MAX_HIST - 1)
        return set_error(RVE_EINVAL, "fehmm_create: bad load-step or Newton settings");
    if (!d->micro) return set_error(RVE_EINVAL, "fehmm_create: micro mesh required");
    static bool band_prepared = false;
    if (!band_prepared) {
        const int lds = (int)band_lds_bytes(kBandMaxBw);
        FH_HIP(hipFuncSetAttribute((const void*)macro_band_solve_blocked<3>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds));
        FH_HIP(hipFuncSetAttribute((const void*)macro_band_solve_blocked<4>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds));
        FH_HIP(hipFuncSetAttribute((const void*)macro_band_solves_win, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)band_solve_win_lds_bytes(16 * kWinMax - 16)));
        FH_HIP(hipFuncSetAttribute((const void*)macro_band_factor_window, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)band_win_lds_bytes()));
        band_prepared = true;
    }
    auto h = std::make_unique<fehmm_s>();
    h->desc = *d;
    const int nx = d->nx, ny = d->ny;
    const double hx = d->Lx / nx, hy = d->Ly / ny;
    // shape gradients at the integration points of a rectangle hx x hy: Q1 at
    // its 2 x 2 Gauss points, or the P1 triangles (0,1,2), (0,2,3) of the
    // counter-clockwise cell nodes, one point each (constant gradients)
    std::memset(h->geom.dN, 0, sizeof(h->geom.dN));
    if (d->elem == FEHMM_ELEM_P1) {
        h->geom.npt = 2;
        h->geom.dN[0][0][0] = -1.0 / hx;
        h->geom.dN[0][1][0] = 1.0 / hx;
        h->geom.dN[0][1][1] = -1.0 / hy;
        h->geom.dN[0][2][1] = 1.0 / hy;
        h->geom.dN[1][0][1] = -1.0 / hy;
        h->geom.dN[1][2][0] = 1.0 / hx;
        h->geom.dN[1][3][0] = -1.0 / hx;
        h->geom.dN[1][3][1] = 1.0 / hy;
        h->geom.wdet = 0.5 * hx * hy;
    } else {
        h->geom.npt = 4;
        const int sx[4] = {-1, 1, 1, -1}, sy[4] = {-1, -1, 1, 1};
        const double g = 1.0 / std::sqrt(3.0);
        for (int p = 0; p < 4; ++p) {
            const double xi = sx[p] * g, eta = sy[p] * g;
            for (int a = 0; a < 4; ++a) {
                h->geom.dN[p][a][0] = 0.25 * sx[a] * (1 + sy[a] * eta) * 2.0 / hx;
                h->geom.dN[p][a][1] = 0.25 * sy[a] * (1 + sx[a] * xi) * 2.0 / hy;
            }
        }
        h->geom.wdet = 0.25 * hx * hy;
    }
    std::vector<int> keep(nx * ny), used((nx + 1) * (ny + 1), 0), ecol;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double cx = (i + 0.5) * hx - 0.5 * d->Lx, cy = (j + 0.5) * hy - 0.5 * d->Ly;
            keep[j * nx + i] = !(d->hole_r > 0 && std::sqrt(cx * cx + cy * cy) < d->hole_r);
        }
    std::vector<int> id((nx + 1) * (ny + 1), -1);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            if (keep[j * nx + i])
                used[j * (nx + 1) + i] = used[j * (nx + 1) + i + 1] = used[(j + 1) * (nx + 1) + i] =
                    used[(j + 1) * (nx + 1) + i + 1] = 1;
    for (int k = 0; k < (nx + 1) * (ny + 1); ++k)
        if (used[k]) id[k] = h->nnode++;
    if (h->nnode == 0) return set_error(RVE_EINVAL, "fehmm_create: the hole removes every element");
    h->xy.resize(2 * h->nnode);
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i)
            if (id[j * (nx + 1) + i] >= 0) {
                h->xy[2 * id[j * (nx + 1) + i]] = i * hx;
                h->xy[2 * id[j * (nx + 1) + i] + 1] = j * hy;
            }
    h->colour.resize(4);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            if (keep[j * nx + i]) {
                const int e = h->nelem++;
                h->conn.push_back(id[j * (nx + 1) + i]);
                h->conn.push_back(id[j * (nx + 1) + i + 1]);
                h->conn.push_back(id[(j + 1) * (nx + 1) + i + 1]);
                h->conn.push_back(id[(j + 1) * (nx + 1) + i]);
                h->colour[(i & 1) + 2 * (j & 1)].push_back(e);
            }
    h->ndof = 2 * h->nnode;
    h->nqp = h->geom.npt * h->nelem;
    h->fixed.assign(h->ndof, 0);
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            const int v = id[j * (nx + 1) + i];
            if (v < 0) continue;
            if (i == 0) {
                h->fixed[2 * v] = 1;
                if (d->bc == FEHMM_BC_CLAMPED_PULL || j == 0) h->fixed[2 * v + 1] = 1;
            }
            if (i == nx) h->fixed[2 * v] = 1;
        }
    for (int e = 0; e < h->nelem; ++e)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                h->bw = std::max(h->bw, std::abs(2 * h->conn[4 * e + a] - 2 * h->conn[4 * e + b]) + 1);
    // one RVE per Gauss point
    std::vector<rve_mesh> meshes(h->nqp, d->micro);
    int st = rve_batch_create(meshes.data(), h->nqp, &h->batch);
    if (st) return st;
    std::vector<int64_t> off(h->nqp + 1);
    rve_batch_state_offsets(h->batch, off.data());
    h->state_doubles = off[h->nqp];
    FH_HIP(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    std::vector<int> rightx(h->ndof, 0);  // x dofs of the right edge (prescribed stretch)
    for (int v = 0; v < h->nnode; ++v)
        if (h->fixed[2 * v] && h->xy[2 * v] > 0.5 * d->Lx) rightx[2 * v] = 1;
    auto up = [&](auto** p, const auto& v) -> int {
        using T = typename std::remove_reference<decltype(v[0])>::type;
        FH_HIP(hipMalloc((void**)p, std::max<size_t>(v.size(), 1) * sizeof(T)));
        if (!v.empty()) FH_HIP(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return RVE_OK;
    };
    auto zal = [&](double** p, int64_t n) -> int {
        FH_HIP(hipMalloc((void**)p, std::max<int64_t>(n, 1) * sizeof(double)));
        FH_HIP(hipMemset(*p, 0, std::max<int64_t>(n, 1) * sizeof(double)));
        return RVE_OK;
    };
    fehmm_s* H = h.get();
    if ((st = up(&H->d_conn, H->conn)) || (st = up(&H->d_fixed, H->fixed)) || (st = up(&H->d_col[0], H->colour[0])) ||
        (st = up(&H->d_col[1], H->colour[1])) || (st = up(&H->d_col[2], H->colour[2])) ||
        (st = up(&H->d_col[3], H->colour[3])) || (st = zal(&H->d_u, H->ndof)) || (st = zal(&H->d_du, H->ndof)) || (st = zal(&H->d_dud, H->ndof)) ||
        (st = up(&H->d_rightx, rightx)) || (st = zal(&H->d_F, 4 * (int64_t)H->nqp)) ||
        (st = zal(&H->d_P, 4 * (int64_t)H->nqp)) || (st = zal(&H->d_A, 16 * (int64_t)H->nqp)) ||
        (st = zal(&H->d_w, H->state_doubles)) || (st = zal(&H->d_ke, 64 * (int64_t)H->nelem)) ||
        (st = zal(&H->d_fe, 8 * (int64_t)H->nelem)) || (st = zal(&H->d_K, (int64_t)H->ndof * (H->bw + 1))) ||
        (st = zal(&H->d_Kt, (int64_t)H->ndof * (H->bw + 1))) ||
        (st = zal(&H->d_R, H->ndof)) || (st = zal(&H->d_norm, 2))) {
        fehmm_free(H);
        return st;
    }
    hipError_t e1 = hipMalloc((void**)&H->d_status, sizeof(int) * H->nqp);
    hipError_t e2 = hipMalloc((void**)&H->d_iters, sizeof(int) * H->nqp);
    hipError_t e3 = hipMalloc((void**)&H->d_state, sizeof(StepState));
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        fehmm_free(H);
        return set_error(RVE_ENOMEM, "fehmm_create: allocation failed");
    }
    FH_HIP(hipMemset(H->d_state, 0, sizeof(StepState)));
    *out = h.release();
    return RVE_OK;
}

int fehmm_destroy(fehmm h) {
    if (!h || !h->alive) return set_error(RVE_EINVAL, "fehmm_destroy: invalid handle");
    fehmm_free(h);
    h->alive = false;
    return RVE_OK;
}

int fehmm_sizes(fehmm h, int32_t* ndof, int32_t* nqp, int64_t* state_doubles) {
    if (!h || !h->alive) return set_error(RVE_EINVAL, "fehmm_sizes: invalid handle");
    if (ndof) *ndof = h->ndof;
    if (nqp) *nqp = h->nqp;
    if (state_doubles) *state_doubles = h->state_doubles;
    return RVE_OK;
}

}  // extern "C"

int rve_internal_solve(rve_batch b, const int32_t* subset, const int32_t* count, const double* F, double* P,
                       double* A, double* w_state, int32_t* status, int32_t* iters, const rve_opts* opts,
                       void* hip_stream, const int* skip);  // rve_abi.cpp
extern "C" int rve_internal_surrogate_eval(rve_surrogate h, const double* F, double* P, double* A, float* indicator,
                                           int64_t n, int32_t precision, void* hip_stream,
                                           const int* skip);  // surrogate.hip

// the kernels of one load step: its start, then macro Newton iterations
// it_begin .. it_end - 1 (each a no-op once the step is done)
static int enqueue_step(fehmm_s* h, int it_begin, int it_end, bool with_init) {
    const fehmm_desc& d = h->desc;
    hipStream_t s = h->stream;
    StepState* st = h->d_state;
    const int* done = &st->done;
    if (with_init) {
        hipLaunchKernelGGL(macro_step_init, dim3(nblk(h->ndof, 256)), dim3(256), 0, s, st, h->d_u, h->d_dud,
                           h->d_fixed, h->d_rightx, (d.stretch - 1.0) * d.Lx / d.nsteps, h->ndof);
        if (h->surr)  // a new load step starts with an empty fallback set
            hipLaunchKernelGGL(macro_zero_ints, dim3(nblk(h->nqp, 256)), dim3(256), 0, s, h->d_smask,
                               (int64_t)h->nqp, (const int*)nullptr);
    }
    rve_opts mo = d.micro_opts;
    const bool alt = d.scheme == FEHMM_ALTERNATING;
    if (alt) {
        mo.max_iter = 1;
        mo.flags |= RVE_FLAG_OUTPUTS_AT_CAP;
    }
    // with the surrogate the stresses carry its FP32 rounding, so the macro
    // Newton stops at surr_rtol, and only in an iteration whose indicator check
    // (at the current state) added no fallback point
    const double rtol = h->surr ? std::max(d.rtol_macro, h->surr_rtol) : d.rtol_macro;
    for (int it = it_begin; it < it_end; ++it) {
        hipLaunchKernelGGL(macro_gather_F, dim3(nblk(h->nqp, 256)), dim3(256), 0, s, h->d_conn, h->nelem, h->d_u,
                           h->geom, h->d_F, done);
        if (h->surr) {
            // surrogate answers where its indicator allows; the rest fall back to
            // the RVE solve, listed on the device (no host round trip)
            int e = rve_internal_surrogate_eval(h->surr, h->d_F, h->d_P, h->d_A, h->d_ind, h->nqp, h->surr_prec, s,
                                                done);
            if (e) return e;
            hipLaunchKernelGGL(macro_merge_fallback, dim3(nblk(h->nqp, 256)), dim3(256), 0, s, h->d_ind, h->d_smask,
                               h->surr_thr, h->nqp, &st->grew, done);
            e = rve_surrogate_select(h->d_ind, h->nqp, 0.5f, h->d_sidx, h->d_scnt, s);
            if (e) return e;
            hipLaunchKernelGGL(macro_zero_ints, dim3(nblk(h->nqp, 256)), dim3(256), 0, s, h->d_status,
                               (int64_t)h->nqp, done);
            hipLaunchKernelGGL(macro_zero_ints, dim3(nblk(h->nqp, 256)), dim3(256), 0, s, h->d_iters,
                               (int64_t)h->nqp, done);
            e = rve_internal_solve(h->batch, h->d_sidx, h->d_scnt, h->d_F, h->d_P, h->d_A, h->d_w, h->d_status,
                                   h->d_iters, &mo, s, done);
            if (e) return e;
        } else {
            int e = rve_internal_solve(h->batch, nullptr, nullptr, h->d_F, h->d_P, h->d_A, h->d_w, h->d_status,
                                       h->d_iters, &mo, s, done);
            if (e) return e;
        }
        hipLaunchKernelGGL(macro_element, dim3(nblk(8 * (int64_t)h->nelem, 256)), dim3(256), 0, s, h->nelem,
                           h->d_P, h->d_A, h->geom, h->d_ke, h->d_fe, done);
        const int64_t nK = (int64_t)h->ndof * (h->bw + 1);
        hipLaunchKernelGGL(macro_zero, dim3(nblk(nK, 256)), dim3(256), 0, s, h->d_K, nK, done);
        hipLaunchKernelGGL(macro_zero, dim3(nblk(h->ndof, 256)), dim3(256), 0, s, h->d_R, (int64_t)h->ndof, done);
        for (int c = 0; c < 4; ++c) {
            const int nel = (int)h->colour[c].size();
            if (nel == 0) continue;
            hipLaunchKernelGGL(macro_scatter, dim3(nblk(8 * (int64_t)nel, 256)), dim3(256), 0, s, h->d_col[c], nel,
                               h->d_conn, h->d_ke, h->d_fe, h->bw, h->d_K, h->d_R, done);
        }
        if (it == 0)
            hipLaunchKernelGGL(macro_dirichlet_rhs, dim3(nblk(h->ndof, 256)), dim3(256), 0, s, h->d_K, h->d_dud,
                               h->d_fixed, h->ndof, h->bw, h->d_R, done);
        hipLaunchKernelGGL(macro_bc, dim3(nblk(h->ndof, 256)), dim3(256), 0, s, h->d_fixed, h->ndof, h->bw, h->d_K,
                           h->d_R, done);
        hipLaunchKernelGGL(macro_norm_step, dim3(1), dim3(256), 0, s, h->d_R, h->ndof, h->d_status, h->d_iters,
                           h->nqp, alt ? 1 : 0, h->surr ? (const int*)h->d_scnt : (const int*)nullptr, st, it, rtol,
                           d.max_macro_iter);
        const int slots = (kPanel + h->bw + 63) / 64;  // panel rows per lane
        const size_t lds = band_lds_bytes(h->bw);
        if (band_win_fits(h->bw)) {
            hipLaunchKernelGGL(macro_band_factor_window, dim3(1), dim3(kWinNT), band_win_lds_bytes(), s, h->d_K,
                               h->d_Kt, h->ndof, h->bw, &st->band_flag, done);
            hipLaunchKernelGGL(macro_band_solves_win, dim3(1), dim3(kBandNT), band_solve_win_lds_bytes(h->bw), s,
                               h->d_K, h->d_Kt, h->d_R, h->ndof, h->bw, h->d_du, done);
        } else if (slots <= 3)
            hipLaunchKernelGGL(macro_band_solve_blocked<3>, dim3(1), dim3(kBandNT), lds, s, h->d_K, h->d_Kt, h->d_R,
                               h->ndof, h->bw, h->d_du, &st->band_flag, done);
        else if (slots == 4)
            hipLaunchKernelGGL(macro_band_solve_blocked<4>, dim3(1), dim3(kBandNT), lds, s, h->d_K, h->d_Kt, h->d_R,
                               h->ndof, h->bw, h->d_du, &st->band_flag, done);
        else
            hipLaunchKernelGGL(macro_band_solve, dim3(1), dim3(NTB), 0, s, h->d_K, h->d_R, h->ndof, h->bw, h->d_du,
                               &st->band_flag, done);
        hipLaunchKernelGGL(macro_update, dim3(nblk(h->ndof, 256)), dim3(256), 0, s, h->d_u, h->d_du, h->d_fixed,
                           it == 0 ? (const double*)h->d_dud : (const double*)nullptr, h->ndof, done);
    }
    FH_HIP(hipGetLastError());
    return RVE_OK;
}

extern "C" {

int fehmm_macro_step(fehmm h, int32_t step, fehmm_step_info* info) {
    if (!h || !h->alive) return set_error(RVE_EINVAL, "fehmm_macro_step: invalid handle");
    const fehmm_desc& d = h->desc;
    if (step < 1 || step > d.nsteps) return set_error(RVE_EINVAL, "fehmm_macro_step: step out of range");
    fehmm_step_info loc;
    fehmm_step_info* I = info ? info : &loc;
    std::memset(I, 0, sizeof(*I));
    hipStream_t s = h->stream;
    FH_HIP(hipMemcpyAsync(&h->d_state->step, &step, sizeof(int), hipMemcpyHostToDevice, s));
    StepState hs{};
    if (h->graph_on) {
        // the whole load step (all max_macro_iter + 1 iterations, no-ops after
        // convergence) as one graph, captured on first use
        if (!h->gexec) {
            FH_HIP(hipStreamSynchronize(s));
            FH_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            int e = enqueue_step(h, 0, d.max_macro_iter + 1, true);
            hipGraph_t g = nullptr;
            hipError_t ce = hipStreamEndCapture(s, &g);
            if (e) {
                if (g) (void)hipGraphDestroy(g);
                return e;
            }
            if (ce != hipSuccess) return set_error(RVE_EHIP, std::string("fehmm_macro_step capture: ") +
                                                                 hipGetErrorString(ce));
            h->graph = g;
            FH_HIP(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
        }
        FH_HIP(hipGraphLaunch(h->gexec, s));
        FH_HIP(hipMemcpyAsync(&hs, h->d_state, sizeof(hs), hipMemcpyDeviceToHost, s));
        FH_HIP(hipStreamSynchronize(s));
    } else {
        // eager: one host check of the device state per macro iteration
        for (int it = 0; it <= d.max_macro_iter; ++it) {
            int e = enqueue_step(h, it, it + 1, it == 0);
            if (e) return e;
            FH_HIP(hipMemcpyAsync(&hs, h->d_state, sizeof(hs), hipMemcpyDeviceToHost, s));
            FH_HIP(hipStreamSynchronize(s));
            if (hs.done) break;
        }
    }
    I->status = hs.status;
    I->macro_iters = hs.it;
    I->micro_iters = hs.micro;
    I->failed_rves = hs.failed;
    I->surrogate_points = hs.surrogate;
    I->fallback_points = hs.fallback;
    for (int k = 0; k <= hs.it && k < FEHMM_MAX_HIST; ++k) I->res_hist[k] = hs.hist[k];
    std::vector<double> u(h->ndof);
    FH_HIP(hipMemcpyAsync(u.data(), h->d_u, sizeof(double) * h->ndof, hipMemcpyDeviceToHost, s));
    FH_HIP(hipStreamSynchronize(s));
    double um = 0.0;
    for (int v = 0; v < h->nnode; ++v) um = std::max(um, std::hypot(u[2 * v], u[2 * v + 1]));
    I->u_max = um;
    if (hs.band_flag && I->status == FEHMM_STEP_CONVERGED) I->status = FEHMM_STEP_NOCONV;
    return I->status == FEHMM_STEP_CONVERGED ? RVE_OK : RVE_EPARTIAL;
}

static void drop_graph(fehmm_s* h) {
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
}

int fehmm_set_graph(fehmm h, int32_t enable) {
    if (!h || !h->alive) return set_error(RVE_EINVAL, "fehmm_set_graph: invalid handle");
    h->graph_on = enable != 0;
    if (!h->graph_on) drop_graph(h);
    return RVE_OK;
}

int fehmm_set_surrogate(fehmm h, rve_surrogate sg, float threshold, int32_t precision, double macro_rtol) {
    if (!h || !h->alive) return set_error(RVE_EINVAL, "fehmm_set_surrogate: invalid handle");
    drop_graph(h);  // the captured step embeds the old setting
    if (!sg) {
        h->surr = nullptr;
        return RVE_OK;
    }
    if (h->desc.scheme != FEHMM_NESTED)
        return set_error(RVE_EUNSUPPORTED, "fehmm_set_surrogate: only the nested scheme uses the surrogate");
    if (precision != RVE_SURR_BF16 && precision != RVE_SURR_BF16X3)
        return set_error(RVE_EINVAL, "fehmm_set_surrogate: unknown precision");
    if (!(threshold >= 0)) return set_error(RVE_EINVAL, "fehmm_set_surrogate: threshold must be >= 0");
    if (!(macro_rtol > 0 && macro_rtol < 1)) return set_error(RVE_EINVAL, "fehmm_set_surrogate: macro_rtol out of (0, 1)");
    if (!h->d_ind) {
        FH_HIP(hipMalloc((void**)&h->d_ind, sizeof(float) * h->nqp));
        FH_HIP(hipMalloc((void**)&h->d_sidx, sizeof(int32_t) * h->nqp));
        FH_HIP(hipMalloc((void**)&h->d_scnt, sizeof(int32_t)));
        FH_HIP(hipMalloc((void**)&h->d_smask, sizeof(int32_t) * h->nqp));
    }
    h->surr_rtol = macro_rtol;
    h->surr = sg;
    h->surr_thr = threshold;
    h->surr_prec = precision;
    return RVE_OK;
}

int fehmm_get_nodes(fehmm h, double* xy) {
    if (!h || !h->alive || !xy) return set_error(RVE_EINVAL, "fehmm_get_nodes: invalid argument");
    std::memcpy(xy, h->xy.data(), sizeof(double) * h->xy.size());
    return RVE_OK;
}

int fehmm_get_u(fehmm h, double* u) {
    if (!h || !h->alive || !u) return set_error(RVE_EINVAL, "fehmm_get_u: invalid argument");
    FH_HIP(hipMemcpy(u, h->d_u, sizeof(double) * h->ndof, hipMemcpyDeviceToHost));
    return RVE_OK;
}

int fehmm_get_qp(fehmm h, double* F, double* P, double* A) {
    if (!h || !h->alive) return set_error(RVE_EINVAL, "fehmm_get_qp: invalid handle");
    FH_HIP(hipStreamSynchronize(h->stream));
    if (F) FH_HIP(hipMemcpy(F, h->d_F, sizeof(double) * 4 * h->nqp, hipMemcpyDeviceToHost));
    if (P) FH_HIP(hipMemcpy(P, h->d_P, sizeof(double) * 4 * h->nqp, hipMemcpyDeviceToHost));
    if (A) FH_HIP(hipMemcpy(A, h->d_A, sizeof(double) * 16 * h->nqp, hipMemcpyDeviceToHost));
    return RVE_OK;
}

int fehmm_get_state(fehmm h, double* u_host, double* w_host) {
    if (!h || !h->alive || !u_host || !w_host) return set_error(RVE_EINVAL, "fehmm_get_state: invalid argument");
    FH_HIP(hipStreamSynchronize(h->stream));
    FH_HIP(hipMemcpy(u_host, h->d_u, sizeof(double) * h->ndof, hipMemcpyDeviceToHost));
    FH_HIP(hipMemcpy(w_host, h->d_w, sizeof(double) * h->state_doubles, hipMemcpyDeviceToHost));
    return RVE_OK;
}

int fehmm_set_state(fehmm h, const double* u_host, const double* w_host) {
    if (!h || !h->alive || !u_host || !w_host) return set_error(RVE_EINVAL, "fehmm_set_state: invalid argument");
    FH_HIP(hipStreamSynchronize(h->stream));
    FH_HIP(hipMemcpy(h->d_u, u_host, sizeof(double) * h->ndof, hipMemcpyHostToDevice));
    FH_HIP(hipMemcpy(h->d_w, w_host, sizeof(double) * h->state_doubles, hipMemcpyHostToDevice));
    return RVE_OK;
}

}  // extern "C"
