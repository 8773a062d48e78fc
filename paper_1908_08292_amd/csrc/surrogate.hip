// Learned homogenized-energy surrogate W(C) of the 2D periodic RVE on gfx950.
//
// One workgroup (4 waves) evaluates a tile of 16 points.  Every neuron carries
// a jet of 10 components per point: value, the three first derivatives and the
// six second derivatives with respect to the network input x (forward-mode
// differentiation), so the first and second input derivatives of the energy
// come out of the same pass.  A tile is a 128 x 160 block (128 neurons x 10
// jet components x 16 points); the 128 x 128 layers multiply it on bf16 MFMA
// (16x16x32, FP32 accumulation) with the weights in registers and the
// activations in LDS.  The stress and tangent are assembled in FP64 from the
// derivatives (chain rule through C = F^T F) in a small per-point head.
//
// Training reuses the same forward pass on tiles of 15 data points plus the
// origin x = 0 (whose derivatives enter the Taylor-free energy), evaluates the
// loss and its derivative with respect to the 9 network outputs in the head,
// and runs the reverse pass through the jets in the same workgroup.  Each tile
// writes its parameter gradient to its own slot; a second kernel sums the
// slots and applies Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../../include/rve.h"
#include "../../include/surrogate.h"

int rve_internal_set_error(int code, const std::string& msg);  // rve_abi.cpp

namespace surr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;                // 4 waves
constexpr int WID = 128;               // hidden width
constexpr int NQ = 10;                 // jet components
constexpr int TP = 16;                 // points per tile
constexpr int NCOL = NQ * TP;          // 160 columns, column = q * 16 + p
constexpr int HSTR = WID + 8;          // LDS row stride (bf16) of a [column][neuron] buffer
constexpr int HBUF = NCOL * HSTR;      // elements of one activation buffer
constexpr int NPARAM = RVE_SURR_NPARAM;
constexpr int OFF_W1 = 0, OFF_B1 = 384, OFF_W2 = 512, OFF_B2 = 512 + 16384;
constexpr int OFF_W3 = OFF_B2 + 128, OFF_B3 = OFF_W3 + 16384, OFF_W4 = OFF_B3 + 128;
static_assert(OFF_W4 + 128 == NPARAM, "parameter layout");
constexpr int GRID = 8;                // indicator cells per input axis
constexpr double kIndicatorMargin = 2.0;  // indicator = margin x the largest calibration error nearby
constexpr int TRAIN_PTS = 15;          // data points per training tile (+ the origin)

enum { MODE_EVAL = 0, MODE_TRAIN = 1 };

// second-derivative pairs m = 0..5 of the jets and of the Hessian outputs:
// (0,0), (1,1), (2,2), (0,1), (0,2), (1,2)

struct Args {
    const float* theta;     // FP32 master parameters
    const __bf16* w_hi;     // [2][128*128] W2, W3 (bf16 nearest)
    const __bf16* w_lo;     // [2][128*128] residuals W - hi
    const __bf16* w_t;      // [2][128*128] transposed bf16 copies (reverse pass)
    double M[9], s[3], sw;  // baseline energy and input / energy scaling
    // evaluation
    const double* F;
    double* P;
    double* A;
    float* ind;
    int64_t n;
    const int* skip;        // device flag: when set, the launch does nothing
    const double* y0;       // [9] network outputs at the origin (Taylor terms)
    double* y0_out;         // when set: write the raw outputs of point 0 and stop
    const float* table;     // [GRID^3] indicator table or null
    float box_lo[3], box_hi[3];
    // training / gradient
    const double* Pt;
    const double* At;
    const int32_t* idx;     // data point of each training slot
    int64_t count;          // valid slots
    float* partial;         // [tiles][NPARAM + 1]
    float* zsave;           // [tiles][80][NT] layer-2 pre-activation jets
    float wP, wA, rhoP, rhoA;
};

// ---------------------------------------------------------------- activation

// SiLU and its first three derivatives
__device__ inline void silu4(float z, float& s0, float& s1, float& s2, float& s3) {
    const float g = 1.0f / (1.0f + __expf(-z));
    const float gp = g * (1.0f - g);
    const float gpp = gp * (1.0f - 2.0f * g);
    const float gppp = gp * (1.0f - 6.0f * g + 6.0f * g * g);
    s0 = z * g;
    s1 = g + z * gp;
    s2 = 2.0f * gp + z * gpp;
    s3 = 3.0f * gpp + z * gppp;
}

// h = silu(z) on a jet: h' = s1 z', h'' = s2 z'_a z'_b + s1 z''
__device__ inline void jet_fwd(const float z[NQ], float h[NQ]) {
    float s0, s1, s2, s3;
    silu4(z[0], s0, s1, s2, s3);
    h[0] = s0;
#pragma unroll
    for (int k = 0; k < 3; ++k) h[1 + k] = s1 * z[1 + k];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const int pa = m < 3 ? m : (m == 5 ? 1 : 0), pb = m < 3 ? m : (m == 3 ? 1 : 2);
        h[4 + m] = s2 * z[1 + pa] * z[1 + pb] + s1 * z[4 + m];
    }
}

// reverse of jet_fwd: dz from dh (all 10 components)
__device__ inline void jet_bwd(const float z[NQ], const float dh[NQ], float dz[NQ]) {
    float s0, s1, s2, s3;
    silu4(z[0], s0, s1, s2, s3);
    float d0 = s1 * dh[0];
    float dzt[3] = {s1 * dh[1], s1 * dh[2], s1 * dh[3]};
#pragma unroll
    for (int k = 0; k < 3; ++k) d0 += s2 * z[1 + k] * dh[1 + k];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const int pa = m < 3 ? m : (m == 5 ? 1 : 0), pb = m < 3 ? m : (m == 3 ? 1 : 2);
        const float g = dh[4 + m];
        d0 += (s3 * z[1 + pa] * z[1 + pb] + s2 * z[4 + m]) * g;
        dzt[pa] += s2 * z[1 + pb] * g;
        dzt[pb] += s2 * z[1 + pa] * g;
        dz[4 + m] = s1 * g;
    }
    dz[0] = d0;
#pragma unroll
    for (int k = 0; k < 3; ++k) dz[1 + k] = dzt[k];
}

// ---------------------------------------------------------------- MFMA tiles

__device__ inline f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// acc[rb][q] (rows 32w + 16rb + .., columns 16q + ..) = W[rows][:] * H[:][cols]
// with H stored [column][neuron] in LDS.  PASSES = 3 adds hi*lo + lo*hi.
template <int PASSES>
__device__ inline void gemm_rows(const __bf16* __restrict__ Whi, const __bf16* __restrict__ Wlo, const __bf16* Hhi,
                                 const __bf16* Hlo, f32x4 (&acc)[2][NQ]) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, lr = l & 15, lg = l >> 4;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[rb][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < WID / 32; ++ks) {
        bf16x8 ahi[2], alo[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int off = (32 * w + 16 * rb + lr) * WID + 32 * ks + 8 * lg;
            ahi[rb] = *reinterpret_cast<const bf16x8*>(Whi + off);
            if constexpr (PASSES == 3) alo[rb] = *reinterpret_cast<const bf16x8*>(Wlo + off);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int hoff = (16 * q + lr) * HSTR + 32 * ks + 8 * lg;
            const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(Hhi + hoff);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) acc[rb][q] = mfma(ahi[rb], bhi, acc[rb][q]);
            if constexpr (PASSES == 3) {
                const bf16x8 blo = *reinterpret_cast<const bf16x8*>(Hlo + hoff);
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    acc[rb][q] = mfma(ahi[rb], blo, acc[rb][q]);
                    acc[rb][q] = mfma(alo[rb], bhi, acc[rb][q]);
                }
            }
        }
    }
}

// dW[r][c] = sum over the 160 columns of D[col][r] * H[col][c] (both LDS
// [column][neuron]); rows r of this wave, all 128 c.  Written to out[r*128+c].
__device__ inline void gemm_weight_grad(const __bf16* D, const __bf16* H, float* __restrict__ out) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, lr = l & 15, lg = l >> 4;
    f32x4 acc[2][8];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) acc[rb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < NCOL / 32; ++ks) {
        bf16x8 a[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int j = 0; j < 8; ++j) a[rb][j] = D[(32 * ks + 8 * lg + j) * HSTR + 32 * w + 16 * rb + lr];
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) {
            bf16x8 b;
#pragma unroll
            for (int j = 0; j < 8; ++j) b[j] = H[(32 * ks + 8 * lg + j) * HSTR + 16 * cb + lr];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) acc[rb][cb] = mfma(a[rb], b, acc[rb][cb]);
        }
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 8; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                out[(32 * w + 16 * rb + 4 * lg + v) * WID + 16 * cb + lr] = acc[rb][cb][v];
}

// store the activation jets of this lane's (row, point) pairs into an LDS
// [column][neuron] buffer (hi part, and the bf16 residual when lo != null)
__device__ inline void store_act(const float (&h)[2][4][NQ], __bf16* hi, __bf16* lo) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, lr = l & 15, lg = l >> 4;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            bf16x4 vh, vl;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float x = h[rb][v][q];
                vh[v] = (__bf16)x;
                vl[v] = (__bf16)(x - (float)vh[v]);
            }
            const int off = (16 * q + lr) * HSTR + 32 * w + 16 * rb + 4 * lg;
            *reinterpret_cast<bf16x4*>(hi + off) = vh;
            if (lo) *reinterpret_cast<bf16x4*>(lo + off) = vl;
        }
}

// ---------------------------------------------------------------- FP64 head

// P [4] and A [16] from the energy derivatives with respect to c = (C11, C22,
// C12): G = dW/dc, Hc = d2W/dc2.  S11 = 2 G0, S22 = 2 G1, S12 = G2;
// CC_IJKL = f(IJ) f(KL) Hc[v(IJ)][v(KL)] with f = 2 on the diagonal, 1 off it,
// v(11) = 0, v(22) = 1, v(12) = v(21) = 2; P = F S;
// A_iJkL = delta_ik S_JL + F_iM F_kN CC_MJNL.  Linear in (G, Hc).
__device__ inline void assemble_PA(const double F[4], const double G[3], const double Hc[9], double P[4], double A[16]) {
    const double S[4] = {2.0 * G[0], G[2], G[2], 2.0 * G[1]};
    const int vI[4] = {0, 2, 2, 1};
    const double fI[4] = {2.0, 1.0, 1.0, 2.0};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int J = 0; J < 2; ++J) P[i * 2 + J] = F[i * 2 + 0] * S[0 * 2 + J] + F[i * 2 + 1] * S[1 * 2 + J];
    if (!A) return;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int J = 0; J < 2; ++J)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int L = 0; L < 2; ++L) {
                    double s = (i == k) ? S[J * 2 + L] : 0.0;
#pragma unroll
                    for (int Mi = 0; Mi < 2; ++Mi)
#pragma unroll
                        for (int Ni = 0; Ni < 2; ++Ni) {
                            const int mj = Mi * 2 + J, nl = Ni * 2 + L;
                            s += F[i * 2 + Mi] * F[k * 2 + Ni] * fI[mj] * fI[nl] * Hc[vI[mj] * 3 + vI[nl]];
                        }
                    A[(i * 2 + J) * 4 + k * 2 + L] = s;
                }
}

__device__ inline void inputs_of(const double F[4], const double s[3], double C[3], double x[3]) {
    C[0] = F[0] * F[0] + F[2] * F[2];
    C[1] = F[1] * F[1] + F[3] * F[3];
    C[2] = F[0] * F[1] + F[2] * F[3];
    x[0] = (C[0] - 1.0) / s[0];
    x[1] = (C[1] - 1.0) / s[1];
    x[2] = C[2] / s[2];
}

// energy derivatives in c from the network outputs y (3 gradient + 6 Hessian
// pairs at x) and y0 (the same at the origin)
__device__ inline void energy_derivs(const Args& a, const double C[3], const double x[3], const double y[9],
                                     const double y0[9], double G[3], double Hc[9]) {
    const double e[3] = {0.5 * (C[0] - 1.0), 0.5 * (C[1] - 1.0), C[2]};
    const double dd[3] = {0.5, 0.5, 1.0};
    double H0[9];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const int pa = m < 3 ? m : (m == 5 ? 1 : 0), pb = m < 3 ? m : (m == 3 ? 1 : 2);
        H0[pa * 3 + pb] = H0[pb * 3 + pa] = y0[3 + m];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double me = 0.0, hx = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            me += a.M[k * 3 + b] * e[b];
            hx += H0[k * 3 + b] * x[b];
        }
        G[k] = dd[k] * me + a.sw / a.s[k] * (y[k] - y0[k] - hx);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) Hc[k] = dd[k / 3] * a.M[k] * dd[k % 3];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const int pa = m < 3 ? m : (m == 5 ? 1 : 0), pb = m < 3 ? m : (m == 3 ? 1 : 2);
        const double v = a.sw / (a.s[pa] * a.s[pb]) * (y[3 + m] - y0[3 + m]);
        Hc[pa * 3 + pb] += v;
        if (pa != pb) Hc[pb * 3 + pa] += v;
    }
}

// ---------------------------------------------------------------- tile kernel

template <int MODE, int PASSES>
__global__ __launch_bounds__(NT, 1) void surr_tile_kernel(Args a) {
    extern __shared__ __align__(16) __bf16 dyn[];
    __shared__ float xs[TP][3];
    __shared__ float ypart[4][TP][9];
    __shared__ double ys[TP][9];
    __shared__ float dys[TP][9];
    __shared__ float c0s[TP][9];
    __shared__ float ls[TP];
    __shared__ int valid[TP];
    __shared__ int64_t pid[TP];

    if (MODE == MODE_EVAL && a.skip && *a.skip) return;
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, lr = l & 15, lg = l >> 4;
    const int64_t tile = blockIdx.x;
    // LDS: evaluation keeps one activation buffer (and its bf16 residual with
    // PASSES = 3) and overwrites it layer by layer; training keeps H1 and H2 for
    // the weight gradients, and a third buffer holds the residual of H1, then
    // of H2, then the reverse pass's pre-activation adjoints
    __bf16* H1 = dyn;
    __bf16* H2 = (MODE == MODE_TRAIN) ? dyn + HBUF : dyn;
    __bf16* LO = (PASSES == 3) ? (MODE == MODE_TRAIN ? dyn + 2 * HBUF : dyn + HBUF) : nullptr;
    __bf16* H1lo = LO;
    __bf16* H2lo = LO;
    __bf16* DZ = dyn + 2 * HBUF;
    const float* th = a.theta;

    // ---- inputs
    if (tid < TP) {
        const int p = tid;
        int64_t id = -1;
        bool ok = false;
        if (MODE == MODE_EVAL) {
            id = tile * TP + p;
            ok = id < a.n;
        } else if (p < TRAIN_PTS) {
            const int64_t slot = tile * TRAIN_PTS + p;
            ok = slot < a.count;
            id = ok ? (int64_t)a.idx[slot] : -1;
        }
        valid[p] = ok;
        pid[p] = id;
        double x[3] = {0.0, 0.0, 0.0};
        if (ok) {
            double F[4], C[3];
#pragma unroll
            for (int c = 0; c < 4; ++c) F[c] = a.F[id * 4 + c];
            inputs_of(F, a.s, C, x);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) xs[p][k] = (float)x[k];
    }
    __syncthreads();

    // ---- layer 1 (3 inputs): z = W1 x + b1, z' = W1 column, z'' = 0
    float h[2][4][NQ];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 32 * w + 16 * rb + 4 * lg + v;
            float z[NQ];
            const float w0 = th[OFF_W1 + 3 * r], w1 = th[OFF_W1 + 3 * r + 1], w2 = th[OFF_W1 + 3 * r + 2];
            z[0] = w0 * xs[lr][0] + w1 * xs[lr][1] + w2 * xs[lr][2] + th[OFF_B1 + r];
            z[1] = w0;
            z[2] = w1;
            z[3] = w2;
#pragma unroll
            for (int m = 0; m < 6; ++m) z[4 + m] = 0.f;
            jet_fwd(z, h[rb][v]);
        }
    store_act(h, H1, H1lo);
    __syncthreads();

    // ---- layer 2
    f32x4 acc[2][NQ];
    gemm_rows<PASSES>(a.w_hi, a.w_lo, H1, H1lo, acc);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 32 * w + 16 * rb + 4 * lg + v;
            float z[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) z[q] = acc[rb][q][v];
            z[0] += th[OFF_B2 + r];
            if (MODE == MODE_TRAIN) {
                float* zs = a.zsave + tile * (80 * NT);
#pragma unroll
                for (int q = 0; q < NQ; ++q) zs[((rb * 4 + v) * NQ + q) * NT + tid] = z[q];
            }
            jet_fwd(z, h[rb][v]);
        }
    if (MODE == MODE_EVAL || PASSES == 3) __syncthreads();  // buffers reused in place
    store_act(h, H2, H2lo);
    __syncthreads();

    // ---- layer 3 (pre-activations stay in acc for the reverse pass)
    gemm_rows<PASSES>(a.w_hi + WID * WID, a.w_lo + WID * WID, H2, H2lo, acc);
    float yp[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) yp[m] = 0.f;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 32 * w + 16 * rb + 4 * lg + v;
            acc[rb][0][v] += th[OFF_B3 + r];
            float z[NQ], hh[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) z[q] = acc[rb][q][v];
            jet_fwd(z, hh);
            const float w4 = th[OFF_W4 + r];
#pragma unroll
            for (int m = 0; m < 9; ++m) yp[m] += w4 * hh[1 + m];
        }
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        yp[m] += __shfl_xor(yp[m], 16);
        yp[m] += __shfl_xor(yp[m], 32);
    }
    if (lg == 0)
#pragma unroll
        for (int m = 0; m < 9; ++m) ypart[w][lr][m] = yp[m];
    __syncthreads();
    if (tid < TP) {
#pragma unroll
        for (int m = 0; m < 9; ++m)
            ys[tid][m] = (double)ypart[0][tid][m] + ypart[1][tid][m] + ypart[2][tid][m] + ypart[3][tid][m];
    }
    __syncthreads();

    if constexpr (MODE == MODE_EVAL) {
        if (a.y0_out) {
            if (tid < 9) a.y0_out[tid] = ys[0][tid];
            return;
        }
        if (tid < TP && valid[tid]) {
            const int p = tid;
            const int64_t id = pid[p];
            double F[4], C[3], x[3], y[9], y0[9], G[3], Hc[9], P[4], A[16];
#pragma unroll
            for (int c = 0; c < 4; ++c) F[c] = a.F[id * 4 + c];
            inputs_of(F, a.s, C, x);
#pragma unroll
            for (int m = 0; m < 9; ++m) {
                y[m] = ys[p][m];
                y0[m] = a.y0[m];
            }
            energy_derivs(a, C, x, y, y0, G, Hc);
            assemble_PA(F, G, Hc, P, a.A ? A : nullptr);
#pragma unroll
            for (int c = 0; c < 4; ++c) a.P[id * 4 + c] = P[c];
            if (a.A)
#pragma unroll
                for (int c = 0; c < 16; ++c) a.A[id * 16 + c] = A[c];
            if (a.ind) {
                float ind = INFINITY;
                if (a.table) {
                    int cell = 0;
                    bool in = true;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const double u = (x[k] - a.box_lo[k]) / ((double)a.box_hi[k] - a.box_lo[k]) * GRID;
                        const int ci = (int)floor(u);
                        in = in && (u >= 0.0) && (u <= (double)GRID);
                        cell = cell * GRID + (ci < 0 ? 0 : (ci >= GRID ? GRID - 1 : ci));
                    }
                    if (in) ind = a.table[cell];
                }
                a.ind[id] = ind;
            }
        }
        return;
    } else {
        // ---- head: loss and its derivative with respect to the 9 outputs
        if (tid < TRAIN_PTS) {
            const int p = tid;
            float dy[9], c0[9];
#pragma unroll
            for (int m = 0; m < 9; ++m) dy[m] = c0[m] = 0.f;
            float li = 0.f;
            if (valid[p]) {
                const int64_t id = pid[p];
                double F[4], C[3], x[3], y[9], y0[9], G[3], Hc[9], P[4], A[16], Pt[4], At[16];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    F[c] = a.F[id * 4 + c];
                    Pt[c] = a.Pt[id * 4 + c];
                }
#pragma unroll
                for (int c = 0; c < 16; ++c) At[c] = a.At[id * 16 + c];
                inputs_of(F, a.s, C, x);
#pragma unroll
                for (int m = 0; m < 9; ++m) {
                    y[m] = ys[p][m];
                    y0[m] = ys[TP - 1][m];
                }
                energy_derivs(a, C, x, y, y0, G, Hc);
                assemble_PA(F, G, Hc, P, A);
                double nP = (double)a.rhoP * a.rhoP, nA = (double)a.rhoA * a.rhoA, eP = 0.0, eA = 0.0;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    nP += Pt[c] * Pt[c];
                    eP += (P[c] - Pt[c]) * (P[c] - Pt[c]);
                }
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    nA += At[c] * At[c];
                    eA += (A[c] - At[c]) * (A[c] - At[c]);
                }
                const double kP = a.wP / nP, kA = a.wA / nA;
                li = (float)(kP * eP + kA * eA);
                // d loss / d y_m: (P, A) are linear in (G, Hc), which are affine in y
                double dyd[9];
#pragma unroll
                for (int m = 0; m < 9; ++m) {
                    double dG[3] = {0.0, 0.0, 0.0}, dH[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, dP[4], dA[16];
                    if (m < 3) {
                        dG[m] = a.sw / a.s[m];
                    } else {
                        const int mm = m - 3;
                        const int pa = mm < 3 ? mm : (mm == 5 ? 1 : 0), pb = mm < 3 ? mm : (mm == 3 ? 1 : 2);
                        const double v = a.sw / (a.s[pa] * a.s[pb]);
                        dH[pa * 3 + pb] = v;
                        dH[pb * 3 + pa] = v;
                    }
                    assemble_PA(F, dG, dH, dP, dA);
                    double g = 0.0;
#pragma unroll
                    for (int c = 0; c < 4; ++c) g += 2.0 * kP * (P[c] - Pt[c]) * dP[c];
#pragma unroll
                    for (int c = 0; c < 16; ++c) g += 2.0 * kA * (A[c] - At[c]) * dA[c];
                    dyd[m] = g;
                    dy[m] = (float)g;
                }
                // the origin's outputs enter with the opposite sign; its Hessian
                // also enters the gradient term through H0 x
#pragma unroll
                for (int k = 0; k < 3; ++k) c0[k] = (float)(-dyd[k]);
#pragma unroll
                for (int mm = 0; mm < 6; ++mm) {
                    const int pa = mm < 3 ? mm : (mm == 5 ? 1 : 0), pb = mm < 3 ? mm : (mm == 3 ? 1 : 2);
                    const double viaG = (pa == pb) ? dyd[pa] * x[pa] : dyd[pa] * x[pb] + dyd[pb] * x[pa];
                    c0[3 + mm] = (float)(-(dyd[3 + mm] + viaG));
                }
            }
#pragma unroll
            for (int m = 0; m < 9; ++m) {
                dys[p][m] = dy[m];
                c0s[p][m] = c0[m];
            }
            ls[p] = li;
        }
        __syncthreads();
        float* part = a.partial + tile * (int64_t)(NPARAM + 1);
        if (tid < 9) {
            float s = 0.f;
            for (int p = 0; p < TRAIN_PTS; ++p) s += c0s[p][tid];
            dys[TP - 1][tid] = s;
        }
        if (tid == 16) {
            float s = 0.f;
            for (int p = 0; p < TRAIN_PTS; ++p) s += ls[p];
            part[NPARAM] = s;
        }
        __syncthreads();

        // ---- reverse pass, layer 3 and output layer
        float dyl[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) dyl[m] = dys[lr][m];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 32 * w + 16 * rb + 4 * lg + v;
                float z[NQ], hh[NQ], dh[NQ], dz[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) z[q] = acc[rb][q][v];
                jet_fwd(z, hh);
                const float w4 = th[OFF_W4 + r];
                float gw4 = 0.f;
                dh[0] = 0.f;
#pragma unroll
                for (int m = 0; m < 9; ++m) {
                    dh[1 + m] = w4 * dyl[m];
                    gw4 += hh[1 + m] * dyl[m];
                }
                jet_bwd(z, dh, dz);
                float gb = dz[0];
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) {
                    gw4 += __shfl_xor(gw4, o);
                    gb += __shfl_xor(gb, o);
                }
                if (lr == 0) {
                    part[OFF_W4 + r] = gw4;
                    part[OFF_B3 + r] = gb;
                }
#pragma unroll
                for (int q = 0; q < NQ; ++q) h[rb][v][q] = dz[q];
            }
        store_act(h, DZ, nullptr);
        __syncthreads();
        gemm_weight_grad(DZ, H2, part + OFF_W3);
        // dH2 = W3^T dZ3: rows = layer-2 neurons of this wave, A operand from W3^T
        gemm_rows<1>(a.w_t + WID * WID, nullptr, DZ, nullptr, acc);
        __syncthreads();  // every wave is done with dZ3
        {
            const float* zs = a.zsave + tile * (80 * NT);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 32 * w + 16 * rb + 4 * lg + v;
                    float z[NQ], dh[NQ], dz[NQ];
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        z[q] = zs[((rb * 4 + v) * NQ + q) * NT + tid];
                        dh[q] = acc[rb][q][v];
                    }
                    jet_bwd(z, dh, dz);
                    float gb = dz[0];
#pragma unroll
                    for (int o = 1; o < 16; o <<= 1) gb += __shfl_xor(gb, o);
                    if (lr == 0) part[OFF_B2 + r] = gb;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) h[rb][v][q] = dz[q];
                }
        }
        store_act(h, DZ, nullptr);
        __syncthreads();
        gemm_weight_grad(DZ, H1, part + OFF_W2);
        gemm_rows<1>(a.w_t, nullptr, DZ, nullptr, acc);  // dH1 = W2^T dZ2
        // ---- layer 1: z' = W1 column is a parameter too
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 32 * w + 16 * rb + 4 * lg + v;
                float z[NQ], dh[NQ], dz[NQ];
                const float w0 = th[OFF_W1 + 3 * r], w1 = th[OFF_W1 + 3 * r + 1], w2 = th[OFF_W1 + 3 * r + 2];
                z[0] = w0 * xs[lr][0] + w1 * xs[lr][1] + w2 * xs[lr][2] + th[OFF_B1 + r];
                z[1] = w0;
                z[2] = w1;
                z[3] = w2;
#pragma unroll
                for (int m = 0; m < 6; ++m) z[4 + m] = 0.f;
#pragma unroll
                for (int q = 0; q < NQ; ++q) dh[q] = acc[rb][q][v];
                jet_bwd(z, dh, dz);
                float g[4] = {dz[0] * xs[lr][0] + dz[1], dz[0] * xs[lr][1] + dz[2], dz[0] * xs[lr][2] + dz[3], dz[0]};
#pragma unroll
                for (int o = 1; o < 16; o <<= 1)
#pragma unroll
                    for (int k = 0; k < 4; ++k) g[k] += __shfl_xor(g[k], o);
                if (lr == 0) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) part[OFF_W1 + 3 * r + k] = g[k];
                    part[OFF_B1 + r] = g[3];
                }
            }
    }
}

// first pass of the slot reduction: chunk c sums tiles c, c + nchunk, ...
// (deterministic order) into chunk_sum[c][i]
constexpr int kReduceChunks = 8;
__global__ void reduce_chunks_kernel(const float* __restrict__ partial, int64_t ntiles, float* __restrict__ chunk_sum) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i > NPARAM) return;
    float s = 0.f;
#pragma unroll 4
    for (int64_t t = c; t < ntiles; t += kReduceChunks) s += partial[t * (NPARAM + 1) + i];
    chunk_sum[(int64_t)c * (NPARAM + 1) + i] = s;
}

// sum of the chunk sums; gradient = sum * inv_n; optional Adam update
__global__ void reduce_adam_kernel(const float* __restrict__ partial, int64_t ntiles, float inv_n, float* theta, float* m,
                                   float* v, float* grad_out, float* loss_out, int do_adam, float lr, float b1, float b2,
                                   float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > NPARAM) return;
    float s = 0.f;
    for (int64_t t = 0; t < ntiles; ++t) s += partial[t * (NPARAM + 1) + i];
    if (i == NPARAM) {
        if (loss_out) *loss_out = s * inv_n;
        return;
    }
    const float g = s * inv_n;
    if (grad_out) grad_out[i] = g;
    if (do_adam) {
        const float mi = b1 * m[i] + (1.f - b1) * g;
        const float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

__global__ void adam_kernel(const float* __restrict__ g, float* theta, float* m, float* v, float lr, float b1, float b2,
                            float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    const float mi = b1 * m[i] + (1.f - b1) * g[i];
    const float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// bf16 copies of W2 and W3: nearest, residual, transposed
__global__ void refresh_bf16_kernel(const float* __restrict__ theta, __bf16* hi, __bf16* lo, __bf16* tr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * WID * WID) return;
    const int layer = i / (WID * WID), e = i % (WID * WID), r = e / WID, c = e % WID;
    const float x = theta[(layer == 0 ? OFF_W2 : OFF_W3) + e];
    const __bf16 h = (__bf16)x;
    hi[i] = h;
    lo[i] = (__bf16)(x - (float)h);
    tr[layer * WID * WID + c * WID + r] = h;
}

__global__ void fill_kernel(float* p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// indices with indicator > threshold (or NaN): one range reservation per block
__global__ void select_kernel(const float* __restrict__ ind, int64_t n, float thr, int32_t* idx, int32_t* count) {
    __shared__ int wsum[NT / 64];
    __shared__ int base;
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const float v = i < n ? ind[i] : 0.f;
    const bool take = i < n && !(v <= thr);
    const unsigned long long mask = __ballot(take);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < NT / 64; ++k) tot += wsum[k];
        base = tot ? atomicAdd(count, tot) : 0;
    }
    __syncthreads();
    int off = base;
    for (int k = 0; k < w; ++k) off += wsum[k];
    if (take) idx[off + before] = (int32_t)i;
}

__global__ void zero_int_kernel(int32_t* p) {
    if (threadIdx.x == 0) *p = 0;
}

constexpr size_t lds_bytes(int mode, int passes) {
    return (size_t)HBUF * sizeof(__bf16) * (mode == MODE_TRAIN ? 3 : (passes == 3 ? 2 : 1));
}
static_assert(lds_bytes(MODE_TRAIN, 3) + 8192 <= 160 * 1024, "training tile exceeds LDS");

}  // namespace surr

using namespace surr;

struct rve_surrogate_s {
    int dev = 0;
    float* theta = nullptr;  // device [NPARAM]
    float* m = nullptr;
    float* v = nullptr;
    __bf16* wbf = nullptr;   // [3][2][128*128]: hi, lo, transposed
    double* y0 = nullptr;    // [2][9]
    double* f_id = nullptr;  // F = I (device, 4 doubles)
    float* table = nullptr;  // [2][GRID^3]
    float box[2][6] = {};
    bool calibrated[2] = {false, false};
    double M[9] = {}, s[3] = {}, sw = 0.0;
    int64_t t = 0;           // Adam steps taken
    // training scratch
    float* partial = nullptr;
    int64_t partial_tiles = 0;
    float* zsave = nullptr;
    int32_t* idx = nullptr;
    int64_t idx_cap = 0;
    float* grad = nullptr;
    float* chunk = nullptr;  // [kReduceChunks][NPARAM + 1] first-pass sums
    float* loss = nullptr;
    int64_t loss_cap = 0;
};

namespace {

int fail(int code, const std::string& msg) { return rve_internal_set_error(code, msg); }

#define SHIP(expr)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(RVE_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool g_prepared = false;

int prepare() {
    if (g_prepared) return RVE_OK;
    SHIP(hipFuncSetAttribute((const void*)surr_tile_kernel<MODE_EVAL, 1>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes(MODE_EVAL, 1)));
    SHIP(hipFuncSetAttribute((const void*)surr_tile_kernel<MODE_EVAL, 3>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes(MODE_EVAL, 3)));
    SHIP(hipFuncSetAttribute((const void*)surr_tile_kernel<MODE_TRAIN, 1>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes(MODE_TRAIN, 1)));
    SHIP(hipFuncSetAttribute((const void*)surr_tile_kernel<MODE_TRAIN, 3>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes(MODE_TRAIN, 3)));
    g_prepared = true;
    return RVE_OK;
}

// splitmix64 (Steele, Lea, Flood 2014) for the host-side initialization and shuffles
struct SplitMix {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

Args base_args(rve_surrogate h) {
    Args a{};
    a.theta = h->theta;
    a.w_hi = h->wbf;
    a.w_lo = h->wbf + 2 * WID * WID;
    a.w_t = h->wbf + 4 * WID * WID;
    std::memcpy(a.M, h->M, sizeof(a.M));
    std::memcpy(a.s, h->s, sizeof(a.s));
    a.sw = h->sw;
    return a;
}

int launch_eval(rve_surrogate h, const Args& a, int64_t ntiles, int precision, hipStream_t st) {
    if (precision == RVE_SURR_BF16X3)
        hipLaunchKernelGGL((surr_tile_kernel<MODE_EVAL, 3>), dim3((unsigned)ntiles), dim3(NT), lds_bytes(MODE_EVAL, 3), st, a);
    else
        hipLaunchKernelGGL((surr_tile_kernel<MODE_EVAL, 1>), dim3((unsigned)ntiles), dim3(NT), lds_bytes(MODE_EVAL, 1), st, a);
    SHIP(hipGetLastError());
    return RVE_OK;
}

// bf16 weight copies and the origin outputs of both precisions
int refresh(rve_surrogate h, hipStream_t st) {
    hipLaunchKernelGGL(refresh_bf16_kernel, dim3(2 * WID * WID / NT), dim3(NT), 0, st, h->theta, h->wbf,
                       h->wbf + 2 * WID * WID, h->wbf + 4 * WID * WID);
    SHIP(hipGetLastError());
    return RVE_OK;
}

int finalize(rve_surrogate h, hipStream_t st) {
    for (int prec = 0; prec < 2; ++prec) {
        Args a = base_args(h);
        a.F = h->f_id;
        a.n = 1;
        a.y0_out = h->y0 + 9 * prec;
        int e = launch_eval(h, a, 1, prec, st);
        if (e) return e;
    }
    return RVE_OK;
}

int ensure_train_scratch(rve_surrogate h, int64_t tiles, int64_t nidx, int64_t nloss) {
    if (tiles > h->partial_tiles) {
        (void)hipFree(h->partial);
        (void)hipFree(h->zsave);
        h->partial = nullptr;
        h->zsave = nullptr;
        h->partial_tiles = 0;
        SHIP(hipMalloc((void**)&h->partial, sizeof(float) * tiles * (NPARAM + 1)));
        SHIP(hipMalloc((void**)&h->zsave, sizeof(float) * tiles * 80 * NT));
        h->partial_tiles = tiles;
    }
    if (nidx > h->idx_cap) {
        (void)hipFree(h->idx);
        h->idx = nullptr;
        h->idx_cap = 0;
        SHIP(hipMalloc((void**)&h->idx, sizeof(int32_t) * nidx));
        h->idx_cap = nidx;
    }
    if (nloss > h->loss_cap) {
        (void)hipFree(h->loss);
        h->loss = nullptr;
        h->loss_cap = 0;
        SHIP(hipMalloc((void**)&h->loss, sizeof(float) * nloss));
        h->loss_cap = nloss;
    }
    return RVE_OK;
}

// tile slots -> gradient (mean) -> optional Adam, in two deterministic passes
int reduce_slots(rve_surrogate h, int64_t tiles, float inv_n, float* grad_out, float* loss_out, int do_adam, float lr,
                 const rve_train_opts& o, float bc1, float bc2, hipStream_t st) {
    const unsigned nb = (NPARAM + 1 + NT - 1) / NT;
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3(nb, kReduceChunks), dim3(NT), 0, st, h->partial, tiles, h->chunk);
    hipLaunchKernelGGL(reduce_adam_kernel, dim3(nb), dim3(NT), 0, st, h->chunk, (int64_t)std::min<int64_t>(tiles, kReduceChunks),
                       inv_n, h->theta, h->m, h->v, grad_out, loss_out, do_adam, lr, o.beta1, o.beta2, o.eps, bc1, bc2);
    SHIP(hipGetLastError());
    return RVE_OK;
}

int check_train_opts(const rve_train_opts& o) {
    if (o.steps < 0 || o.batch < 1 || !(o.lr > 0) || !(o.lr_final > 0) || !(o.beta1 >= 0 && o.beta1 < 1) ||
        !(o.beta2 >= 0 && o.beta2 < 1) || !(o.eps > 0) || !(o.wP >= 0) || !(o.wA >= 0) || !(o.rhoP >= 0) ||
        !(o.rhoA >= 0) || (o.wP == 0 && o.wA == 0) ||
        (o.precision != RVE_SURR_BF16 && o.precision != RVE_SURR_BF16X3))
        return fail(RVE_EINVAL, "rve_train_opts out of range");
    return RVE_OK;
}

}  // namespace

extern "C" {

void rve_train_opts_default(rve_train_opts* o) {
    if (!o) return;
    o->steps = 80000;
    o->batch = 3840;
    o->lr = 2e-3f;
    o->lr_final = 2e-5f;
    o->beta1 = 0.9f;
    o->beta2 = 0.999f;
    o->eps = 1e-8f;
    o->wP = 1.0f;
    o->wA = 0.1f;
    o->rhoP = 1e-3f;
    o->rhoA = 1e-3f;
    o->seed = 1;
    o->precision = RVE_SURR_BF16X3;
}

int rve_surrogate_create(const rve_surrogate_desc* d, rve_surrogate* out) {
    if (!d || !out) return fail(RVE_EINVAL, "rve_surrogate_create: NULL argument");
    *out = nullptr;
    for (int k = 0; k < 3; ++k)
        if (!(d->c_scale[k] > 0)) return fail(RVE_EINVAL, "rve_surrogate_create: c_scale must be > 0");
    if (!(d->w_scale > 0)) return fail(RVE_EINVAL, "rve_surrogate_create: w_scale must be > 0");
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(d->A0[k])) return fail(RVE_EINVAL, "rve_surrogate_create: A0 not finite");
    int e = prepare();
    if (e) return e;
    rve_surrogate h = new rve_surrogate_s();
    (void)hipGetDevice(&h->dev);
    // M from A0: average of the entries that minor symmetry identifies, then symmetrized
    static const int pairs[3][2][2] = {{{0, 0}, {0, 0}}, {{1, 1}, {1, 1}}, {{0, 1}, {1, 0}}};
    static const int npair[3] = {1, 1, 2};
    double M[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double sum = 0.0;
            for (int u = 0; u < npair[a]; ++u)
                for (int w = 0; w < npair[b]; ++w) {
                    const int I = pairs[a][u][0], J = pairs[a][u][1], K = pairs[b][w][0], L = pairs[b][w][1];
                    sum += d->A0[(I * 2 + J) * 4 + K * 2 + L];
                }
            M[a * 3 + b] = sum / (npair[a] * npair[b]);
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) h->M[a * 3 + b] = 0.5 * (M[a * 3 + b] + M[b * 3 + a]);
    for (int k = 0; k < 3; ++k) h->s[k] = d->c_scale[k];
    h->sw = d->w_scale;
    hipError_t he = hipSuccess;
    if ((he = hipMalloc((void**)&h->theta, sizeof(float) * NPARAM)) != hipSuccess ||
        (he = hipMalloc((void**)&h->m, sizeof(float) * NPARAM)) != hipSuccess ||
        (he = hipMalloc((void**)&h->v, sizeof(float) * NPARAM)) != hipSuccess ||
        (he = hipMalloc((void**)&h->wbf, sizeof(__bf16) * 6 * WID * WID)) != hipSuccess ||
        (he = hipMalloc((void**)&h->y0, sizeof(double) * 18)) != hipSuccess ||
        (he = hipMalloc((void**)&h->f_id, sizeof(double) * 4)) != hipSuccess ||
        (he = hipMalloc((void**)&h->table, sizeof(float) * 2 * GRID * GRID * GRID)) != hipSuccess ||
        (he = hipMalloc((void**)&h->grad, sizeof(float) * NPARAM)) != hipSuccess ||
        (he = hipMalloc((void**)&h->chunk, sizeof(float) * kReduceChunks * (NPARAM + 1))) != hipSuccess) {
        rve_surrogate_destroy(h);
        return fail(RVE_ENOMEM, std::string("rve_surrogate_create: ") + hipGetErrorString(he));
    }
    static const double Fi[4] = {1.0, 0.0, 0.0, 1.0};
    if ((he = hipMemcpy(h->f_id, Fi, sizeof(Fi), hipMemcpyHostToDevice)) != hipSuccess) {
        rve_surrogate_destroy(h);
        return fail(RVE_EHIP, std::string("rve_surrogate_create: ") + hipGetErrorString(he));
    }
    // Glorot-uniform weights, zero biases
    std::vector<float> th(NPARAM, 0.f);
    SplitMix rng{d->seed};
    auto glorot = [&](int off, int fi, int fo) {
        const double lim = std::sqrt(6.0 / (fi + fo));
        for (int i = 0; i < fi * fo; ++i) th[off + i] = (float)((2.0 * rng.uniform() - 1.0) * lim);
    };
    glorot(OFF_W1, 3, WID);
    glorot(OFF_W2, WID, WID);
    glorot(OFF_W3, WID, WID);
    glorot(OFF_W4, WID, 1);
    *out = h;
    return rve_surrogate_set_params(h, th.data());
}

int rve_surrogate_destroy(rve_surrogate h) {
    if (!h) return fail(RVE_EINVAL, "rve_surrogate_destroy: NULL handle");
    (void)hipFree(h->theta);
    (void)hipFree(h->m);
    (void)hipFree(h->v);
    (void)hipFree(h->wbf);
    (void)hipFree(h->y0);
    (void)hipFree(h->f_id);
    (void)hipFree(h->table);
    (void)hipFree(h->grad);
    (void)hipFree(h->chunk);
    (void)hipFree(h->partial);
    (void)hipFree(h->zsave);
    (void)hipFree(h->idx);
    (void)hipFree(h->loss);
    delete h;
    return RVE_OK;
}

int rve_surrogate_set_params(rve_surrogate h, const float* theta_host) {
    if (!h || !theta_host) return fail(RVE_EINVAL, "rve_surrogate_set_params: NULL argument");
    for (int i = 0; i < NPARAM; ++i)
        if (!std::isfinite(theta_host[i])) return fail(RVE_EINVAL, "rve_surrogate_set_params: non-finite parameter");
    SHIP(hipMemcpy(h->theta, theta_host, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(fill_kernel, dim3((NPARAM + NT - 1) / NT), dim3(NT), 0, 0, h->m, (int64_t)NPARAM, 0.f);
    hipLaunchKernelGGL(fill_kernel, dim3((NPARAM + NT - 1) / NT), dim3(NT), 0, 0, h->v, (int64_t)NPARAM, 0.f);
    h->t = 0;
    h->calibrated[0] = h->calibrated[1] = false;
    int e = refresh(h, 0);
    if (e) return e;
    e = finalize(h, 0);
    if (e) return e;
    SHIP(hipDeviceSynchronize());
    return RVE_OK;
}

int rve_surrogate_get_params(rve_surrogate h, float* theta_host) {
    if (!h || !theta_host) return fail(RVE_EINVAL, "rve_surrogate_get_params: NULL argument");
    SHIP(hipDeviceSynchronize());
    SHIP(hipMemcpy(theta_host, h->theta, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    return RVE_OK;
}

int rve_internal_surrogate_eval(rve_surrogate h, const double* F, double* P, double* A, float* indicator, int64_t n,
                                int32_t precision, void* hip_stream, const int* skip);

int rve_surrogate_eval(rve_surrogate h, const double* F, double* P, double* A, float* indicator, int64_t n,
                       int32_t precision, void* hip_stream) {
    return rve_internal_surrogate_eval(h, F, P, A, indicator, n, precision, hip_stream, nullptr);
}

}  // extern "C"

// rve_surrogate_eval whose launch does nothing while *skip is set on the device
int rve_internal_surrogate_eval(rve_surrogate h, const double* F, double* P, double* A, float* indicator, int64_t n,
                                int32_t precision, void* hip_stream, const int* skip) {
    if (!h) return fail(RVE_EINVAL, "rve_surrogate_eval: NULL handle");
    if (n < 0 || n > (int64_t)TP * 0x7fffffff) return fail(RVE_EINVAL, "rve_surrogate_eval: bad n");
    if (n > 0 && (!F || !P)) return fail(RVE_EINVAL, "rve_surrogate_eval: F and P are required");
    if (precision != RVE_SURR_BF16 && precision != RVE_SURR_BF16X3)
        return fail(RVE_EINVAL, "rve_surrogate_eval: unknown precision");
    if (n == 0) return RVE_OK;
    Args a = base_args(h);
    a.F = F;
    a.P = P;
    a.A = A;
    a.ind = indicator;
    a.n = n;
    a.y0 = h->y0 + 9 * precision;
    a.skip = skip;
    if (h->calibrated[precision]) {
        a.table = h->table + precision * GRID * GRID * GRID;
        for (int k = 0; k < 3; ++k) {
            a.box_lo[k] = h->box[precision][k];
            a.box_hi[k] = h->box[precision][3 + k];
        }
    }
    return launch_eval(h, a, (n + TP - 1) / TP, precision, (hipStream_t)hip_stream);
}

extern "C" {

static int run_grad(rve_surrogate h, const double* F, const double* P, const double* A, const int32_t* idx,
                    int64_t count, const rve_train_opts& o, hipStream_t st) {
    const int64_t tiles = (count + TRAIN_PTS - 1) / TRAIN_PTS;
    Args a = base_args(h);
    a.F = F;
    a.Pt = P;
    a.At = A;
    a.idx = idx;
    a.count = count;
    a.partial = h->partial;
    a.zsave = h->zsave;
    a.wP = o.wP;
    a.wA = o.wA;
    a.rhoP = o.rhoP;
    a.rhoA = o.rhoA;
    if (o.precision == RVE_SURR_BF16X3)
        hipLaunchKernelGGL((surr_tile_kernel<MODE_TRAIN, 3>), dim3((unsigned)tiles), dim3(NT), lds_bytes(MODE_TRAIN, 3),
                           st, a);
    else
        hipLaunchKernelGGL((surr_tile_kernel<MODE_TRAIN, 1>), dim3((unsigned)tiles), dim3(NT), lds_bytes(MODE_TRAIN, 1),
                           st, a);
    SHIP(hipGetLastError());
    return RVE_OK;
}

int rve_surrogate_loss_grad(rve_surrogate h, const double* F, const double* P, const double* A, int64_t n,
                            const rve_train_opts* opts, float* grad_dev, double* loss_host, void* hip_stream) {
    if (!h || !F || !P || !A || !grad_dev) return fail(RVE_EINVAL, "rve_surrogate_loss_grad: NULL argument");
    if (n < 1 || n > (1ll << 30)) return fail(RVE_EINVAL, "rve_surrogate_loss_grad: bad n");
    rve_train_opts o;
    rve_train_opts_default(&o);
    if (opts) o = *opts;
    int e = check_train_opts(o);
    if (e) return e;
    const int64_t tiles = (n + TRAIN_PTS - 1) / TRAIN_PTS;
    e = ensure_train_scratch(h, tiles, n, 1);
    if (e) return e;
    std::vector<int32_t> id(n);
    for (int64_t i = 0; i < n; ++i) id[i] = (int32_t)i;
    hipStream_t st = (hipStream_t)hip_stream;
    SHIP(hipMemcpyAsync(h->idx, id.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    e = run_grad(h, F, P, A, h->idx, n, o, st);
    if (e) return e;
    e = reduce_slots(h, tiles, (float)(1.0 / n), grad_dev, h->loss, 0, 0.f, o, 1.f, 1.f, st);
    if (e) return e;
    float L = 0.f;
    SHIP(hipMemcpyAsync(&L, h->loss, sizeof(float), hipMemcpyDeviceToHost, st));
    SHIP(hipStreamSynchronize(st));
    if (loss_host) *loss_host = L;
    return RVE_OK;
}

int rve_surrogate_adam_step(rve_surrogate h, const float* grad_dev, const rve_train_opts* opts, void* hip_stream) {
    if (!h || !grad_dev) return fail(RVE_EINVAL, "rve_surrogate_adam_step: NULL argument");
    rve_train_opts o;
    rve_train_opts_default(&o);
    if (opts) o = *opts;
    int e = check_train_opts(o);
    if (e) return e;
    hipStream_t st = (hipStream_t)hip_stream;
    h->t += 1;
    const float bc1 = (float)(1.0 - std::pow((double)o.beta1, (double)h->t));
    const float bc2 = (float)(1.0 - std::pow((double)o.beta2, (double)h->t));
    hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + NT - 1) / NT), dim3(NT), 0, st, grad_dev, h->theta, h->m, h->v,
                       o.lr, o.beta1, o.beta2, o.eps, bc1, bc2);
    SHIP(hipGetLastError());
    h->calibrated[0] = h->calibrated[1] = false;
    e = refresh(h, st);
    if (e) return e;
    return finalize(h, st);
}

int rve_surrogate_train(rve_surrogate h, const double* F, const double* P, const double* A, int64_t n,
                        const rve_train_opts* opts, float* loss_host, void* hip_stream) {
    if (!h || !F || !P || !A) return fail(RVE_EINVAL, "rve_surrogate_train: NULL argument");
    if (n < 1 || n > (1ll << 30)) return fail(RVE_EINVAL, "rve_surrogate_train: bad n");
    rve_train_opts o;
    rve_train_opts_default(&o);
    if (opts) o = *opts;
    int e = check_train_opts(o);
    if (e) return e;
    if (o.steps == 0) return RVE_OK;
    const int64_t tiles = (std::min<int64_t>(o.batch, n) + TRAIN_PTS - 1) / TRAIN_PTS;
    const int64_t batch = tiles * TRAIN_PTS;
    const int64_t total = batch * (int64_t)o.steps;
    if (total > (1ll << 31)) return fail(RVE_EINVAL, "rve_surrogate_train: steps * batch too large");
    e = ensure_train_scratch(h, tiles, total, o.steps);
    if (e) return e;
    // index stream: consecutive shuffles of 0..n-1
    std::vector<int32_t> stream((size_t)total);
    {
        SplitMix rng{o.seed};
        std::vector<int32_t> perm(n);
        for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
        int64_t pos = n;
        for (int64_t k = 0; k < total; ++k) {
            if (pos == n) {
                for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[(int64_t)(rng.next() % (uint64_t)(i + 1))]);
                pos = 0;
            }
            stream[k] = perm[pos++];
        }
    }
    hipStream_t st = (hipStream_t)hip_stream;
    SHIP(hipMemcpyAsync(h->idx, stream.data(), sizeof(int32_t) * total, hipMemcpyHostToDevice, st));
    const double ratio = (double)o.lr_final / o.lr;
    for (int s = 0; s < o.steps; ++s) {
        e = run_grad(h, F, P, A, h->idx + (int64_t)s * batch, batch, o, st);
        if (e) return e;
        h->t += 1;
        const double lr = o.lr * std::pow(ratio, o.steps > 1 ? (double)s / (o.steps - 1) : 0.0);
        const float bc1 = (float)(1.0 - std::pow((double)o.beta1, (double)h->t));
        const float bc2 = (float)(1.0 - std::pow((double)o.beta2, (double)h->t));
        e = reduce_slots(h, tiles, (float)(1.0 / batch), nullptr, h->loss + s, 1, (float)lr, o, bc1, bc2, st);
        if (e) return e;
        e = refresh(h, st);
        if (e) return e;
    }
    e = finalize(h, st);
    if (e) return e;
    h->calibrated[0] = h->calibrated[1] = false;
    if (loss_host) SHIP(hipMemcpyAsync(loss_host, h->loss, sizeof(float) * o.steps, hipMemcpyDeviceToHost, st));
    SHIP(hipStreamSynchronize(st));
    return RVE_OK;
}

int rve_surrogate_calibrate(rve_surrogate h, const double* F, const double* P, int64_t n, int32_t precision,
                            void* hip_stream) {
    if (!h || !F || !P) return fail(RVE_EINVAL, "rve_surrogate_calibrate: NULL argument");
    if (n < 1 || n > (1ll << 30)) return fail(RVE_EINVAL, "rve_surrogate_calibrate: bad n");
    if (precision != RVE_SURR_BF16 && precision != RVE_SURR_BF16X3)
        return fail(RVE_EINVAL, "rve_surrogate_calibrate: unknown precision");
    hipStream_t st = (hipStream_t)hip_stream;
    double* Ps = nullptr;
    SHIP(hipMalloc((void**)&Ps, sizeof(double) * 4 * n));
    h->calibrated[precision] = false;
    int e = rve_surrogate_eval(h, F, Ps, nullptr, nullptr, n, precision, hip_stream);
    std::vector<double> hF(4 * n), hP(4 * n), hS(4 * n);
    if (!e) {
        hipError_t he;
        if ((he = hipMemcpyAsync(hF.data(), F, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (he = hipMemcpyAsync(hP.data(), P, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (he = hipMemcpyAsync(hS.data(), Ps, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (he = hipStreamSynchronize(st)) != hipSuccess)
            e = fail(RVE_EHIP, std::string("rve_surrogate_calibrate: ") + hipGetErrorString(he));
    }
    (void)hipFree(Ps);
    if (e) return e;
    // host bookkeeping: box of x, per-cell maximum relative error
    std::vector<double> X(3 * n);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < n; ++i) {
        const double* f = &hF[4 * i];
        const double C[3] = {f[0] * f[0] + f[2] * f[2], f[1] * f[1] + f[3] * f[3], f[0] * f[1] + f[2] * f[3]};
        const double x[3] = {(C[0] - 1.0) / h->s[0], (C[1] - 1.0) / h->s[1], C[2] / h->s[2]};
        for (int k = 0; k < 3; ++k) {
            X[3 * i + k] = x[k];
            lo[k] = std::min(lo[k], x[k]);
            hi[k] = std::max(hi[k], x[k]);
        }
    }
    for (int k = 0; k < 3; ++k)
        if (!(hi[k] > lo[k])) return fail(RVE_EINVAL, "rve_surrogate_calibrate: degenerate input range");
    const int NC = GRID * GRID * GRID;
    std::vector<double> cmax(NC, 0.0);
    std::vector<int> cnt(NC, 0);
    for (int64_t i = 0; i < n; ++i) {
        int cell = 0;
        for (int k = 0; k < 3; ++k) {
            int ci = (int)std::floor((X[3 * i + k] - lo[k]) / (hi[k] - lo[k]) * GRID);
            ci = std::min(std::max(ci, 0), GRID - 1);
            cell = cell * GRID + ci;
        }
        double num = 0.0, den = 0.0;
        for (int c = 0; c < 4; ++c) {
            num += (hS[4 * i + c] - hP[4 * i + c]) * (hS[4 * i + c] - hP[4 * i + c]);
            den += hP[4 * i + c] * hP[4 * i + c];
        }
        const double err = std::sqrt(num) / std::max(std::sqrt(den), 1e-300);
        cmax[cell] = std::max(cmax[cell], std::isfinite(err) ? err : 1e300);
        cnt[cell] += 1;
    }
    std::vector<float> tab(NC);
    for (int c0 = 0; c0 < GRID; ++c0)
        for (int c1 = 0; c1 < GRID; ++c1)
            for (int c2 = 0; c2 < GRID; ++c2) {
                const int cell = (c0 * GRID + c1) * GRID + c2;
                double m = cnt[cell] >= 2 ? 0.0 : INFINITY;
                for (int d0 = -1; d0 <= 1; ++d0)
                    for (int d1 = -1; d1 <= 1; ++d1)
                        for (int d2 = -1; d2 <= 1; ++d2) {
                            const int e0 = c0 + d0, e1 = c1 + d1, e2 = c2 + d2;
                            if (e0 < 0 || e1 < 0 || e2 < 0 || e0 >= GRID || e1 >= GRID || e2 >= GRID) continue;
                            m = std::max(m, cmax[(e0 * GRID + e1) * GRID + e2]);
                        }
                // margin for points worse than any calibration point nearby
                tab[cell] = (float)(kIndicatorMargin * m);
            }
    SHIP(hipMemcpy(h->table + precision * NC, tab.data(), sizeof(float) * NC, hipMemcpyHostToDevice));
    for (int k = 0; k < 3; ++k) {
        h->box[precision][k] = (float)lo[k];
        h->box[precision][3 + k] = (float)hi[k];
    }
    h->calibrated[precision] = true;
    return RVE_OK;
}

int rve_surrogate_select(const float* indicator, int64_t n, float threshold, int32_t* idx, int32_t* count,
                         void* hip_stream) {
    if (!count || (n > 0 && (!indicator || !idx))) return fail(RVE_EINVAL, "rve_surrogate_select: NULL argument");
    if (n < 0 || n > 0x7fffffff) return fail(RVE_EINVAL, "rve_surrogate_select: bad n");
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, st, count);
    if (n > 0)
        hipLaunchKernelGGL(select_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, indicator, n, threshold,
                           idx, count);
    SHIP(hipGetLastError());
    return RVE_OK;
}

}  // extern "C"
