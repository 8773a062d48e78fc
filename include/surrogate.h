/* Learned homogenized-energy surrogate of the 2D periodic RVE (C ABI).
 *
 * The homogenized response of the micro problem is hyperelastic: the macro
 * stress P-bar is the derivative of the volume-averaged strain energy with
 * respect to F-bar and the macro tangent A-bar its second derivative (the
 * Hill-Mandel condition of the two-scale formulation, paper Sec. 2.3).
 * Frame invariance makes that energy a function of C = F^T F, so the surrogate
 * is an energy
 *
 *   W(C) = W0(C) + s_W * [ N(x) - N(0) - grad N(0).x - 1/2 x^T hess N(0) x ]
 *
 * with W0 = 1/2 e^T M e, e = (E11, E22, 2 E12), E = (C - I)/2, M read off the
 * homogenized small-strain tangent A0 (so the surrogate reproduces P(I) = 0
 * and A(I) = A0 exactly), x = ((C11-1)/s0, (C22-1)/s1, C12/s2) and N an MLP
 * 3 -> 128 -> 128 -> 128 -> 1 with SiLU activations.  P = 2 F dW/dC and A are
 * assembled in FP64 from the network's first and second input derivatives,
 * which the kernels carry forward through the layers as jets (value, three
 * tangents, six second derivatives per neuron); the 128 x 128 layers run on
 * bf16 MFMA with FP32 accumulation.  Training (Adam on the loss below) runs in
 * the library's own forward / backward kernels on triples (F, P, A) produced
 * by rve_solve_batch.  An error indicator per evaluation (calibrated against
 * RVE solves) decides where the surrogate may replace the RVE solve.
 *
 * Parameter vector (float, RVE_SURR_NPARAM entries): W1[128][3], b1[128],
 * W2[128][128], b2[128], W3[128][128], b3[128], w4[128] (W[out][in]).
 *
 * Training loss over n points:
 *   L = 1/n sum_i [ wP |P_i - P*_i|^2 / (|P*_i|^2 + rhoP^2)
 *                 + wA |A_i - A*_i|^2 / (|A*_i|^2 + rhoA^2) ]
 *
 * Layouts as in rve.h: F, P [n][4] row-major [i][J]; A [n][16] with
 * A[(i*2+J)*4 + (k*2+L)] = dP_iJ/dF_kL.  All array arguments named *_dev or
 * documented as device pointers are device memory owned by the caller.
 * Return codes are the RVE_* codes of rve.h.  Calls on one handle are not
 * thread-safe.
 */
#ifndef RVE_SURROGATE_H
#define RVE_SURROGATE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RVE_SURR_NPARAM 33664
#define RVE_SURR_BF16 0   /* one bf16 MFMA product per layer */
#define RVE_SURR_BF16X3 1 /* split bf16 operands (hi*hi + hi*lo + lo*hi): near-FP32 products */

typedef struct rve_surrogate_s* rve_surrogate;

typedef struct {
    double A0[16];      /* homogenized tangent at F = I (e.g. rve_solve_batch at F = I) */
    double c_scale[3];  /* input scaling s0, s1, s2 (> 0) */
    double w_scale;     /* energy scale s_W of the network part (> 0) */
    uint64_t seed;      /* weight initialization (Glorot uniform, zero biases) */
} rve_surrogate_desc;

typedef struct {
    int32_t steps;          /* Adam steps */
    int32_t batch;          /* points per step (rounded up to whole tiles of 15) */
    float lr, lr_final;     /* learning rate, decayed geometrically to lr_final */
    float beta1, beta2, eps;
    float wP, wA, rhoP, rhoA;
    uint64_t seed;          /* mini-batch sampling (epoch-wise shuffles) */
    int32_t precision;      /* forward products of training: RVE_SURR_BF16 or RVE_SURR_BF16X3;
                               the reverse pass multiplies plain bf16 operands */
} rve_train_opts;

/* Fills defaults: steps 80000, batch 3840, lr 2e-3 -> 2e-5, Adam (0.9, 0.999,
 * 1e-8), wP 1, wA 0.1, rhoP 1e-3, rhoA 1e-3, seed 1, precision BF16X3. */
void rve_train_opts_default(rve_train_opts* o);

/* Creates a surrogate on the current device.  EINVAL for non-positive scales. */
int rve_surrogate_create(const rve_surrogate_desc* desc, rve_surrogate* out);
int rve_surrogate_destroy(rve_surrogate h);

/* Host float [RVE_SURR_NPARAM] in / out.  set_params resets the Adam state and
 * the indicator calibration. */
int rve_surrogate_set_params(rve_surrogate h, const float* theta_host);
int rve_surrogate_get_params(rve_surrogate h, float* theta_host);

/* Evaluates P [n][4] and A [n][16] (A may be NULL) and the error indicator
 * [n] (may be NULL; +inf where the surrogate is not calibrated or x lies
 * outside the calibrated region) at the given precision.  Device pointers;
 * asynchronous on the stream. */
int rve_surrogate_eval(rve_surrogate h, const double* F, double* P, double* A, float* indicator, int64_t n,
                       int32_t precision, void* hip_stream);

/* Mean loss over the n points and its gradient (device float [RVE_SURR_NPARAM])
 * at the current parameters, with the loss weights of opts (NULL: defaults).
 * Host-blocking; loss_host may be NULL. */
int rve_surrogate_loss_grad(rve_surrogate h, const double* F, const double* P, const double* A, int64_t n,
                            const rve_train_opts* opts, float* grad_dev, double* loss_host, void* hip_stream);

/* One Adam update with the given gradient (device float [RVE_SURR_NPARAM]),
 * learning rate opts->lr and step count advanced by one. */
int rve_surrogate_adam_step(rve_surrogate h, const float* grad_dev, const rve_train_opts* opts, void* hip_stream);

/* Trains on n device-resident triples; host-blocking.  loss_host [steps] (may
 * be NULL) receives the mini-batch loss of every step.  Resets calibration. */
int rve_surrogate_train(rve_surrogate h, const double* F, const double* P, const double* A, int64_t n,
                        const rve_train_opts* opts, float* loss_host, void* hip_stream);

/* Calibrates the indicator at one precision from n judged points (P from
 * rve_solve_batch): relative stress error |P_s - P|_F / |P|_F on a grid of
 * 8^3 cells over the bounding box of the points' x, each cell reporting 2
 * times the largest error found in it and its 26 neighbours (+inf with fewer
 * than 2 points in the cell).  Host-blocking. */
int rve_surrogate_calibrate(rve_surrogate h, const double* F, const double* P, int64_t n, int32_t precision,
                            void* hip_stream);

/* Compacts the indices r with indicator[r] > threshold (or NaN) into idx [n]
 * (device) and their count into count (device int32); order within the list
 * is unspecified.  Asynchronous. */
int rve_surrogate_select(const float* indicator, int64_t n, float threshold, int32_t* idx, int32_t* count,
                         void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
