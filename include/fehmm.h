/*
 * fehmm.h -- C ABI of the two-scale FE-HMM driver on the GPU (Eidel, Fischer,
 * Gote, arXiv:1908.08292, Sec. 3.1-3.2 and Sec. 5).
 *
 * Macro problem: bilinear quadrilaterals on the rectangle [0,Lx] x [0,Ly]
 * (nx x ny elements, optionally without the elements whose centroid lies in a
 * centred hole of radius hole_r), 2 x 2 Gauss points, plane strain; or the
 * paper's linear triangles (P1, Sec. 3.1): every cell split along its
 * (0,0)-(1,1) diagonal, one quadrature point per triangle (qp = 2 e + t).  At every
 * macro Gauss point the displacement is linearized (eq. linearization-uH) and a
 * periodic RVE (rve.h) is driven by Fbar = I + grad u^H.  The macro residual is
 * R_H = sum_qp B_mac^T Pbar w|J|, i.e. f_I^int = int B_I^T S^H with
 * S^H = <F>^-1 <P> (eqs. f_I^int, macro-mean-stress); the macro tangent is the
 * stiffness transfer sum_qp B_mac^T Abar B_mac w|J|, equal to the FE-HMM
 * transfer sum omega/|K_delta| T^T K T of eq. (k-mac-element-6) for the unit
 * displacement states of the macro nodes.  Load steps apply the prescribed
 * right-edge displacement in nsteps equal increments; the increment of a step
 * enters its first macro Newton iteration through the linear solve (an
 * inhomogeneous Dirichlet condition: K_ff du_f = -(R_f + K_fd du_d), then the
 * fixed dofs take du_d), and the step runs the macro Newton to
 * ||R_H|| <= rtol_macro ||R_H^(0)|| with R_H^(0) = R_f + K_fd du_d, the
 * load-equivalent first residual.
 *
 * Schemes (Sec. 5): FEHMM_NESTED runs every micro Newton to convergence per
 * macro iteration, warm-started from the stored fluctuations (Algorithm 1);
 * FEHMM_ALTERNATING performs one micro Newton update per macro iteration and
 * transfers stress and stiffness at the updated micro state (Algorithm 2).
 *
 * Boundary conditions: FEHMM_BC_CLAMPED_PULL: left edge u = 0, right edge
 * u_x = (stretch - 1) Lx * step / nsteps, u_y free there.  FEHMM_BC_UNIAXIAL:
 * left edge u_x = 0, node (0,0) u_y = 0, right edge u_x prescribed, top and
 * bottom free.
 *
 * Errors follow rve.h (RVE_OK, RVE_E*).  fehmm_macro_step returns RVE_OK when
 * the step converged, RVE_EPARTIAL when some RVE failed or the macro Newton hit
 * max_macro_iter (info->status tells which).
 */
#ifndef FEHMM_FEHMM_H
#define FEHMM_FEHMM_H

#include "rve.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FEHMM_BC_CLAMPED_PULL 0
#define FEHMM_BC_UNIAXIAL 1
#define FEHMM_NESTED 0
#define FEHMM_ALTERNATING 1

#define FEHMM_STEP_CONVERGED 0
#define FEHMM_STEP_NOCONV 1     /* macro Newton reached max_macro_iter */
#define FEHMM_STEP_RVE_FAILED 2 /* some micro problem failed (status from rve.h) */

#define FEHMM_MAX_HIST 64

typedef struct fehmm_s* fehmm;

typedef struct {
    int32_t nx, ny;
    double Lx, Ly;
    double hole_r;          /* <= 0: no hole */
    int32_t bc;             /* FEHMM_BC_* */
    double stretch;         /* final right-edge stretch (1 + u_x / Lx) */
    int32_t nsteps;
    double rtol_macro;
    int32_t max_macro_iter; /* <= FEHMM_MAX_HIST - 1 */
    int32_t scheme;         /* FEHMM_NESTED or FEHMM_ALTERNATING */
    rve_mesh micro;         /* 2D RVE shared by every quadrature point (must outlive the driver) */
    rve_opts micro_opts;    /* Newton options of the micro solves */
    int32_t elem;           /* FEHMM_ELEM_Q1 (2 x 2 Gauss points) or FEHMM_ELEM_P1 (each grid cell split
                               into the triangles of its (0,0)-(1,1) diagonal, one point each) */
} fehmm_desc;

#define FEHMM_ELEM_Q1 0
#define FEHMM_ELEM_P1 1

typedef struct {
    int32_t status;                      /* FEHMM_STEP_* */
    int32_t macro_iters;                 /* macro Newton updates */
    int64_t micro_iters;                 /* micro Newton updates summed over all RVEs */
    double res_hist[FEHMM_MAX_HIST];     /* ||R_H|| / ||R_H^(0)|| per macro iteration (macro_iters + 1 entries) */
    double u_max;                        /* largest nodal |u| after the step */
    int32_t failed_rves;
    int64_t surrogate_points;            /* quadrature-point evaluations answered by the surrogate */
    int64_t fallback_points;             /* evaluations sent to the RVE solve by the indicator */
} fehmm_step_info;

/* Builds the macro mesh, uploads it, and creates the RVE batch (one RVE per
 * macro Gauss point, all of desc->micro).  Host-blocking. */
int fehmm_create(const fehmm_desc* desc, fehmm* out);
int fehmm_destroy(fehmm h);
/* Counts: macro dofs (2 per node), Gauss points, doubles of the micro state. */
int fehmm_sizes(fehmm h, int32_t* ndof, int32_t* nqp, int64_t* state_doubles);
/* One load step (1-based); host-blocking.  info may be NULL. */
int fehmm_macro_step(fehmm h, int32_t step, fehmm_step_info* info);
/* Host copies: node coordinates [nnode][2], displacements [ndof], and the
 * quadrature-point data F, P [nqp][4], A [nqp][16] of the last micro solves. */
int fehmm_get_nodes(fehmm h, double* xy);
int fehmm_get_u(fehmm h, double* u);
int fehmm_get_qp(fehmm h, double* F, double* P, double* A);
/* Replaces micro solves by a trained surrogate (surrogate.h) wherever its
 * error indicator is <= threshold; the other quadrature points fall back to
 * the RVE solve (rve_solve_batch_subset).  The fallback set of a load step
 * only grows: every macro iteration evaluates the indicator at the current
 * state and adds the points that fail it, and the step counts as converged
 * only in an iteration that added none, with ||R_H|| <= max(rtol_macro,
 * macro_rtol) ||R_H^(0)|| (the surrogate's stresses carry FP32 rounding of
 * order 1e-5 of a load increment, so rtol_macro = 1e-10 is out of reach).
 * precision: RVE_SURR_BF16 or RVE_SURR_BF16X3.  s = NULL switches the
 * surrogate off.  The surrogate must outlive its use by the driver.  Only the
 * nested scheme uses it (alternating: EUNSUPPORTED). */
int fehmm_set_surrogate(fehmm h, struct rve_surrogate_s* s, float threshold, int32_t precision, double macro_rtol);
/* enable != 0: each later fehmm_macro_step runs as one HIP graph launch -- the
 * load step's start and max_macro_iter + 1 macro iterations, with the macro
 * Newton's convergence test on the device and every kernel after convergence a
 * no-op -- captured on first use and replayed for the following steps; the
 * host waits once per step instead of once per macro iteration.  Results are
 * identical to the eager path.  Changing the surrogate drops the graph. */
int fehmm_set_graph(fehmm h, int32_t enable);
/* Checkpoint / resume: u [ndof] in host memory, the micro fluctuations
 * [state_doubles] in host memory.  set_state restores both. */
int fehmm_get_state(fehmm h, double* u_host, double* w_host);
int fehmm_set_state(fehmm h, const double* u_host, const double* w_host);

#ifdef __cplusplus
}
#endif
#endif /* FEHMM_FEHMM_H */
