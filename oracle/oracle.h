/*
 * oracle.h -- plain, slow FP64 CPU reference for the periodic-RVE hot path of
 * the nonlinear FE-HMM (Eidel, Fischer, Gote, arXiv:1908.08292).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only tests/, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source with the HIP path.
 *
 * Formulation (all in the paper's total-Lagrangian S/E setting):
 *   - constitutive law: compressible neo-Hookean, eq. (NH-free-energy) and the
 *     S / C_ijkl / A_ijkl relations that follow it (Sec. 6); 2D is plane strain;
 *   - micro element residual f_I = int B_I^T S dV (eq. f_I^int) and tangent
 *     k_IK = int (B_I^T C B_K + S_hat_IK 1) dV (eqs. DG^h, G_IK, S_IK);
 *   - periodic coupling (Sec. 3.2, eq. ConstraintCondition) realised by
 *     identifying partner nodes; one node pinned against rigid translation;
 *   - micro Newton on K_T dD = -R (eq. Saddlepoint-problem with G^T dLambda = 0
 *     for PBC), sparse LDL^T of the free block with an RCM profile ordering;
 *   - outputs: P = <P^eps> (eq. Average-of-P-and-F) and the stiffness carried by
 *     the unit macro-gradient states, T^T K T / |K_delta| (eqs. k-mac-element-5..7),
 *     evaluated at the converged tangent (end of Sec. 3.3).
 *
 * Layouts: node (i,j[,k]) of the n^d periodic grid has id i + n j [+ n^2 k];
 * element (i,j[,k]) has the same id and nodes (i+{0,1}, j+{0,1}[, k+{0,1}]) mod n
 * in counter-clockwise (2D) / hex (3D) order.  Fluctuations w are node-major
 * [node][d].  F and P are row-major d x d ([i][J]); A is the d^2 x d^2 row-major
 * matrix A[(i*d+J)*d*d + (k*d+L)] = dP_iJ / dF_kL.
 */
#ifndef FEHMM_ORACLE_H
#define FEHMM_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_NOCONV = 1, ORC_DETF = 2, ORC_SINGULAR = 3, ORC_NONFINITE = 4 };

/* Neo-Hookean point update in the paper's S/C form (Sec. 6).  d = 2 (plane strain)
 * or 3.  Outputs: S (d x d), Cmat (d^4, Cmat[((I*d+J)*d+K)*d+L]), psi. Returns 0,
 * or ORC_DETF when det F <= 0. */
int oracle_nh_sc(int d, double lam, double mu, const double* F, double* S, double* Cmat, double* psi);

/* Micro constitutive law used by every later call (process-wide; default the
 * neo-Hookean law).  ORC_LAW_SVK: geometrically nonlinear linear elasticity
 * (St. Venant-Kirchhoff, S = lambda tr(E) 1 + 2 mu E); ORC_LAW_LINEAR: the
 * fully linear case (small strain, sigma = lambda tr(eps) 1 + 2 mu eps, which
 * stands for both S and P; no geometric stiffness) -- the laws of the paper's
 * micro-convergence comparisons (Sec. 6). */
enum { ORC_LAW_NEOHOOKE = 0, ORC_LAW_SVK = 1, ORC_LAW_LINEAR = 2 };
void oracle_set_law(int law);
int oracle_get_law(void);
/* S (or sigma), the material tangent (d^4) and psi of law at F; as oracle_nh_sc. */
int oracle_law_sc(int law, int d, double lam, double mu, const double* F, double* S, double* Cmat, double* psi);

/* Micro boundary conditions of every later call (process-wide; default
 * periodic).  ORC_BC_PERIODIC: periodic fluctuation, node 0 pinned.
 * ORC_BC_LINEAR: linear displacements u = Fbar X on the RVE boundary (KUBC, the
 * coupling of the paper's 3D example): the fluctuation vanishes on every
 * boundary node -- on the n^d numbering, every node with some grid index 0. */
enum { ORC_BC_PERIODIC = 0, ORC_BC_LINEAR = 1 };
void oracle_set_bc(int bc);
int oracle_get_bc(void);

/* Micro element kind of every later call (process-wide; default Q1).
 * ORC_ELEM_P1: the paper's linear simplices -- each grid cell split into d!
 * simplices along its (0..0)-(1..1) diagonal (Kuhn), one integration point each
 * (the gradient is constant); the cell's phase, node numbering and unknowns are
 * unchanged. */
enum { ORC_ELEM_Q1 = 0, ORC_ELEM_P1 = 1 };
void oracle_set_element(int kind);
int oracle_get_element(void);

/* Phase of every element by centroid: phase = incl_phase iff |centroid - c| < r. */
void oracle_phase_by_centroid(int d, int n, const double* center, double r, int incl_phase,
                              int base_phase, uint8_t* phase);

/* Element routines for element e of the periodic mesh at fluctuation w.
 * fe: [2^d][d]; ke: [2^d*d][2^d*d] row-major; energy: sum_gp psi w|J|.
 * Returns 0 or ORC_DETF if some Gauss point has J <= 0. */
int oracle_element(int d, int n, const uint8_t* phase, const double* lame, int e,
                   const double* Fbar, const double* w, double* fe, double* ke, double* energy);

/* Total residual (all d*n^d entries, pinned node included) and energy. */
int oracle_residual(int d, int n, const uint8_t* phase, const double* lame,
                    const double* Fbar, const double* w, double* R, double* energy);

typedef struct {
    double rtol;        /* relative Newton tolerance on ||R_f||_2 */
    double atol;        /* absolute floor */
    int max_iter;       /* Newton iterations (factorizations before convergence) */
    int max_backtrack;  /* halvings of the step while some J <= 0 */
    int want_A;         /* 1: compute the stiffness transfer */
} oracle_opts;

/* One RVE solve.  w: in/out node-major fluctuation (d*n^d), may be NULL (zero
 * start, no store).  res_hist (may be NULL) receives ||R_f|| for iterations
 * 0..iters.  Returns the status code. */
int oracle_rve_solve(int d, int n, const uint8_t* phase, const double* lame,
                     const double* Fbar, double* w, const oracle_opts* o,
                     double* P, double* A, int* iters, double* res_hist);

/* Batch of B RVEs of one mesh size; phases [B][n^d]; F [B][d*d]; w [B][d*n^d]
 * (may be NULL).  OpenMP over RVEs with nthreads (<=0: runtime default). */
int oracle_rve_solve_batch(int d, int n, int64_t B, const uint8_t* phases, const double* lame,
                           const double* F, double* w, const oracle_opts* o,
                           double* P, double* A, int32_t* status, int32_t* iters, int nthreads);

/* Small-strain linear elasticity (lambda 1x1 + 2 mu I) homogenized tensor
 * C^{0,h} of the same periodic mesh, from the d(d+1)/2 unit-strain cell
 * problems (linear FE-HMM, Sec. 4 eq. Estimate-ElasticityTensor).  Output as a
 * d^2 x d^2 matrix in the same [(iJ)][(kL)] layout. */
int oracle_linear_homogenized(int d, int n, const uint8_t* phase, const double* lame, double* Chom);

/* Test hook: free residual, dense free-free tangent (natural node-major order,
 * pinned nodes excluded) and the skyline-LDL^T Newton step dw = -K_ff^-1 R_f. */
int oracle_debug_system(int d, int n, const uint8_t* phase, const double* lame, const double* Fbar, const double* w,
                        double* Rf, double* Kff, double* dw);

/* ---- macro level (Sec. 3.1-3.2, Algorithms 1/2 of Sec. 5) -------------------- */
typedef struct {
    int nx, ny;            /* Q1 macro elements */
    double Lx, Ly;         /* plate size */
    double hole_r;         /* centred hole radius (elements removed by centroid); <= 0: none */
    int bc;                /* 0: left clamped, right u_x prescribed; 1: uniaxial (left u_x=0, node (0,0) u_y=0, right u_x) */
    double stretch;        /* final right-edge u_x = (stretch-1) * Lx */
    int nsteps;
    double rtol_macro;
    int scheme;            /* 0 nested (Algorithm 1), 1 alternating (Algorithm 2) */
    int max_macro_iter;
    /* micro */
    int n;                 /* RVE elements per edge (2D only) */
    const uint8_t* phase;  /* n^2 phases shared by every RVE */
    const double* lame;    /* [nphase][2] */
    int elem;              /* macro elements: 0 Q1 with 2x2 Gauss points; 1 P1 triangles (each grid cell split
                              along its (0,0)-(1,1) diagonal, one point per triangle) */
} oracle_macro_desc;

typedef struct oracle_macro oracle_macro;
oracle_macro* oracle_macro_create(const oracle_macro_desc* d, const oracle_opts* micro);
void oracle_macro_destroy(oracle_macro* m);
int oracle_macro_ndof(const oracle_macro* m);
int oracle_macro_nqp(const oracle_macro* m);
/* One load step (1-based; load factor step/nsteps).  The increment of the
 * prescribed displacements enters the first macro Newton iteration through the
 * linear solve (K_ff du_f = -(R_f + K_fd du_d), then u_d += du_d), so the first
 * residual of the step is the load-equivalent R_f + K_fd du_d.  Fills the macro
 * iteration count, the residual history normalized to that first residual
 * (max_macro_iter+1 entries) and the total micro iterations.  Returns 0, 1 if
 * the macro Newton did not converge, or 2 if some RVE failed. */
int oracle_macro_step(oracle_macro* m, int step, int* macro_iters, double* res_hist, int64_t* micro_iters);
void oracle_macro_get_u(const oracle_macro* m, double* u);
void oracle_macro_get_qp(const oracle_macro* m, double* F, double* P, double* A);
void oracle_macro_get_nodes(const oracle_macro* m, double* xy);
int oracle_macro_nelem(const oracle_macro* m);
void oracle_macro_get_conn(const oracle_macro* m, int* conn);
/* micro states [nqp][2 n^2] of the last solves; set_qp overwrites the stored
 * Fbar, Pbar, Abar and micro states (each may be NULL) */
void oracle_macro_get_state(const oracle_macro* m, double* w);
void oracle_macro_set_qp(oracle_macro* m, const double* F, const double* P, const double* A, const double* w);
/* Macro element stiffness [8][8] of element e at the stored micro states:
 * literal = 1, the FE-HMM transfer of eqs. (k-mac-element-5..7) -- the unit
 * nodal displacement states (I, x_i) of the element, linearized at each Gauss
 * point, drive the micro problem and k = sum omega T^T K T / |K_delta|;
 * literal = 0, sum omega B^T Abar B with the stored tangents Abar. */
int oracle_macro_element_stiffness(const oracle_macro* m, int e, int literal, double* k);

/* The micro responses to nstate prescribed linearized displacement states
 * (gradient G [nstate][d*d], translation tvec [nstate][d] or NULL) at the micro
 * state (Fbar, w), and T^T K T / |K_delta| [nstate][nstate] with the tangent
 * there (eq. Lagrange-Functional-for-StiffnessTransfer, eqs. k-mac-element-5..7). */
int oracle_rve_transfer_states(int d, int n, const uint8_t* phase, const double* lame, const double* Fbar,
                               const double* w, int nstate, const double* G, const double* tvec, double* kT);

#ifdef __cplusplus
}
#endif
#endif
