/*
 * rve.h -- C ABI of the MI355X (gfx950) batched periodic-RVE solver of the
 * nonlinear FE-HMM (Eidel, Fischer, Gote, arXiv:1908.08292).
 *
 * Problem solved per RVE (micro problem of Sec. 3.3 under periodic coupling,
 * Sec. 3.2 eq. ConstraintCondition): on the unit cell [0,1]^d meshed by n^d
 * bilinear quadrilaterals (d = 2, plane strain) or trilinear hexahedra (d = 3)
 * with 2^d Gauss points each, find the periodic fluctuation w (one node pinned
 * against rigid translation) such that the first-order coupled deformation
 * F = Fbar + grad w (eq. linearization-uH) is in equilibrium,
 *     R(w) = sum_e int P(F) . grad N dV = 0,
 * with the compressible neo-Hookean law of Sec. 6 (eq. NH-free-energy).  The
 * outputs are the volume average Pbar = <P> (eq. Average-of-P-and-F) and the
 * consistent tangent Abar = dPbar/dFbar at the converged state, i.e. the
 * micro-to-macro stiffness transfer T^T K T / |K_delta| of eqs.
 * (k-mac-element-5..7) written for the d^2 unit macro-gradient states.
 *
 * Conventions.
 *   - Node (i,j[,k]) of the periodic grid has id i + n j [+ n^2 k]; element
 *     (i,j[,k]) has the same id and its centroid at ((i+1/2)/n, ...).
 *   - F and P are row-major d x d: F[i*d + J] = F_iJ (i spatial, J material).
 *   - A is the d^2 x d^2 row-major matrix A[(i*d+J)*d*d + (k*d+L)] = dP_iJ/dF_kL.
 *   - Fluctuations are node-major: w[node*d + i]; node 0 is pinned (w = 0).
 *
 * Errors.  Every call returns an int: RVE_OK (0), a negative RVE_E* code for
 * API/usage/device failures (nothing was computed; rve_last_error() explains),
 * or RVE_EPARTIAL (1) from rve_solve_batch when some RVEs failed.  Per-RVE
 * codes (RVE_S_*) go to the status array; failed RVEs get NaN P and A and their
 * w_state is left unchanged, the rest of the batch is unaffected.
 *
 * Ownership.  The library owns meshes, batches and their device workspaces
 * (freed by the *_destroy calls).  The caller owns every input/output buffer.
 * Calls on one handle are not thread-safe.
 */
#ifndef FEHMM_RVE_H
#define FEHMM_RVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------------- */
#define RVE_OK 0
#define RVE_EPARTIAL 1        /* some RVEs of the batch failed (see status[]) */
#define RVE_EINVAL (-1)       /* bad argument (NULL, size, range, destroyed handle) */
#define RVE_ENOMEM (-2)       /* host or device allocation failed */
#define RVE_EHIP (-3)         /* a HIP runtime call failed */
#define RVE_EUNSUPPORTED (-4) /* valid request this library does not support */

/* ---- per-RVE status -------------------------------------------------------- */
#define RVE_S_CONVERGED 0
#define RVE_S_NOCONV 1    /* Newton did not reach the tolerance in max_iter updates */
#define RVE_S_DETF 2      /* det F <= 0 at a Gauss point survived all step halvings */
#define RVE_S_SINGULAR 3  /* a pivot of the LDL^T factorization vanished */
#define RVE_S_NONFINITE 4 /* non-finite input or residual */

typedef struct rve_mesh_s* rve_mesh;
typedef struct rve_batch_s* rve_batch;

/* Lame parameters from Young's modulus and Poisson's ratio (the 3D relations,
 * also used for plane strain; the paper's material table, Sec. 6). */
int rve_lame(double E, double nu, double* lambda_out, double* mu_out);

/* ---- meshes ------------------------------------------------------------------
 * rve_mesh_create: one periodic RVE discretisation (Sec. 3.1 micro triangulation,
 * here a structured grid) with its phase field and material table.
 *   ndim       2 or 3
 *   n          elements per edge, 2 <= n <= 64 (2D) or 2 <= n <= 24 (3D)
 *   nphase     1..255; lame: host array [nphase][2] = (lambda, mu), mu > 0
 *   phase      host array [n^d] of phase ids (x-fastest), or NULL: then an
 *              element is in incl_phase iff |centroid - incl_center| < incl_radius
 *              (strict), else in phase 0.  The data are copied.
 *   law        micro constitutive law (RVE_LAW_*): the compressible neo-Hookean
 *              law of Sec. 6 (default, 0), or the two laws the paper sets beside
 *              it in its micro-convergence studies: geometrically nonlinear
 *              linear elasticity (St. Venant-Kirchhoff, S = lambda tr(E) 1 +
 *              2 mu E, E the Green-Lagrange strain) and the fully linear case
 *              (small strain, sigma = lambda tr(eps) 1 + 2 mu eps takes the place
 *              of P; A is the constant elasticity tensor).  The J > 0 guard of the
 *              Newton update applies to every law.
 *   bc         micro boundary conditions (RVE_BC_*; Sec. 3.2, the energetically
 *              consistent couplings): periodic fluctuations (default, 0; node 0
 *              pinned against translation), or linear displacements u = Fbar X
 *              on the cell boundary (KUBC, the coupling of the paper's 3D
 *              example): the fluctuation vanishes on every boundary node, so
 *              only the (n-1)^d interior nodes are free.  Fluctuations keep the
 *              n^d node layout either way (boundary nodes -- every node with
 *              some grid index 0 -- hold 0).
 *   elem       micro element kind (RVE_ELEM_*): bilinear quadrilaterals /
 *              trilinear hexahedra with 2^d Gauss points (default, 0), or the
 *              paper's linear simplices P1 (Sec. 3.1): every grid cell split into
 *              d! simplices along its (0..0)-(1..1) diagonal (a conforming Kuhn
 *              triangulation), one integration point each, the cell's phase.
 *              Nodes and unknowns are the same for both kinds.
 * The symbolic factorization plan for (ndim, n) is built on first use and shared
 * by every mesh of that size. */
typedef struct {
    int32_t ndim;
    int32_t n;
    int32_t nphase;
    const double* lame;
    const uint8_t* phase;
    double incl_center[3];
    double incl_radius;
    int32_t incl_phase;
    int32_t law;
    int32_t bc;
    int32_t elem;
} rve_mesh_desc;

#define RVE_ELEM_Q1 0
#define RVE_ELEM_P1 1

#define RVE_BC_PERIODIC 0
#define RVE_BC_LINEAR 1

#define RVE_LAW_NEOHOOKE 0
#define RVE_LAW_SVK 1
#define RVE_LAW_LINEAR 2

int rve_mesh_create(const rve_mesh_desc* desc, rve_mesh* out);
int rve_mesh_destroy(rve_mesh m);
/* Copies the element phases (n^d bytes) to host memory. */
int rve_mesh_get_phase(rve_mesh m, uint8_t* host_phase);

/* ---- batches -----------------------------------------------------------------
 * rve_batch_create: B RVEs (host array of mesh handles, sizes may differ).  The
 * meshes must outlive the batch.  Allocates the device workspaces of the
 * persistent solver; the device pointers are fixed for the life of the handle, so
 * rve_solve_batch can be captured in a HIP graph.  w_state of RVE r occupies
 * doubles [off[r], off[r+1]) with off[r+1]-off[r] = d * n_r^d. */
int rve_batch_create(const rve_mesh* meshes, int64_t B, rve_batch* out);
int rve_batch_destroy(rve_batch b);
int rve_batch_state_offsets(rve_batch b, int64_t* host_off /* [B+1] */);

#define RVE_PREC_FP64 0
/* FP32: the Newton element tangents are stored in FP32 and factored in FP32 (MFMA
 * trailing updates); the Newton residual, its norm, the det F guard and the
 * refinement residual b - K x stay FP64, with K x applied matrix-free by the
 * element kernel in FP64 (no FP64 matrix is stored); the tangent condensation
 * takes FP64 element tangents of the converged state.  (The paper's method is
 * FP64 throughout; this is an acceleration whose outputs meet the FP64 bar:
 * Newton counts may differ by one from the FP64 solve's.) */
#define RVE_PREC_FP32_IR 1 /* FP32 assembly and factorization, FP64 residuals + refinement */

typedef struct {
    double rtol;           /* Newton: stop when ||R_f||_2 <= rtol ||R_f^0||_2 + atol */
    double atol;           /* < 0: per-RVE default 1e-12 * mu_max * h^(d-1) */
    int32_t max_iter;      /* Newton updates before RVE_S_NOCONV */
    int32_t precision;     /* RVE_PREC_* */
    int32_t det_backtrack; /* halvings of a Newton step while some J <= 0 */
    int32_t flags;         /* RVE_FLAG_* */
} rve_opts;

/* With this flag an RVE that reaches max_iter updates without meeting the
 * tolerance still gets P and A evaluated at its last state (and stores it in
 * w_state); its status is RVE_S_NOCONV.  The alternating two-level Newton of
 * Sec. 5.2 (one micro update per macro iteration) relies on it. */
#define RVE_FLAG_OUTPUTS_AT_CAP 1
/* The condensation of Sec. 3.3 (A = <A> - Y^T K^-1 Y at the converged state w)
 * by default reuses the last Newton factorization (2D meshes, and 3D meshes
 * whose fronts live in global memory): when the quadratic convergence model
 * r_next = r^3 / r_prev^2 predicts that the next Newton state converges, that
 * factorization (of the tangent K' one Newton step before w) also takes the d^2
 * columns Y' of its state.  X = K'^-1 Y' is then one backward substitution, and
 * A = <A> - Y^T X - X^T (Y - K X) with Y, K of w is exact up to
 * (X - X*)^T K (X - X*), second order in the last Newton step (X is refined
 * while ||Y - K X||_F > 1e-4 ||Y||_F).  Where the prediction missed, and on 3D
 * meshes whose fronts fit LDS, a factorization at w is made.  With this flag the
 * condensation always factorizes at w (the direct Schur form). */
#define RVE_FLAG_DIRECT_TANGENT 2

/* rtol 1e-10, atol -1 (default), max_iter 25, FP64, det_backtrack 8, flags 0 */
void rve_opts_default(rve_opts* o);

/* ---- the hot path ------------------------------------------------------------
 * rve_solve_batch: solve every RVE of the batch for its macro deformation.
 * All array arguments are DEVICE pointers owned by the caller:
 *   F        [B][d*d]   in   macro deformation gradient per RVE (det F > 0)
 *   P        [B][d*d]   out  Pbar
 *   A        [B][d^4]   out  Abar = dPbar/dFbar (may be NULL: tangent skipped)
 *   w_state  ragged     in/out warm start and converged fluctuation per RVE
 *                       (layout from rve_batch_state_offsets); NULL: zero start,
 *                       nothing stored
 *   status   [B] int32  out  RVE_S_* per RVE (may be NULL)
 *   iters    [B] int32  out  Newton updates per RVE (may be NULL)
 * All meshes of a batch share d (rve_batch_create rejects a mix).  The call is
 * asynchronous on hip_stream (a hipStream_t; NULL = default stream); results are
 * valid after the stream synchronizes.  Returns RVE_OK once the work is
 * enqueued; per-RVE failures are only visible in status[] (RVE_EPARTIAL is
 * returned by rve_solve_batch_sync). */
int rve_solve_batch(rve_batch b, const double* F, double* P, double* A, double* w_state, int32_t* status,
                    int32_t* iters, const rve_opts* opts, void* hip_stream);

/* As rve_solve_batch, restricted to the RVEs listed in idx[0 .. *count) (both
 * device pointers; the count is read on the device when the kernel runs, so a
 * list produced by an earlier kernel on the same stream needs no host round
 * trip).  Entries outside [0, B) are skipped; RVEs not listed keep their P, A,
 * w_state, status and iters untouched.  This is the fallback path of the
 * surrogate (surrogate.h: rve_surrogate_select).  Asynchronous. */
int rve_solve_batch_subset(rve_batch b, const int32_t* idx, const int32_t* count, const double* F, double* P,
                           double* A, double* w_state, int32_t* status, int32_t* iters, const rve_opts* opts,
                           void* hip_stream);

/* As rve_solve_batch, then synchronizes the stream and returns RVE_EPARTIAL if
 * any RVE failed (status must then be non-NULL). */
int rve_solve_batch_sync(rve_batch b, const double* F, double* P, double* A, double* w_state, int32_t* status,
                         int32_t* iters, const rve_opts* opts, void* hip_stream);

/* ---- solve without allocation --------------------------------------------------
 * rve_solve_batch_static: for callers that cannot allocate device memory while
 * they solve (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and asynchrony as rve_solve_batch,
 * bitwise identical outputs; the solver's workspace (the persistent queue counter
 * and one slot per persistent workgroup) lives in a static device array of
 * RVE_STATIC_SCRATCH_BYTES instead of the batch's own slots, so the call makes
 * no hipMalloc, hipFree or other allocating call.  The number of persistent
 * workgroups is min(the batch's slots, what fits the array): 1398 for 2D 8 x 8,
 * 232 for 16 x 16, 43 for 32 x 32 (rve_solve_batch: up to 1024), so batches of
 * large RVEs take longer; 3D: 19 (8^3), 4 (12^3), 1 (16^3).
 * Each device holds its own copy of the array from the first call on it until
 * the process ends (the first call on a device also looks its address up).
 * Errors: RVE_EINVAL when one slot of the batch exceeds the array (3D meshes
 * beyond 16^3) or when the batch was created on another device than the current
 * one; otherwise as rve_solve_batch.
 * All calls on one device share its array: calls that overlap on one device
 * (other streams, other threads) race and give wrong results; serialize them
 * (one stream, or events).  The array keeps the last call's contents; the queue
 * counter is cleared by the call itself, and nothing else needs to start at zero. */
#define RVE_STATIC_SCRATCH_BYTES (256ull << 20)
int rve_solve_batch_static(rve_batch b, const double* F, double* P, double* A, double* w_state, int32_t* status,
                           int32_t* iters, const rve_opts* opts, void* hip_stream);

/* ---- autotuning -------------------------------------------------------------
 * Choices that shape the solve of one mesh size: the leaf size of the nested
 * dissection (largest leaf box, in nodes: front sizes and tree depth), the
 * largest front that one wave factors on its own (small subtrees run
 * wave-per-front, larger fronts use the whole workgroup), the number of
 * persistent workgroups of a batch, and the workgroup size (four waves, or eight
 * waves for 2D plans whose fronts live in LDS).  rve_autotune times candidates
 * on the caller's own deformation gradients and keeps the fastest for (ndim,
 * n); meshes and batches created afterwards use it.  Results stay within the
 * parity bar for any choice (only the elimination order and the schedule
 * change). */
typedef struct {
    int32_t leaf;        /* 0: default (16 nodes in 2D, 27 in 3D) */
    int32_t wave_max_m;  /* 0 .. 64; 64 is the default */
    int32_t slots;       /* 0: default (min(B, 1024)) */
    int32_t threads;     /* 0: by front size (eight waves when the fronts leave room for one four-wave
                            workgroup per CU only), 256 or 512; 512 applies to 2D plans with fronts
                            in LDS and is taken as 256 elsewhere */
    double ms;           /* measured time of the tuning batch (rve_autotune), else 0 */
} rve_tuning;

/* Times every candidate (leaf in {8, 16, 32} (2D) or {8, 27, 64} (3D), wave
 * limit in {0, 32, 64} where fronts fit LDS, slots in {512, 1024}, threads in
 * {256, 512} for 2D plans with fronts in LDS) with rve_solve_batch on nF RVEs
 * of mesh m's microstructure driven by F (device, [nF][d^2]) and options o
 * (timed in o's precision), keeps the fastest for (ndim, n) and returns it in
 * best.  Host-blocking; allocates its own buffers. */
int rve_autotune(rve_mesh m, const double* F, int64_t nF, const rve_opts* o, rve_tuning* best, void* hip_stream);
/* Current choice for (ndim, n) (defaults when untuned); set installs one (e.g.
 * saved from an earlier run); reset returns (ndim, n) -- or every size when
 * n == 0 -- to the defaults.  Affect meshes and batches created afterwards. */
int rve_tuning_get(int32_t ndim, int32_t n, rve_tuning* out);
int rve_tuning_set(int32_t ndim, int32_t n, const rve_tuning* t);
int rve_tuning_reset(int32_t ndim, int32_t n);

/* Algorithmic work of the last plan for (ndim, n): floating-point operations of
 * one LDL^T factorization, nonzeros of L, front count and largest front. */
int rve_plan_info(int32_t ndim, int32_t n, double* factor_flops, int64_t* nnz_L, int32_t* nfronts,
                  int32_t* max_front);

/* Introspection of the (ndim, n) plan, for tooling and tests (host only).
 * sizes[6] receives the counts (fronts, rows, relind, children, kpair,
 * kcontrib); each non-NULL array receives: fronts [nf][8] = (m, p, parent,
 * rows_off, relind_off, child_begin, child_end, kmap_begin) in elimination
 * (post)order, rows (global dof = node*d+comp of every front row, pivots
 * first), relind (positions of a front's update rows in its parent front),
 * children, kpair [.][4] = (row node, pivot node, contrib begin, count) in
 * front-local node indices, kcontrib [.][3] = (element, local a, local b). */
int rve_plan_export(int32_t ndim, int32_t n, int64_t* sizes, int32_t* fronts, int32_t* rows, int32_t* relind,
                    int32_t* children, int32_t* kpair, int32_t* kcontrib);

/* Processing schedule of the (ndim, n) plan's LDS path, for tooling and tests
 * (host only).  *nsteps receives the number of workgroup-front steps (0 when
 * the fronts live in global memory); steps, if non-NULL, receives [nsteps][4]
 * in processing order: the 1, 2 or 4 fronts processed side by side on equal
 * parts of the workgroup, -1 padded; wave, if non-NULL, receives one flag per
 * front (elimination order): 1 for the fronts eliminated one per wave before
 * the workgroup fronts. */
int rve_plan_schedule(int32_t ndim, int32_t n, int64_t* nsteps, int32_t* steps, int32_t* wave);

/* ---- the assembly phase alone ------------------------------------------------
 * rve_assemble_batch: runs one assembly of every RVE of the batch -- the element
 * pass (F at the Gauss points, the neo-Hookean P and A, element residual and
 * tangent) and the node gather of the residual, Sec. 3.3 -- at its stored
 * fluctuation (w_state, may be NULL: zero) and the macro gradient F, into the
 * batch's workspace, without the linear solve.  It exists to time the assembly
 * phase of the Newton iteration on its own.  status [B] (may be NULL) receives
 * RVE_S_DETF where some J <= 0, else RVE_S_CONVERGED.  Asynchronous. */
int rve_assemble_batch(rve_batch b, const double* F, const double* w_state, int32_t* status, void* hip_stream);

/* ---- measured ceilings -------------------------------------------------------
 * rve_probe_peaks: rates this device reaches on plain probes, for reading the
 * solver's roofline fractions beside the published peaks: dense FP64 and FP32
 * MFMA (v_mfma_*_16x16x4, eight independent accumulators per wave, eight
 * four-wave workgroups per CU) in TFLOP/s, and a 1 GiB device-to-device copy in
 * GB/s (bytes read + written).  Host-blocking; allocates and frees 2 GiB. */
int rve_probe_peaks(double* fp64_mfma_tflops, double* fp32_mfma_tflops, double* hbm_copy_gbs, void* hip_stream);

/* ---- errors ------------------------------------------------------------------ */
const char* rve_strerror(int code);
/* Copies the calling thread's last error message (NUL-terminated) into buf. */
int rve_last_error(char* buf, size_t n);

#ifdef __cplusplus
}
#endif
#endif /* FEHMM_RVE_H */
