/*
 * rve.c -- FP64 CPU oracle for one periodic RVE (test infrastructure only; the
 * product library never links it).
 *
 * Everything here is written in the paper's total-Lagrangian notation:
 *   S, C (= 4 d^2 psi / dC dC) from the neo-Hookean energy of Sec. 6,
 *   B_I (dE = B_I dd_I), f_I = int B_I^T S, k_IK = int B_I^T C B_K + S_hat_IK 1
 *   (Sec. 3.3, eqs. DG^h, G_IK-InitStressMatr, S_IK), and the micro-to-macro
 *   stiffness transfer T^T K T / |K_delta| of Sec. 3.2 evaluated with the d^2 unit
 *   macro-gradient states.  Periodic partner nodes are identified (the PBC form of
 *   eq. ConstraintCondition), so G^T dLambda = 0 drops out as the paper notes.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "sparse.h"

#define MAXD 3
#define MAXNE 8   /* nodes per element */
#define MAXV 6    /* Voigt size */

/* ------------------------------------------------------------------ small linear algebra */
static double det_d(int d, const double* A) {
    if (d == 2) return A[0] * A[3] - A[1] * A[2];
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

static void inv_d(int d, const double* A, double* Ai) {
    double D = det_d(d, A);
    if (d == 2) {
        Ai[0] = A[3] / D; Ai[1] = -A[1] / D; Ai[2] = -A[2] / D; Ai[3] = A[0] / D;
        return;
    }
    Ai[0] = (A[4] * A[8] - A[5] * A[7]) / D;
    Ai[1] = (A[2] * A[7] - A[1] * A[8]) / D;
    Ai[2] = (A[1] * A[5] - A[2] * A[4]) / D;
    Ai[3] = (A[5] * A[6] - A[3] * A[8]) / D;
    Ai[4] = (A[0] * A[8] - A[2] * A[6]) / D;
    Ai[5] = (A[2] * A[3] - A[0] * A[5]) / D;
    Ai[6] = (A[3] * A[7] - A[4] * A[6]) / D;
    Ai[7] = (A[1] * A[6] - A[0] * A[7]) / D;
    Ai[8] = (A[0] * A[4] - A[1] * A[3]) / D;
}

/* ------------------------------------------------------------------ constitutive law */
/* Compressible neo-Hookean law, eq. (NH-free-energy) and the S, C_ijkl, A_ijkl
 * expressions that follow it (Sec. 6).  In 2D (plane strain) C is the in-plane
 * 2x2 block, C_33 = 1, so tr C = C11 + C22 + 1 and J = det of the in-plane F. */
int oracle_nh_sc(int d, double lam, double mu, const double* F, double* S, double* Cmat, double* psi) {
    double C[9], Ci[9];
    for (int I = 0; I < d; ++I)
        for (int J = 0; J < d; ++J) {
            double s = 0;
            for (int k = 0; k < d; ++k) s += F[k * d + I] * F[k * d + J];
            C[I * d + J] = s;
        }
    double Jdet = det_d(d, F);
    if (!(Jdet > 0)) return ORC_DETF;
    inv_d(d, C, Ci);
    double J2 = Jdet * Jdet;
    for (int I = 0; I < d; ++I)
        for (int J = 0; J < d; ++J)
            S[I * d + J] = 0.5 * lam * (J2 - 1.0) * Ci[I * d + J] + mu * ((I == J ? 1.0 : 0.0) - Ci[I * d + J]);
    if (Cmat) {
        double c1 = lam * (J2 - 1.0) - 2.0 * mu;
        for (int I = 0; I < d; ++I)
            for (int J = 0; J < d; ++J)
                for (int K = 0; K < d; ++K)
                    for (int L = 0; L < d; ++L) {
                        double Aijkl = -0.5 * (Ci[I * d + K] * Ci[J * d + L] + Ci[J * d + K] * Ci[I * d + L]);
                        Cmat[((I * d + J) * d + K) * d + L] = c1 * Aijkl + lam * J2 * Ci[I * d + J] * Ci[K * d + L];
                    }
    }
    if (psi) {
        double trC = 0;
        for (int I = 0; I < d; ++I) trC += C[I * d + I];
        if (d == 2) trC += 1.0;
        *psi = 0.25 * lam * (J2 - 1.0) - (0.5 * lam + mu) * log(Jdet) + 0.5 * mu * (trC - 3.0);
    }
    return ORC_OK;
}

/* The constitutive variants of the paper's examples (Sec. 6 material table and
 * micro-convergence studies): geometrically nonlinear linear elasticity, i.e.
 * the St. Venant-Kirchhoff law S = lambda tr(E) 1 + 2 mu E with the
 * Green-Lagrange strain E = (C - 1)/2 (psi = lambda/2 tr(E)^2 + mu E:E), and the
 * fully linear case, small strain eps = sym(F - 1), sigma = lambda tr(eps) 1 +
 * 2 mu eps, which takes the place of both S and P (no geometric stiffness).
 * Cmat is the constant C_IJKL = lambda d_IJ d_KL + mu (d_IK d_JL + d_IL d_JK) for
 * both.  2D is plane strain (E_33 = eps_33 = 0).  The J > 0 guard is kept for
 * every law. */
static int g_law = ORC_LAW_NEOHOOKE;

void oracle_set_law(int law) { g_law = law; }
int oracle_get_law(void) { return g_law; }

int oracle_law_sc(int law, int d, double lam, double mu, const double* F, double* S, double* Cmat, double* psi) {
    if (law == ORC_LAW_NEOHOOKE) return oracle_nh_sc(d, lam, mu, F, S, Cmat, psi);
    if (!(det_d(d, F) > 0)) return ORC_DETF;
    double E[9];
    for (int I = 0; I < d; ++I)
        for (int J = 0; J < d; ++J) {
            double v;
            if (law == ORC_LAW_SVK) {
                v = 0;
                for (int k = 0; k < d; ++k) v += F[k * d + I] * F[k * d + J];
                v = 0.5 * (v - (I == J ? 1.0 : 0.0));
            } else {
                v = 0.5 * (F[I * d + J] + F[J * d + I]) - (I == J ? 1.0 : 0.0);
            }
            E[I * d + J] = v;
        }
    double trE = 0, EE = 0;
    for (int I = 0; I < d; ++I) trE += E[I * d + I];
    for (int q = 0; q < d * d; ++q) EE += E[q] * E[q];
    for (int I = 0; I < d; ++I)
        for (int J = 0; J < d; ++J) S[I * d + J] = (I == J ? lam * trE : 0.0) + 2.0 * mu * E[I * d + J];
    if (Cmat)
        for (int I = 0; I < d; ++I)
            for (int J = 0; J < d; ++J)
                for (int K = 0; K < d; ++K)
                    for (int L = 0; L < d; ++L)
                        Cmat[((I * d + J) * d + K) * d + L] = (I == J && K == L ? lam : 0.0) +
                                                              mu * ((I == K && J == L ? 1.0 : 0.0) +
                                                                    (I == L && J == K ? 1.0 : 0.0));
    if (psi) *psi = 0.5 * lam * trE * trE + mu * EE;
    return ORC_OK;
}

/* Micro boundary conditions (Sec. 3.2, eq. ConstraintCondition and the list of
 * energetically consistent couplings).  Periodic: the fluctuation is periodic,
 * partner nodes are identified and node 0 is pinned against rigid translation.
 * Linear displacement (KUBC): u = Fbar X on the boundary, i.e. the fluctuation
 * vanishes on every boundary node and only interior nodes are free.  On the
 * n^d node numbering the boundary faces x_k = 0 and x_k = 1 are the nodes with
 * grid index 0 (the periodic wrap maps x_k = 1 onto them), and both carry w = 0,
 * so the element loop is the same for both couplings: only the set of pinned
 * nodes changes -- every node with some grid index 0. */
static int g_bc = ORC_BC_PERIODIC;

void oracle_set_bc(int bc) { g_bc = bc; }
int oracle_get_bc(void) { return g_bc; }

static int is_pinned(int d, int n, int node) {
    if (g_bc == ORC_BC_PERIODIC) return node == 0;
    for (int k = 0; k < d; ++k) {
        if (node % n == 0) return 1;
        node /= n;
    }
    return 0;
}

/* first Piola-Kirchhoff stress: P = F S, or sigma itself in the fully linear case */
static void first_piola(int d, const double* F, const double* S, double* P) {
    for (int i = 0; i < d; ++i)
        for (int J = 0; J < d; ++J) {
            double v = 0;
            if (g_law == ORC_LAW_LINEAR) v = S[i * d + J];
            else
                for (int K = 0; K < d; ++K) v += F[i * d + K] * S[K * d + J];
            P[i * d + J] = v;
        }
}

/* ------------------------------------------------------------------ mesh */
static int ipow(int n, int d) { int r = 1; for (int i = 0; i < d; ++i) r *= n; return r; }

/* local node a of an element: offsets in {0,1}^d, counter-clockwise in 2D, hex order in 3D */
static void local_offset(int d, int a, int* o) {
    static const int q[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    o[0] = q[a & 3][0];
    o[1] = q[a & 3][1];
    if (d == 3) o[2] = a >> 2;
}

static void element_nodes(int d, int n, int e, int* nodes) {
    int c[MAXD];
    int t = e;
    for (int k = 0; k < d; ++k) { c[k] = t % n; t /= n; }
    int nen = 1 << d;
    for (int a = 0; a < nen; ++a) {
        int o[MAXD];
        local_offset(d, a, o);
        int id = 0, s = 1;
        for (int k = 0; k < d; ++k) { id += ((c[k] + o[k]) % n) * s; s *= n; }
        nodes[a] = id;
    }
}

void oracle_phase_by_centroid(int d, int n, const double* center, double r, int incl_phase, int base_phase,
                              uint8_t* phase) {
    int ne = ipow(n, d);
    double h = 1.0 / n;
    for (int e = 0; e < ne; ++e) {
        int t = e;
        double dist2 = 0;
        for (int k = 0; k < d; ++k) {
            double x = ((t % n) + 0.5) * h - center[k];
            dist2 += x * x;
            t /= n;
        }
        phase[e] = (uint8_t)(sqrt(dist2) < r ? incl_phase : base_phase);
    }
}

/* Micro element kind.  ORC_ELEM_Q1: bilinear quadrilaterals / trilinear
 * hexahedra with 2^d Gauss points.  ORC_ELEM_P1: the paper's linear simplices
 * (P1, Sec. 3.1 micro spaces), here the Kuhn triangulation of every grid cell
 * into d! simplices sharing the cell's diagonal from local corner (0..0) to
 * (1..1) (conforming across cells): the simplex of axis order s visits
 * 0, e_s0, e_s0 + e_s1, ..., 1; its barycentric gradients are -e_s0 / h,
 * (e_s(k-1) - e_sk) / h and e_s(d-1) / h.  The phase of a simplex is its cell's. */
static int g_elem = ORC_ELEM_Q1;

void oracle_set_element(int kind) { g_elem = kind; }
int oracle_get_element(void) { return g_elem; }

/* Integration points of one cell: gradients dN[p][a][k] of the cell's 2^d local
 * nodes (zero for a node the point's simplex does not contain, P1) and the weight
 * wJ of each point; returns the number of points. */
static int shape_grads(int d, int n, double dN[MAXNE][MAXNE][MAXD], double* wJ) {
    double h = 1.0 / n;
    int nen = 1 << d;
    if (g_elem == ORC_ELEM_P1) {
        int perm[6][3], np = 0;
        if (d == 2) {
            int q[2][2] = {{0, 1}, {1, 0}};
            for (int t = 0; t < 2; ++t) { perm[t][0] = q[t][0]; perm[t][1] = q[t][1]; }
            np = 2;
        } else {
            int q[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
            for (int t = 0; t < 6; ++t) for (int k = 0; k < 3; ++k) perm[t][k] = q[t][k];
            np = 6;
        }
        for (int p = 0; p < np; ++p) {
            for (int a = 0; a < nen; ++a) for (int k = 0; k < d; ++k) dN[p][a][k] = 0.0;
            int v[MAXD] = {0, 0, 0};
            for (int j = 0; j <= d; ++j) {  /* vertex j of the simplex */
                if (j > 0) v[perm[p][j - 1]] = 1;
                int a = -1;
                for (int b = 0; b < nen; ++b) {
                    int o[MAXD];
                    local_offset(d, b, o);
                    int same = 1;
                    for (int k = 0; k < d; ++k) same &= o[k] == v[k];
                    if (same) a = b;
                }
                double g[MAXD] = {0, 0, 0};
                if (j == 0) g[perm[p][0]] = -1.0;
                else if (j == d) g[perm[p][d - 1]] = 1.0;
                else { g[perm[p][j - 1]] = 1.0; g[perm[p][j]] = -1.0; }
                for (int k = 0; k < d; ++k) dN[p][a][k] = g[k] / h;
            }
        }
        *wJ = pow(h, d) / (d == 2 ? 2.0 : 6.0);
        return np;
    }
    double gq = 1.0 / sqrt(3.0);
    for (int p = 0; p < nen; ++p) {
        int op[MAXD];
        local_offset(d, p, op);
        double xi[MAXD];
        for (int k = 0; k < d; ++k) xi[k] = op[k] ? gq : -gq;
        for (int a = 0; a < nen; ++a) {
            int oa[MAXD];
            local_offset(d, a, oa);
            double sa[MAXD];
            for (int k = 0; k < d; ++k) sa[k] = oa[k] ? 1.0 : -1.0;
            for (int k = 0; k < d; ++k) {
                double vv = 1.0;
                for (int m = 0; m < d; ++m) vv *= (m == k) ? 0.5 * sa[m] : 0.5 * (1.0 + sa[m] * xi[m]);
                dN[p][a][k] = vv * 2.0 / h; /* dN/dX = dN/dxi * 2/h */
            }
        }
    }
    *wJ = pow(0.5 * h, d);
    return nen;
}

/* Voigt pairs (engineering shear) */
static int voigt_pairs(int d, int pr[MAXV][2]) {
    if (d == 2) {
        pr[0][0] = 0; pr[0][1] = 0; pr[1][0] = 1; pr[1][1] = 1; pr[2][0] = 0; pr[2][1] = 1;
        return 3;
    }
    pr[0][0] = 0; pr[0][1] = 0; pr[1][0] = 1; pr[1][1] = 1; pr[2][0] = 2; pr[2][1] = 2;
    pr[3][0] = 0; pr[3][1] = 1; pr[4][0] = 1; pr[4][1] = 2; pr[5][0] = 0; pr[5][1] = 2;
    return 6;
}

/* Element residual and tangent in B-matrix form (Sec. 3.3). */
int oracle_element(int d, int n, const uint8_t* phase, const double* lame, int e, const double* Fbar,
                   const double* w, double* fe, double* ke, double* energy) {
    double dN[MAXNE][MAXNE][MAXD], wJ;
    const int npt = shape_grads(d, n, dN, &wJ);
    int nen = 1 << d, nd = nen * d;
    int nodes[MAXNE];
    element_nodes(d, n, e, nodes);
    /* (npt integration points: the Q1 Gauss points or the cell's P1 simplices) */
    double lam = lame[2 * phase[e]], mu = lame[2 * phase[e] + 1];
    int pr[MAXV][2];
    int nv = voigt_pairs(d, pr);
    if (fe) memset(fe, 0, sizeof(double) * nd);
    if (ke) memset(ke, 0, sizeof(double) * nd * nd);
    double en = 0;
    for (int p = 0; p < npt; ++p) {
        double F[9];
        for (int i = 0; i < d; ++i)
            for (int J = 0; J < d; ++J) {
                double s = Fbar[i * d + J];
                for (int a = 0; a < nen; ++a) s += w[nodes[a] * d + i] * dN[p][a][J];
                F[i * d + J] = s;
            }
        double S[9], Cm[81], psi;
        int st = oracle_law_sc(g_law, d, lam, mu, F, S, Cm, &psi);
        if (st) return st;
        en += psi * wJ;
        /* B[r][a*d+k] : dE_r = sum B dd (the linear B at F = 1 in the fully linear case) */
        const int lin = g_law == ORC_LAW_LINEAR;
        double B[MAXV][MAXNE * MAXD];
        for (int r = 0; r < nv; ++r) {
            int I = pr[r][0], J = pr[r][1];
            for (int a = 0; a < nen; ++a)
                for (int k = 0; k < d; ++k) {
                    double fkI = lin ? (k == I ? 1.0 : 0.0) : F[k * d + I];
                    double fkJ = lin ? (k == J ? 1.0 : 0.0) : F[k * d + J];
                    double v = fkI * dN[p][a][J];
                    if (I != J) v += fkJ * dN[p][a][I];
                    B[r][a * d + k] = v;
                }
        }
        double Sv[MAXV], Cv[MAXV][MAXV];
        for (int r = 0; r < nv; ++r) {
            Sv[r] = S[pr[r][0] * d + pr[r][1]];
            for (int s = 0; s < nv; ++s)
                Cv[r][s] = Cm[((pr[r][0] * d + pr[r][1]) * d + pr[s][0]) * d + pr[s][1]];
        }
        if (fe)
            for (int q = 0; q < nd; ++q) {
                double s = 0;
                for (int r = 0; r < nv; ++r) s += B[r][q] * Sv[r];
                fe[q] += s * wJ;
            }
        if (ke) {
            double CB[MAXV][MAXNE * MAXD];
            for (int r = 0; r < nv; ++r)
                for (int q = 0; q < nd; ++q) {
                    double s = 0;
                    for (int t = 0; t < nv; ++t) s += Cv[r][t] * B[t][q];
                    CB[r][q] = s;
                }
            for (int q1 = 0; q1 < nd; ++q1)
                for (int q2 = 0; q2 < nd; ++q2) {
                    double s = 0;
                    for (int r = 0; r < nv; ++r) s += B[r][q1] * CB[r][q2];
                    ke[q1 * nd + q2] += s * wJ;
                }
            /* initial-stress matrix S_hat_IK 1 (geometric stiffness; none in the fully linear case) */
            for (int a = 0; a < nen && !lin; ++a)
                for (int b = 0; b < nen; ++b) {
                    double sh = 0;
                    for (int I = 0; I < d; ++I)
                        for (int J = 0; J < d; ++J) sh += dN[p][a][I] * S[I * d + J] * dN[p][b][J];
                    for (int k = 0; k < d; ++k) ke[(a * d + k) * nd + (b * d + k)] += sh * wJ;
                }
        }
    }
    if (energy) *energy = en;
    return ORC_OK;
}

int oracle_residual(int d, int n, const uint8_t* phase, const double* lame, const double* Fbar, const double* w,
                    double* R, double* energy) {
    int ne = ipow(n, d), nen = 1 << d, nd = nen * d;
    memset(R, 0, sizeof(double) * d * ne);
    double en = 0;
    for (int e = 0; e < ne; ++e) {
        double fe[MAXNE * MAXD], ee;
        int nodes[MAXNE];
        int st = oracle_element(d, n, phase, lame, e, Fbar, w, fe, NULL, &ee);
        if (st) return st;
        element_nodes(d, n, e, nodes);
        for (int q = 0; q < nd; ++q) R[nodes[q / d] * d + q % d] += fe[q];
        en += ee;
    }
    if (energy) *energy = en;
    return ORC_OK;
}

/* ------------------------------------------------------------------ RVE system (periodic or KUBC) */
typedef struct {
    int d, n, nn, ne, nf;  /* nf: free dofs */
    int* dof;              /* dof[node*d+k] -> free index or -1 (pinned node) */
    skyline K;
} rve_sys;

static void rve_sys_free(rve_sys* r) { free(r->dof); sky_free(&r->K); }

static int rve_sys_init(rve_sys* r, int d, int n) {
    memset(r, 0, sizeof(*r));
    r->d = d; r->n = n; r->nn = ipow(n, d); r->ne = r->nn;
    /* free nodes (not pinned) in ascending order and the graph among them */
    int* fid = (int*)malloc(sizeof(int) * r->nn); /* node -> compact free index or -1 */
    int nv = 0;
    for (int node = 0; node < r->nn; ++node) fid[node] = is_pinned(d, n, node) ? -1 : nv++;
    r->nf = d * nv;
    int* fnode = (int*)malloc(sizeof(int) * (nv ? nv : 1));
    for (int node = 0; node < r->nn; ++node) if (fid[node] >= 0) fnode[fid[node]] = node;
    int nb = ipow(3, d);
    int* xadj = (int*)malloc(sizeof(int) * (nv + 1));
    int* adj = (int*)calloc((size_t)nv * nb + 1, sizeof(int));
    int cnt = 0;
    for (int v = 0; v < nv; ++v) {
        int node = fnode[v], c[MAXD], t = node;
        for (int k = 0; k < d; ++k) { c[k] = t % n; t /= n; }
        xadj[v] = cnt;
        for (int o = 0; o < nb; ++o) {
            int oo = o, id = 0, s = 1;
            for (int k = 0; k < d; ++k) { int dk = oo % 3 - 1; oo /= 3; id += ((c[k] + dk + n) % n) * s; s *= n; }
            if (id == node || fid[id] < 0) continue;
            int dup = 0;
            for (int q = xadj[v]; q < cnt; ++q) if (adj[q] == fid[id]) dup = 1;
            if (!dup) adj[cnt++] = fid[id];
        }
    }
    xadj[nv] = cnt;
    int* perm = (int*)malloc(sizeof(int) * (nv ? nv : 1));
    if (nv) rcm(nv, xadj, adj, perm);
    int* pos = (int*)malloc(sizeof(int) * (nv ? nv : 1));
    for (int k = 0; k < nv; ++k) pos[perm[k]] = k;
    r->dof = (int*)malloc(sizeof(int) * d * r->nn);
    for (int node = 0; node < r->nn; ++node)
        for (int k = 0; k < d; ++k) r->dof[node * d + k] = fid[node] < 0 ? -1 : pos[fid[node]] * d + k;
    /* profile: first column of each row = smallest dof of any neighbour node */
    int* fc = (int*)malloc(sizeof(int) * (r->nf ? r->nf : 1));
    for (int v = 0; v < nv; ++v) {
        int mn = pos[v];
        for (int q = xadj[v]; q < xadj[v + 1]; ++q) if (pos[adj[q]] < mn) mn = pos[adj[q]];
        for (int k = 0; k < d; ++k) fc[pos[v] * d + k] = mn * d;
    }
    free(fid); free(fnode);
    int st = sky_alloc(&r->K, r->nf, fc);
    free(fc); free(pos); free(perm); free(adj); free(xadj);
    return st;
}

/* Assemble R (full, node-major) and the free-free tangent into r->K.
 * Returns ORC_DETF if some Gauss point has J <= 0. */
static int rve_assemble(rve_sys* r, const uint8_t* phase, const double* lame, const double* Fbar,
                        const double* w, double* R, int want_K) {
    int d = r->d, n = r->n, nen = 1 << d, nd = nen * d;
    memset(R, 0, sizeof(double) * d * r->nn);
    if (want_K) memset(r->K.val, 0, sizeof(double) * r->K.ptr[r->K.N]);
    double fe[MAXNE * MAXD], ke[MAXNE * MAXD * MAXNE * MAXD];
    for (int e = 0; e < r->ne; ++e) {
        int nodes[MAXNE];
        int st = oracle_element(d, n, phase, lame, e, Fbar, w, fe, want_K ? ke : NULL, NULL);
        if (st) return st;
        element_nodes(d, n, e, nodes);
        for (int q = 0; q < nd; ++q) R[nodes[q / d] * d + q % d] += fe[q];
        if (!want_K) continue;
        for (int q1 = 0; q1 < nd; ++q1) {
            int g1 = r->dof[nodes[q1 / d] * d + q1 % d];
            if (g1 < 0) continue;
            for (int q2 = 0; q2 <= q1; ++q2) {
                int g2 = r->dof[nodes[q2 / d] * d + q2 % d];
                if (g2 < 0) continue;
                sky_add(&r->K, g1, g2, ke[q1 * nd + q2]);
            }
        }
    }
    return ORC_OK;
}

static double norm_free(const rve_sys* r, const double* R) {
    double s = 0;
    for (int i = 0; i < r->d * r->nn; ++i)
        if (r->dof[i] >= 0) s += R[i] * R[i];
    return sqrt(s);
}

static int all_J_positive(const rve_sys* r, const uint8_t* phase, const double* lame, const double* Fbar,
                          const double* w) {
    double dN[MAXNE][MAXNE][MAXD], wJ;
    int d = r->d, nen = 1 << d;
    const int npt = shape_grads(d, r->n, dN, &wJ);
    (void)phase; (void)lame;
    for (int e = 0; e < r->ne; ++e) {
        int nodes[MAXNE];
        element_nodes(d, r->n, e, nodes);
        for (int p = 0; p < npt; ++p) {
            double F[9];
            for (int i = 0; i < d; ++i)
                for (int J = 0; J < d; ++J) {
                    double s = Fbar[i * d + J];
                    for (int a = 0; a < nen; ++a) s += w[nodes[a] * d + i] * dN[p][a][J];
                    F[i * d + J] = s;
                }
            if (!(det_d(d, F) > 0)) return 0;
        }
    }
    return 1;
}

/* P = <P^eps> = sum_gp P(F) w|J| / |B_0| with |B_0| = 1 (eq. Average-of-P-and-F); P = F S, or sigma in
 * the fully linear case. */
static void average_P(const rve_sys* r, const uint8_t* phase, const double* lame, const double* Fbar,
                      const double* w, double* P) {
    double dN[MAXNE][MAXNE][MAXD], wJ;
    int d = r->d, nen = 1 << d;
    const int npt = shape_grads(d, r->n, dN, &wJ);
    memset(P, 0, sizeof(double) * d * d);
    for (int e = 0; e < r->ne; ++e) {
        int nodes[MAXNE];
        element_nodes(d, r->n, e, nodes);
        double lam = lame[2 * phase[e]], mu = lame[2 * phase[e] + 1];
        for (int p = 0; p < npt; ++p) {
            double F[9], S[9];
            for (int i = 0; i < d; ++i)
                for (int J = 0; J < d; ++J) {
                    double s = Fbar[i * d + J];
                    for (int a = 0; a < nen; ++a) s += w[nodes[a] * d + i] * dN[p][a][J];
                    F[i * d + J] = s;
                }
            double Pq[9];
            oracle_law_sc(g_law, d, lam, mu, F, S, NULL, NULL);
            first_piola(d, F, S, Pq);
            for (int q = 0; q < d * d; ++q) P[q] += Pq[q] * wJ;
        }
    }
}

/* Stiffness transfer with the d^2 unit macro-gradient states G = e_k (x) e_L:
 * the micro response is D_G = G X + w_G with periodic w_G solving
 * K_ff w_G = -sum_e k_e (G X_e), and A_(G)(G') = D_G^T K D_G' / |K_delta|
 * (Sec. 3.2: T^T K T / |K_delta| with T built from unit displacement states).
 * r->K must hold the LDL^T factor of the tangent at the converged state. */
static int stiffness_transfer(rve_sys* r, const uint8_t* phase, const double* lame, const double* Fbar,
                              const double* w, double* A) {
    int d = r->d, n = r->n, nen = 1 << d, nd = nen * d, d2 = d * d;
    double h = 1.0 / n;
    double* rhs = (double*)calloc((size_t)d2 * r->nf, sizeof(double));
    double* wG = (double*)calloc((size_t)d2 * d * r->nn, sizeof(double));
    double ke[MAXNE * MAXD * MAXNE * MAXD];
    double uaff[9][MAXNE * MAXD];
    for (int G = 0; G < d2; ++G)
        for (int a = 0; a < nen; ++a) {
            int o[MAXD];
            local_offset(d, a, o);
            for (int i = 0; i < d; ++i) {
                double v = 0;
                for (int J = 0; J < d; ++J) v += ((G == i * d + J) ? 1.0 : 0.0) * o[J] * h;
                uaff[G][a * d + i] = v;
            }
        }
    for (int e = 0; e < r->ne; ++e) {
        int nodes[MAXNE];
        int st = oracle_element(d, n, phase, lame, e, Fbar, w, NULL, ke, NULL);
        if (st) { free(rhs); free(wG); return st; }
        element_nodes(d, n, e, nodes);
        for (int G = 0; G < d2; ++G)
            for (int q1 = 0; q1 < nd; ++q1) {
                int g1 = r->dof[nodes[q1 / d] * d + q1 % d];
                if (g1 < 0) continue;
                double s = 0;
                for (int q2 = 0; q2 < nd; ++q2) s += ke[q1 * nd + q2] * uaff[G][q2];
                rhs[(size_t)G * r->nf + g1] -= s;
            }
    }
    for (int G = 0; G < d2; ++G) {
        sky_solve(&r->K, rhs + (size_t)G * r->nf);
        for (int node = 0; node < r->nn; ++node)
            for (int k = 0; k < d; ++k) {
                int g = r->dof[node * d + k];
                wG[(size_t)G * d * r->nn + node * d + k] = g < 0 ? 0.0 : rhs[(size_t)G * r->nf + g];
            }
    }
    memset(A, 0, sizeof(double) * d2 * d2);
    for (int e = 0; e < r->ne; ++e) {
        int nodes[MAXNE];
        oracle_element(d, n, phase, lame, e, Fbar, w, NULL, ke, NULL);
        element_nodes(d, n, e, nodes);
        double De[9][MAXNE * MAXD];
        for (int G = 0; G < d2; ++G)
            for (int q = 0; q < nd; ++q)
                De[G][q] = uaff[G][q] + wG[(size_t)G * d * r->nn + nodes[q / d] * d + q % d];
        for (int G = 0; G < d2; ++G) {
            double kD[MAXNE * MAXD];
            for (int q1 = 0; q1 < nd; ++q1) {
                double s = 0;
                for (int q2 = 0; q2 < nd; ++q2) s += ke[q1 * nd + q2] * De[G][q2];
                kD[q1] = s;
            }
            for (int G2 = 0; G2 < d2; ++G2) {
                double s = 0;
                for (int q = 0; q < nd; ++q) s += De[G2][q] * kD[q];
                A[G2 * d2 + G] += s; /* |K_delta| = 1 */
            }
        }
    }
    free(rhs); free(wG);
    return ORC_OK;
}

static int all_finite(const double* x, int m) {
    for (int i = 0; i < m; ++i) if (!isfinite(x[i])) return 0;
    return 1;
}

static void fill_nan(double* x, int m) { for (int i = 0; i < m; ++i) x[i] = NAN; }

int oracle_rve_solve(int d, int n, const uint8_t* phase, const double* lame, const double* Fbar, double* w_io,
                     const oracle_opts* o, double* P, double* A, int* iters, double* res_hist) {
    int d2 = d * d;
    if (iters) *iters = 0;
    if (!all_finite(Fbar, d2) || !(det_d(d, Fbar) > 0)) {
        if (P) fill_nan(P, d2);
        if (A) fill_nan(A, d2 * d2);
        return all_finite(Fbar, d2) ? ORC_DETF : ORC_NONFINITE;
    }
    rve_sys r;
    if (rve_sys_init(&r, d, n)) return ORC_SINGULAR;
    int ndof = d * r.nn;
    double* w = (double*)calloc(ndof, sizeof(double));
    double* R = (double*)malloc(sizeof(double) * ndof);
    double* dw = (double*)malloc(sizeof(double) * (r.nf ? r.nf : 1));
    double* wt = (double*)malloc(sizeof(double) * ndof);
    if (w_io) memcpy(w, w_io, sizeof(double) * ndof);
    for (int i = 0; i < ndof; ++i)
        if (r.dof[i] < 0) w[i] = 0.0; /* pinned nodes */
    int status = ORC_OK, it = 0, restarted = 0;
    double r0 = 0;
    for (;;) {
        int st = rve_assemble(&r, phase, lame, Fbar, w, R, 1);
        if (st == ORC_DETF && it == 0 && w_io && !restarted) {
            /* a stored fluctuation that folds an element under the new Fbar is
             * discarded: restart from w = 0, where J = det Fbar > 0 */
            memset(w, 0, sizeof(double) * ndof);
            restarted = 1;
            continue;
        }
        if (st) { status = st; break; }
        double rn = norm_free(&r, R);
        if (!isfinite(rn)) { status = ORC_NONFINITE; break; }
        if (it == 0) r0 = rn;
        if (res_hist) res_hist[it] = rn;
        if (rn <= o->rtol * r0 + o->atol) break;
        if (it == o->max_iter) { status = ORC_NOCONV; break; }
        st = sky_ldlt(&r.K);
        if (st) { status = st; break; }
        for (int i = 0; i < ndof; ++i)
            if (r.dof[i] >= 0) dw[r.dof[i]] = -R[i];
        sky_solve(&r.K, dw);
        double alpha = 1.0;
        int ok = 0;
        for (int bt = 0; bt <= o->max_backtrack; ++bt) {
            memcpy(wt, w, sizeof(double) * ndof);
            for (int i = 0; i < ndof; ++i)
                if (r.dof[i] >= 0) wt[i] += alpha * dw[r.dof[i]];
            if (all_J_positive(&r, phase, lame, Fbar, wt)) { ok = 1; break; }
            alpha *= 0.5;
        }
        if (!ok) { status = ORC_DETF; break; }
        memcpy(w, wt, sizeof(double) * ndof);
        ++it;
    }
    if (iters) *iters = it;
    if (status == ORC_OK) {
        if (P) average_P(&r, phase, lame, Fbar, w, P);
        if (A && o->want_A) {
            int st = sky_ldlt(&r.K); /* tangent at the converged state */
            if (!st) st = stiffness_transfer(&r, phase, lame, Fbar, w, A);
            if (st) status = st;
        }
    }
    if (status != ORC_OK) {
        if (P) fill_nan(P, d2);
        if (A) fill_nan(A, d2 * d2);
    } else if (w_io) {
        memcpy(w_io, w, sizeof(double) * ndof);
    }
    free(w); free(R); free(dw); free(wt);
    rve_sys_free(&r);
    return status;
}

int oracle_rve_solve_batch(int d, int n, int64_t B, const uint8_t* phases, const double* lame, const double* F,
                           double* w, const oracle_opts* o, double* P, double* A, int32_t* status,
                           int32_t* iters, int nthreads) {
    int nn = ipow(n, d), d2 = d * d;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int nbad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nbad)
    for (int64_t b = 0; b < B; ++b) {
        int it = 0;
        int st = oracle_rve_solve(d, n, phases + b * nn, lame, F + b * d2, w ? w + b * d * nn : NULL, o,
                                  P ? P + b * d2 : NULL, A ? A + b * d2 * d2 : NULL, &it, NULL);
        if (status) status[b] = st;
        if (iters) iters[b] = it;
        nbad += st != 0;
    }
    return nbad;
}

/* ------------------------------------------------------------------ linear FE-HMM cell problems */
/* Small-strain elasticity C = lambda 1 (x) 1 + 2 mu I on the same periodic mesh:
 * for every unit engineering strain e_s the periodic fluctuation solves
 * K w_s = -sum_e int B_L^T C e_s, and C^h_rs = <(e_r + B_L w_r) . C (e_s + B_L w_s)>. */
int oracle_linear_homogenized(int d, int n, const uint8_t* phase, const double* lame, double* Chom) {
    rve_sys r;
    if (rve_sys_init(&r, d, n)) return ORC_SINGULAR;
    double dN[MAXNE][MAXNE][MAXD], wJ;
    const int npt = shape_grads(d, n, dN, &wJ);
    int nen = 1 << d, nd = nen * d, pr[MAXV][2];
    int nv = voigt_pairs(d, pr);
    double* rhs = (double*)calloc((size_t)nv * r.nf, sizeof(double));
    memset(r.K.val, 0, sizeof(double) * r.K.ptr[r.K.N]);
    /* per element: BL[p][v][q], C_lin[v][v] */
    for (int pass = 0; pass < 2; ++pass) {
        double Ch[MAXV][MAXV];
        memset(Ch, 0, sizeof(Ch));
        for (int e = 0; e < r.ne; ++e) {
            int nodes[MAXNE];
            element_nodes(d, n, e, nodes);
            double lam = lame[2 * phase[e]], mu = lame[2 * phase[e] + 1];
            double Cl[MAXV][MAXV];
            for (int a = 0; a < nv; ++a)
                for (int b = 0; b < nv; ++b) {
                    int na = pr[a][0] == pr[a][1], nb2 = pr[b][0] == pr[b][1];
                    Cl[a][b] = (na && nb2 ? lam : 0.0) + (a == b ? (na ? 2.0 * mu : mu) : 0.0);
                }
            for (int p = 0; p < npt; ++p) {
                double BL[MAXV][MAXNE * MAXD];
                for (int v = 0; v < nv; ++v) {
                    int I = pr[v][0], J = pr[v][1];
                    for (int a = 0; a < nen; ++a)
                        for (int k = 0; k < d; ++k) {
                            double val = (k == I ? dN[p][a][J] : 0.0);
                            if (I != J) val += (k == J ? dN[p][a][I] : 0.0);
                            BL[v][a * d + k] = val;
                        }
                }
                if (pass == 0) {
                    for (int q1 = 0; q1 < nd; ++q1) {
                        int g1 = r.dof[nodes[q1 / d] * d + q1 % d];
                        if (g1 < 0) continue;
                        for (int s = 0; s < nv; ++s) {
                            double t = 0;
                            for (int v = 0; v < nv; ++v) t += BL[v][q1] * Cl[v][s];
                            rhs[(size_t)s * r.nf + g1] -= t * wJ;
                        }
                        for (int q2 = 0; q2 <= q1; ++q2) {
                            int g2 = r.dof[nodes[q2 / d] * d + q2 % d];
                            if (g2 < 0) continue;
                            double t = 0;
                            for (int v = 0; v < nv; ++v)
                                for (int u = 0; u < nv; ++u) t += BL[v][q1] * Cl[v][u] * BL[u][q2];
                            sky_add(&r.K, g1, g2, t * wJ);
                        }
                    }
                } else {
                    double eps[MAXV][MAXV]; /* eps[s][v] = e_s + B_L w_s */
                    for (int s = 0; s < nv; ++s)
                        for (int v = 0; v < nv; ++v) {
                            double t = (s == v) ? 1.0 : 0.0;
                            for (int q = 0; q < nd; ++q) {
                                int g = r.dof[nodes[q / d] * d + q % d];
                                if (g >= 0) t += BL[v][q] * rhs[(size_t)s * r.nf + g];
                            }
                            eps[s][v] = t;
                        }
                    for (int s1 = 0; s1 < nv; ++s1)
                        for (int s2 = 0; s2 < nv; ++s2) {
                            double t = 0;
                            for (int v = 0; v < nv; ++v)
                                for (int u = 0; u < nv; ++u) t += eps[s1][v] * Cl[v][u] * eps[s2][u];
                            Ch[s1][s2] += t * wJ;
                        }
                }
            }
        }
        if (pass == 0) {
            int st = sky_ldlt(&r.K);
            if (st) { free(rhs); rve_sys_free(&r); return st; }
            for (int s = 0; s < nv; ++s) sky_solve(&r.K, rhs + (size_t)s * r.nf);
        } else {
            int d2 = d * d;
            for (int i = 0; i < d; ++i)
                for (int J = 0; J < d; ++J)
                    for (int k = 0; k < d; ++k)
                        for (int L = 0; L < d; ++L) {
                            int a = -1, b = -1;
                            for (int v = 0; v < nv; ++v) {
                                if ((pr[v][0] == i && pr[v][1] == J) || (pr[v][0] == J && pr[v][1] == i)) a = v;
                                if ((pr[v][0] == k && pr[v][1] == L) || (pr[v][0] == L && pr[v][1] == k)) b = v;
                            }
                            Chom[(i * d + J) * d2 + k * d + L] = Ch[a][b];
                        }
        }
    }
    free(rhs);
    rve_sys_free(&r);
    return ORC_OK;
}


/* The literal stiffness transfer of eqs. (k-mac-element-5..7): for each of
 * nstate prescribed linearized displacement states (eq. linearization-uH) --
 * a constant gradient G_j (d x d) plus a translation t_j (d) -- the micro
 * response D_j solves the linear constrained problem of
 * eq. (Lagrange-Functional-for-StiffnessTransfer) with the tangent K_T^h at the
 * micro state (Fbar, w): D_j = t_j + G_j X + w_j with the admissible fluctuation
 * w_j from K_ff w_j = -K_f(t_j + G_j X).  The output is the nstate x nstate
 * matrix T^T K T / |K_delta| with T = [D_1 ... D_nstate] and |K_delta| = 1,
 * computed element by element with the full element tangents (k_e annihilates
 * translations, so each element takes its affine part in local coordinates). */
int oracle_rve_transfer_states(int d, int n, const uint8_t* phase, const double* lame, const double* Fbar,
                               const double* w, int nstate, const double* G, const double* tvec, double* kT) {
    rve_sys r;
    if (rve_sys_init(&r, d, n)) return ORC_SINGULAR;
    int nen = 1 << d, nd = nen * d, ndof = d * r.nn;
    double h = 1.0 / n;
    double* R = (double*)malloc(sizeof(double) * ndof);
    double* rhs = (double*)calloc((size_t)nstate * (r.nf ? r.nf : 1), sizeof(double));
    double* wS = (double*)calloc((size_t)nstate * ndof, sizeof(double));
    double* Daff = (double*)malloc(sizeof(double) * (size_t)nstate * nd);
    double ke[MAXNE * MAXD * MAXNE * MAXD];
    int st = rve_assemble(&r, phase, lame, Fbar, w, R, 1);
    if (!st) st = sky_ldlt(&r.K);
    /* element-local affine part of every state */
    for (int j = 0; j < nstate && !st; ++j)
        for (int a = 0; a < nen; ++a) {
            int o[MAXD];
            local_offset(d, a, o);
            for (int i = 0; i < d; ++i) {
                double v = tvec ? tvec[j * d + i] : 0.0;
                for (int J = 0; J < d; ++J) v += G[(j * d + i) * d + J] * o[J] * h;
                Daff[j * nd + a * d + i] = v;
            }
        }
    for (int e = 0; e < r.ne && !st; ++e) {
        int nodes[MAXNE];
        st = oracle_element(d, n, phase, lame, e, Fbar, w, NULL, ke, NULL);
        element_nodes(d, n, e, nodes);
        for (int j = 0; j < nstate && !st; ++j)
            for (int q1 = 0; q1 < nd; ++q1) {
                int g1 = r.dof[nodes[q1 / d] * d + q1 % d];
                if (g1 < 0) continue;
                double v = 0;
                for (int q2 = 0; q2 < nd; ++q2) v += ke[q1 * nd + q2] * Daff[j * nd + q2];
                rhs[(size_t)j * r.nf + g1] -= v;
            }
    }
    for (int j = 0; j < nstate && !st; ++j) {
        sky_solve(&r.K, rhs + (size_t)j * r.nf);
        for (int i = 0; i < ndof; ++i)
            wS[(size_t)j * ndof + i] = r.dof[i] < 0 ? 0.0 : rhs[(size_t)j * r.nf + r.dof[i]];
    }
    if (!st) {
        memset(kT, 0, sizeof(double) * nstate * nstate);
        double* De = (double*)malloc(sizeof(double) * (size_t)nstate * nd);
        double* kD = (double*)malloc(sizeof(double) * nd);
        for (int e = 0; e < r.ne; ++e) {
            int nodes[MAXNE];
            oracle_element(d, n, phase, lame, e, Fbar, w, NULL, ke, NULL);
            element_nodes(d, n, e, nodes);
            for (int j = 0; j < nstate; ++j)
                for (int q = 0; q < nd; ++q)
                    De[j * nd + q] = Daff[j * nd + q] + wS[(size_t)j * ndof + nodes[q / d] * d + q % d];
            for (int k = 0; k < nstate; ++k) {
                for (int q1 = 0; q1 < nd; ++q1) {
                    double v = 0;
                    for (int q2 = 0; q2 < nd; ++q2) v += ke[q1 * nd + q2] * De[k * nd + q2];
                    kD[q1] = v;
                }
                for (int j = 0; j < nstate; ++j) {
                    double v = 0;
                    for (int q = 0; q < nd; ++q) v += De[j * nd + q] * kD[q];
                    kT[j * nstate + k] += v;
                }
            }
        }
        free(De);
        free(kD);
    }
    free(R); free(rhs); free(wS); free(Daff);
    rve_sys_free(&r);
    return st;
}

/* One micro Newton iteration for the alternating scheme (Algorithm 2, Sec. 5.2):
 * from the stored fluctuation w, one update D_{K,0} -> D_{K,1} (skipped when the
 * residual is already below atol), then stress and stiffness transfer at the
 * updated state.  rnorm receives ||R_f|| before the update. */
int oracle__rve_one_step(int d, int n, const uint8_t* phase, const double* lame, const double* Fbar, double* w_io,
                         const oracle_opts* o, double* P, double* A, double* rnorm) {
    int d2 = d * d;
    rve_sys r;
    if (rve_sys_init(&r, d, n)) return ORC_SINGULAR;
    int ndof = d * r.nn;
    double* R = (double*)malloc(sizeof(double) * ndof);
    double* dw = (double*)malloc(sizeof(double) * (r.nf ? r.nf : 1));
    double* wt = (double*)malloc(sizeof(double) * ndof);
    int status = rve_assemble(&r, phase, lame, Fbar, w_io, R, 1);
    if (status == ORC_DETF) {
        /* stored fluctuation infeasible under the new Fbar: restart from w = 0 */
        memset(w_io, 0, sizeof(double) * ndof);
        status = rve_assemble(&r, phase, lame, Fbar, w_io, R, 1);
    }
    double rn = status ? NAN : norm_free(&r, R);
    if (rnorm) *rnorm = rn;
    if (!status && rn > o->atol) {
        status = sky_ldlt(&r.K);
        if (!status) {
            for (int i = 0; i < ndof; ++i)
                if (r.dof[i] >= 0) dw[r.dof[i]] = -R[i];
            sky_solve(&r.K, dw);
            double alpha = 1.0;
            int ok = 0;
            for (int bt = 0; bt <= o->max_backtrack; ++bt) {
                memcpy(wt, w_io, sizeof(double) * ndof);
                for (int i = 0; i < ndof; ++i)
                    if (r.dof[i] >= 0) wt[i] += alpha * dw[r.dof[i]];
                if (all_J_positive(&r, phase, lame, Fbar, wt)) { ok = 1; break; }
                alpha *= 0.5;
            }
            if (!ok) status = ORC_DETF;
            else memcpy(w_io, wt, sizeof(double) * ndof);
        }
        if (!status) status = rve_assemble(&r, phase, lame, Fbar, w_io, R, 1);
    }
    if (!status) {
        average_P(&r, phase, lame, Fbar, w_io, P);
        status = sky_ldlt(&r.K);
        if (!status) status = stiffness_transfer(&r, phase, lame, Fbar, w_io, A);
    }
    if (status) { fill_nan(P, d2); fill_nan(A, d2 * d2); }
    free(R); free(dw); free(wt);
    rve_sys_free(&r);
    return status;
}

/* Test hook: free residual R_f, dense free-free tangent K_ff (both in natural
 * dof order: node-major, pinned nodes excluded) and the Newton step dw = -K_ff^-1 R_f
 * computed by the skyline LDL^T.  Small meshes only (K_ff is dense). */
int oracle_debug_system(int d, int n, const uint8_t* phase, const double* lame, const double* Fbar, const double* w,
                        double* Rf, double* Kff, double* dw) {
    rve_sys r;
    if (rve_sys_init(&r, d, n)) return ORC_SINGULAR;
    int ndof = d * r.nn, nf = r.nf;
    double* R = (double*)malloc(sizeof(double) * ndof);
    int* nat = (int*)malloc(sizeof(int) * ndof); /* natural index among the free dofs */
    for (int a = 0, q = 0; a < ndof; ++a) nat[a] = r.dof[a] >= 0 ? q++ : -1;
    int st = rve_assemble(&r, phase, lame, Fbar, w, R, 1);
    if (!st) {
        for (int a = 0; a < ndof; ++a) {
            if (nat[a] < 0) continue;
            Rf[nat[a]] = R[a];
            for (int b = 0; b < ndof; ++b) {
                if (nat[b] < 0) continue;
                int ga = r.dof[a], gb = r.dof[b];
                int i = ga > gb ? ga : gb, j = ga > gb ? gb : ga;
                double v = 0;
                if (j >= r.K.fc[i]) v = r.K.val[r.K.ptr[i] + (j - r.K.fc[i])];
                Kff[(size_t)nat[a] * nf + nat[b]] = v;
            }
        }
        st = sky_ldlt(&r.K);
        if (!st) {
            double* x = (double*)malloc(sizeof(double) * (nf ? nf : 1));
            for (int a = 0; a < ndof; ++a) if (nat[a] >= 0) x[r.dof[a]] = -R[a];
            sky_solve(&r.K, x);
            for (int a = 0; a < ndof; ++a) if (nat[a] >= 0) dw[nat[a]] = x[r.dof[a]];
            free(x);
        }
    }
    free(nat);
    free(R);
    rve_sys_free(&r);
    return st;
}
