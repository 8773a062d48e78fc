/*
 * macro.c -- FP64 CPU oracle of the macro level of the FE-HMM (test
 * infrastructure only).
 *
 * Macro Q1 quadrilaterals with 2x2 Gauss points on a rectangle (optionally with
 * a centred hole, elements removed by centroid).  At every quadrature point the
 * macro displacement is linearized (eq. linearization-uH), so the RVE is driven
 * by Fbar = I + grad u^H(x_qp).  Internal forces use S^H = <F>^-1 <P>
 * (eq. macro-mean-stress) through f_I = int B_I^T S^H = int (Fbar S^H) . grad N_I,
 * i.e. <P> . grad N_I; the tangent is the stiffness transfer
 * sum_l omega_l / |K_delta| T^T K T of eq. (k-mac-element-6), which for the
 * unit displacement states of a macro node (gradients e_i (x) grad N_I) is
 * B_mac^T Abar B_mac with Abar the RVE transfer of the unit gradient states.
 * Solution algorithms of Sec. 5: nested (Algorithm 1: full micro Newton per macro
 * iteration, warm-started from the stored fluctuations) and alternating
 * (Algorithm 2: one micro Newton iteration per macro iteration).
 */
#include "oracle.h"
#include "sparse.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

int oracle__rve_one_step(int d, int n, const uint8_t* phase, const double* lame, const double* Fbar, double* w,
                         const oracle_opts* o, double* P, double* A, double* rnorm);
int oracle_rve_transfer_states(int d, int n, const uint8_t* phase, const double* lame, const double* Fbar,
                               const double* w, int nstate, const double* G, const double* tvec, double* kT);

struct oracle_macro {
    oracle_macro_desc desc;
    oracle_opts micro;
    int nnode, nelem, ndof, nqp, nfree, nw;
    double* xy;       /* [nnode][2] */
    int* conn;        /* [nelem][4] */
    int* fixed;       /* [ndof] 1 if Dirichlet */
    int* dofmap;      /* [ndof] -> free index or -1 */
    double* u;        /* [ndof] */
    double* wq;       /* [nqp][nw] micro fluctuations */
    double* Fq; double* Pq; double* Aq;
    int npt;              /* quadrature points per grid cell: 4 (Q1) or 2 (P1 triangles) */
    double dN[4][4][2];   /* [gp][node][dir] for the (uniform) element size */
    double Nv[4][4];      /* shape values [gp][node] */
    double wdet;
    skyline K;
};

/* Q1: 2x2 Gauss points.  P1: the cell's triangles (0,1,2) and (0,2,3) in its
 * counter-clockwise node order, one point each at the centroid (linear shape
 * functions: constant gradients, value 1/3 at the centroid), weight hx hy / 2. */
static int macro_points(int elem, double hx, double hy, double dN[4][4][2], double Nv[4][4], double* wdet) {
    static const int sx[4] = {-1, 1, 1, -1}, sy[4] = {-1, -1, 1, 1};
    memset(dN, 0, sizeof(double) * 32);
    memset(Nv, 0, sizeof(double) * 16);
    if (elem == 1) {
        /* triangle 0: (0,0) (hx,0) (hx,hy); triangle 1: (0,0) (hx,hy) (0,hy) */
        dN[0][0][0] = -1.0 / hx;                         dN[0][1][0] = 1.0 / hx; dN[0][1][1] = -1.0 / hy;
        dN[0][2][1] = 1.0 / hy;
        dN[1][0][1] = -1.0 / hy; dN[1][2][0] = 1.0 / hx; dN[1][3][0] = -1.0 / hx; dN[1][3][1] = 1.0 / hy;
        Nv[0][0] = Nv[0][1] = Nv[0][2] = 1.0 / 3.0;
        Nv[1][0] = Nv[1][2] = Nv[1][3] = 1.0 / 3.0;
        *wdet = 0.5 * hx * hy;
        return 2;
    }
    double g = 1.0 / sqrt(3.0);
    for (int p = 0; p < 4; ++p) {
        double xi = sx[p] * g, eta = sy[p] * g;
        for (int a = 0; a < 4; ++a) {
            dN[p][a][0] = 0.25 * sx[a] * (1 + sy[a] * eta) * 2.0 / hx;
            dN[p][a][1] = 0.25 * sy[a] * (1 + sx[a] * xi) * 2.0 / hy;
            Nv[p][a] = 0.25 * (1 + sx[a] * xi) * (1 + sy[a] * eta);
        }
    }
    *wdet = 0.25 * hx * hy;
    return 4;
}

oracle_macro* oracle_macro_create(const oracle_macro_desc* d, const oracle_opts* micro) {
    oracle_macro* m = (oracle_macro*)calloc(1, sizeof(oracle_macro));
    m->desc = *d;
    m->micro = *micro;
    int nx = d->nx, ny = d->ny;
    double hx = d->Lx / nx, hy = d->Ly / ny;
    m->npt = macro_points(d->elem, hx, hy, m->dN, m->Nv, &m->wdet);
    int* keep = (int*)malloc(sizeof(int) * nx * ny);
    int* used = (int*)calloc((nx + 1) * (ny + 1), sizeof(int));
    m->nelem = 0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double cx = (i + 0.5) * hx - 0.5 * d->Lx, cy = (j + 0.5) * hy - 0.5 * d->Ly;
            int k = !(d->hole_r > 0 && sqrt(cx * cx + cy * cy) < d->hole_r);
            keep[j * nx + i] = k;
            if (k) {
                m->nelem++;
                used[j * (nx + 1) + i] = used[j * (nx + 1) + i + 1] = 1;
                used[(j + 1) * (nx + 1) + i] = used[(j + 1) * (nx + 1) + i + 1] = 1;
            }
        }
    int* id = (int*)malloc(sizeof(int) * (nx + 1) * (ny + 1));
    m->nnode = 0;
    for (int k = 0; k < (nx + 1) * (ny + 1); ++k) id[k] = used[k] ? m->nnode++ : -1;
    m->xy = (double*)malloc(sizeof(double) * 2 * m->nnode);
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i)
            if (id[j * (nx + 1) + i] >= 0) {
                m->xy[2 * id[j * (nx + 1) + i]] = i * hx;
                m->xy[2 * id[j * (nx + 1) + i] + 1] = j * hy;
            }
    m->conn = (int*)malloc(sizeof(int) * 4 * m->nelem);
    int e = 0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            if (keep[j * nx + i]) {
                m->conn[4 * e + 0] = id[j * (nx + 1) + i];
                m->conn[4 * e + 1] = id[j * (nx + 1) + i + 1];
                m->conn[4 * e + 2] = id[(j + 1) * (nx + 1) + i + 1];
                m->conn[4 * e + 3] = id[(j + 1) * (nx + 1) + i];
                ++e;
            }
    m->ndof = 2 * m->nnode;
    m->fixed = (int*)calloc(m->ndof, sizeof(int));
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            int v = id[j * (nx + 1) + i];
            if (v < 0) continue;
            if (i == 0) {
                m->fixed[2 * v] = 1;
                if (d->bc == 0 || j == 0) m->fixed[2 * v + 1] = 1;
            }
            if (i == nx) m->fixed[2 * v] = 1;
        }
    m->dofmap = (int*)malloc(sizeof(int) * m->ndof);
    /* free dofs numbered node by node in RCM order of the node graph */
    int nv = m->nnode;
    int* xadj = (int*)calloc(nv + 1, sizeof(int));
    int* adj = (int*)malloc(sizeof(int) * nv * 8);
    int* cnt = (int*)calloc(nv, sizeof(int));
    for (int q = 0; q < m->nelem; ++q)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                if (a == b) continue;
                int va = m->conn[4 * q + a], vb = m->conn[4 * q + b], dup = 0;
                for (int k = 0; k < cnt[va]; ++k) if (adj[va * 8 + k] == vb) dup = 1;
                if (!dup) adj[va * 8 + cnt[va]++] = vb;
            }
    int* adjc = (int*)calloc((size_t)nv * 8 + 1, sizeof(int));
    int tot = 0;
    for (int v = 0; v < nv; ++v) { xadj[v] = tot; for (int k = 0; k < cnt[v]; ++k) adjc[tot++] = adj[v * 8 + k]; }
    xadj[nv] = tot;
    int* perm = (int*)malloc(sizeof(int) * nv);
    rcm(nv, xadj, adjc, perm);
    int* pos = (int*)malloc(sizeof(int) * nv);
    for (int k = 0; k < nv; ++k) pos[perm[k]] = k;
    /* free index = order of (pos, component) among free dofs */
    m->nfree = 0;
    for (int k = 0; k < nv; ++k) {
        int v = perm[k];
        for (int c = 0; c < 2; ++c) m->dofmap[2 * v + c] = m->fixed[2 * v + c] ? -1 : m->nfree++;
    }
    int* fc = (int*)malloc(sizeof(int) * (m->nfree ? m->nfree : 1));
    for (int v = 0; v < nv; ++v)
        for (int c = 0; c < 2; ++c) {
            int g = m->dofmap[2 * v + c];
            if (g < 0) continue;
            int mn = g;
            for (int k = xadj[v]; k <= xadj[v + 1]; ++k) {
                int nb = (k < xadj[v + 1]) ? adjc[k] : v;
                for (int c2 = 0; c2 < 2; ++c2) {
                    int g2 = m->dofmap[2 * nb + c2];
                    if (g2 >= 0 && g2 < mn) mn = g2;
                }
            }
            fc[g] = mn;
        }
    sky_alloc(&m->K, m->nfree, fc);
    free(fc); free(pos); free(perm); free(adjc); free(cnt); free(adj); free(xadj);
    free(id); free(used); free(keep);
    m->u = (double*)calloc(m->ndof, sizeof(double));
    m->nqp = m->npt * m->nelem;
    m->nw = 2 * d->n * d->n;
    m->wq = (double*)calloc((size_t)m->nqp * m->nw, sizeof(double));
    m->Fq = (double*)calloc((size_t)m->nqp * 4, sizeof(double));
    m->Pq = (double*)calloc((size_t)m->nqp * 4, sizeof(double));
    m->Aq = (double*)calloc((size_t)m->nqp * 16, sizeof(double));
    return m;
}

void oracle_macro_destroy(oracle_macro* m) {
    if (!m) return;
    free(m->xy); free(m->conn); free(m->fixed); free(m->dofmap); free(m->u); free(m->wq);
    free(m->Fq); free(m->Pq); free(m->Aq);
    sky_free(&m->K);
    free(m);
}

int oracle_macro_ndof(const oracle_macro* m) { return m->ndof; }
int oracle_macro_nqp(const oracle_macro* m) { return m->nqp; }
void oracle_macro_get_u(const oracle_macro* m, double* u) { memcpy(u, m->u, sizeof(double) * m->ndof); }
void oracle_macro_get_nodes(const oracle_macro* m, double* xy) { memcpy(xy, m->xy, sizeof(double) * 2 * m->nnode); }
void oracle_macro_get_qp(const oracle_macro* m, double* F, double* P, double* A) {
    if (F) memcpy(F, m->Fq, sizeof(double) * 4 * m->nqp);
    if (P) memcpy(P, m->Pq, sizeof(double) * 4 * m->nqp);
    if (A) memcpy(A, m->Aq, sizeof(double) * 16 * m->nqp);
}

static void macro_gather_F(oracle_macro* m) {
    for (int e = 0; e < m->nelem; ++e)
        for (int p = 0; p < m->npt; ++p) {
            double* F = m->Fq + 4 * (m->npt * e + p);
            F[0] = 1; F[1] = 0; F[2] = 0; F[3] = 1;
            for (int a = 0; a < 4; ++a) {
                int v = m->conn[4 * e + a];
                for (int i = 0; i < 2; ++i)
                    for (int J = 0; J < 2; ++J) F[i * 2 + J] += m->u[2 * v + i] * m->dN[p][a][J];
            }
        }
}

/* runs the micro problems of every quadrature point; returns #failed */
static int macro_micro(oracle_macro* m, int one_step, int64_t* micro_iters) {
    int nbad = 0;
    int64_t its = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nbad, its)
    for (int q = 0; q < m->nqp; ++q) {
        double* w = m->wq + (size_t)q * m->nw;
        int st, it = 1;
        if (one_step) {
            double rn;
            st = oracle__rve_one_step(2, m->desc.n, m->desc.phase, m->desc.lame, m->Fq + 4 * q, w, &m->micro,
                                      m->Pq + 4 * q, m->Aq + 16 * q, &rn);
        } else {
            st = oracle_rve_solve(2, m->desc.n, m->desc.phase, m->desc.lame, m->Fq + 4 * q, w, &m->micro,
                                  m->Pq + 4 * q, m->Aq + 16 * q, &it, NULL);
        }
        nbad += st != 0;
        its += it;
    }
    *micro_iters += its;
    return nbad;
}

/* R_H (free dofs) and K_H; with dud (first iteration of a load step) also the
 * prescribed increment's pull on the free dofs, R_f += K_fd dud */
static double macro_assemble(oracle_macro* m, double* R, const double* dud) {
    memset(R, 0, sizeof(double) * (m->nfree ? m->nfree : 1));
    memset(m->K.val, 0, sizeof(double) * m->K.ptr[m->K.N]);
    for (int e = 0; e < m->nelem; ++e)
        for (int p = 0; p < m->npt; ++p) {
            const double* P = m->Pq + 4 * (m->npt * e + p);
            const double* A = m->Aq + 16 * (m->npt * e + p);
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 2; ++i) {
                    int g = m->dofmap[2 * m->conn[4 * e + a] + i];
                    if (g < 0) continue;
                    double s = 0;
                    for (int J = 0; J < 2; ++J) s += P[i * 2 + J] * m->dN[p][a][J];
                    R[g] += s * m->wdet;
                    for (int b = 0; b < 4; ++b)
                        for (int k = 0; k < 2; ++k) {
                            int g2 = m->dofmap[2 * m->conn[4 * e + b] + k];
                            if (g2 < 0 && dud) {
                                double t = 0;
                                for (int J = 0; J < 2; ++J)
                                    for (int L = 0; L < 2; ++L)
                                        t += m->dN[p][a][J] * A[(i * 2 + J) * 4 + k * 2 + L] * m->dN[p][b][L];
                                R[g] += t * m->wdet * dud[2 * m->conn[4 * e + b] + k];
                                continue;
                            }
                            if (g2 < 0 || g2 > g) continue;
                            double t = 0;
                            for (int J = 0; J < 2; ++J)
                                for (int L = 0; L < 2; ++L)
                                    t += m->dN[p][a][J] * A[(i * 2 + J) * 4 + k * 2 + L] * m->dN[p][b][L];
                            sky_add(&m->K, g, g2, t * m->wdet);
                        }
                }
        }
    double s = 0;
    for (int g = 0; g < m->nfree; ++g) s += R[g] * R[g];
    return sqrt(s);
}

int oracle_macro_step(oracle_macro* m, int step, int* macro_iters, double* res_hist, int64_t* micro_iters) {
    const oracle_macro_desc* d = &m->desc;
    /* the prescribed displacements of the step enter the first macro Newton
     * iteration as an inhomogeneous Dirichlet condition of the linearized
     * system: K_ff du_f = -(R_f + K_fd dud), u_d += dud; the first residual of
     * the step is that load-equivalent residual */
    double ux = (d->stretch - 1.0) * d->Lx * (double)step / d->nsteps;
    double* dud = (double*)calloc(m->ndof, sizeof(double));
    for (int v = 0; v < m->nnode; ++v) {
        if (m->fixed[2 * v]) dud[2 * v] = ((m->xy[2 * v] > 0.5 * d->Lx) ? ux : 0.0) - m->u[2 * v];
        if (m->fixed[2 * v + 1]) dud[2 * v + 1] = 0.0 - m->u[2 * v + 1];
    }
    double* R = (double*)malloc(sizeof(double) * (m->nfree ? m->nfree : 1));
    int64_t mic = 0;
    double r0 = 0;
    int it = 0, status = 0;
    for (;;) {
        macro_gather_F(m);
        if (macro_micro(m, d->scheme == 1, &mic)) { status = 2; break; }
        double rn = macro_assemble(m, R, it == 0 ? dud : NULL);
        if (it == 0) r0 = rn;
        if (res_hist) res_hist[it] = r0 > 0 ? rn / r0 : 0.0;
        if (rn <= d->rtol_macro * r0 || rn == 0.0) break;
        if (it == d->max_macro_iter) { status = 1; break; }
        if (sky_ldlt(&m->K)) { status = 2; break; }
        for (int g = 0; g < m->nfree; ++g) R[g] = -R[g];
        sky_solve(&m->K, R);
        for (int k = 0; k < m->ndof; ++k) {
            if (m->dofmap[k] >= 0) m->u[k] += R[m->dofmap[k]];
            else if (it == 0) m->u[k] += dud[k];
        }
        ++it;
    }
    free(R);
    free(dud);
    if (macro_iters) *macro_iters = it;
    if (micro_iters) *micro_iters = mic;
    return status;
}

/* Macro element stiffness of element (grid cell) e at the stored micro states,
 * two ways.  Literal (eqs. k-mac-element-5..7): at each quadrature point the 4 x 2 unit nodal
 * displacement states (I, x_i) of the element, linearized at the point
 * (eq. linearization-uH: translation N_I(x_qp) e_i, gradient e_i (x) grad N_I),
 * drive the micro problem; k = sum_qp omega_qp T^T K T / |K_delta|.
 * Condensed: k = sum_qp omega_qp B^T Abar B with the stored Abar of the point.
 * Both [8][8] in the element's (node, direction) order. */
int oracle_macro_element_stiffness(const oracle_macro* m, int e, int literal, double* k) {
    if (e < 0 || e >= m->nelem) return -1;
    memset(k, 0, sizeof(double) * 64);
    for (int p = 0; p < m->npt; ++p) {
        const int q = m->npt * e + p;
        if (literal) {
            double G[8 * 4], t[8 * 2], kT[64];
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 2; ++i) {
                    const int j = 2 * a + i;
                    for (int c = 0; c < 4; ++c) G[j * 4 + c] = 0.0;
                    for (int J = 0; J < 2; ++J) G[j * 4 + i * 2 + J] = m->dN[p][a][J];
                    t[j * 2 + 0] = i == 0 ? m->Nv[p][a] : 0.0;
                    t[j * 2 + 1] = i == 1 ? m->Nv[p][a] : 0.0;
                }
            int st = oracle_rve_transfer_states(2, m->desc.n, m->desc.phase, m->desc.lame, m->Fq + 4 * q,
                                                m->wq + (size_t)q * m->nw, 8, G, t, kT);
            if (st) return st;
            for (int c = 0; c < 64; ++c) k[c] += kT[c] * m->wdet;
        } else {
            const double* A = m->Aq + 16 * q;
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 2; ++i)
                    for (int b = 0; b < 4; ++b)
                        for (int kk = 0; kk < 2; ++kk) {
                            double v = 0;
                            for (int J = 0; J < 2; ++J)
                                for (int L = 0; L < 2; ++L)
                                    v += m->dN[p][a][J] * A[(i * 2 + J) * 4 + kk * 2 + L] * m->dN[p][b][L];
                            k[(2 * a + i) * 8 + 2 * b + kk] += v * m->wdet;
                        }
        }
    }
    return 0;
}

int oracle_macro_nelem(const oracle_macro* m) { return m->nelem; }
void oracle_macro_get_conn(const oracle_macro* m, int* conn) { memcpy(conn, m->conn, sizeof(int) * 4 * m->nelem); }
void oracle_macro_get_state(const oracle_macro* m, double* w) {
    memcpy(w, m->wq, sizeof(double) * (size_t)m->nqp * m->nw);
}
void oracle_macro_set_qp(oracle_macro* m, const double* F, const double* P, const double* A, const double* w) {
    if (F) memcpy(m->Fq, F, sizeof(double) * 4 * m->nqp);
    if (P) memcpy(m->Pq, P, sizeof(double) * 4 * m->nqp);
    if (A) memcpy(m->Aq, A, sizeof(double) * 16 * m->nqp);
    if (w) memcpy(m->wq, w, sizeof(double) * (size_t)m->nqp * m->nw);
}
