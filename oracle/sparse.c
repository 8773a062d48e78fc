/*
 * sparse.c -- the oracle's own sparse direct solver (test infrastructure only).
 * Profile (skyline) storage, reverse Cuthill-McKee ordering and an in-place
 * LDL^T (Crout) factorization with forward/diagonal/backward substitution.
 * The paper does not name its linear solver (Sec. 3.3 only states the
 * linearized system); any exact direct method serves.
 */
#include "sparse.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ profile (skyline) LDL^T */
/* Symmetric matrix of order N in skyline form: row i stores columns fc[i]..i at
 * val[ptr[i] + (j - fc[i])].  The oracle's own sparse direct solver: reverse
 * Cuthill-McKee keeps the profile small; LDL^T is computed in place (Crout). */

void sky_free(skyline* s) {
    free(s->fc); free(s->ptr); free(s->val); free(s->D);
    memset(s, 0, sizeof(*s));
}

int sky_alloc(skyline* s, int N, const int* fc) {
    s->N = N;
    s->fc = (int*)malloc(sizeof(int) * (N ? N : 1));
    s->ptr = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
    s->D = (double*)malloc(sizeof(double) * (N ? N : 1));
    int64_t tot = 0;
    for (int i = 0; i < N; ++i) { s->fc[i] = fc[i]; s->ptr[i] = tot; tot += i - fc[i] + 1; }
    s->ptr[N] = tot;
    s->val = (double*)calloc((size_t)(tot ? tot : 1), sizeof(double));
    return s->val ? 0 : -1;
}

static double* sky_at(skyline* s, int i, int j) { /* requires fc[i] <= j <= i */
    return &s->val[s->ptr[i] + (j - s->fc[i])];
}

void sky_add(skyline* s, int i, int j, double v) {
    if (i < j) { int t = i; i = j; j = t; }
    *sky_at(s, i, j) += v;
}

/* returns 0, or 3 (singular) when a pivot vanishes relative to its diagonal
 * entry (|D_i| <= 1e-14 |K_ii|) or is not finite; negative pivots are kept
 * (symmetric indefinite tangents occur past micro-instabilities). */
int sky_ldlt(skyline* s) {
    int N = s->N;
    for (int i = 0; i < N; ++i) {
        int fi = s->fc[i];
        double* ri = &s->val[s->ptr[i]] - fi; /* ri[j] valid for fi <= j <= i */
        for (int j = fi; j < i; ++j) {
            int fj = s->fc[j];
            double* rj = &s->val[s->ptr[j]] - fj;
            int k0 = fi > fj ? fi : fj;
            double g = ri[j];
            for (int k = k0; k < j; ++k) g -= ri[k] * rj[k];
            ri[j] = g; /* g_ij = L_ij D_j */
        }
        double dii = ri[i], aii = fabs(ri[i]);
        for (int j = fi; j < i; ++j) {
            double l = ri[j] / s->D[j];
            dii -= ri[j] * l;
            ri[j] = l;
        }
        if (!(fabs(dii) > 1e-14 * aii) || !isfinite(dii)) return 3;
        s->D[i] = dii;
        ri[i] = 1.0;
    }
    return 0;
}

void sky_solve(const skyline* s, double* x) {
    int N = s->N;
    for (int i = 0; i < N; ++i) {
        int fi = s->fc[i];
        const double* ri = &s->val[s->ptr[i]] - fi;
        double v = x[i];
        for (int j = fi; j < i; ++j) v -= ri[j] * x[j];
        x[i] = v;
    }
    for (int i = 0; i < N; ++i) x[i] /= s->D[i];
    for (int i = N - 1; i >= 0; --i) {
        int fi = s->fc[i];
        const double* ri = &s->val[s->ptr[i]] - fi;
        double v = x[i];
        for (int j = fi; j < i; ++j) x[j] -= ri[j] * v;
    }
}

/* Reverse Cuthill-McKee of a graph in CSR form (adjacency without self loops).
 * perm[k] = vertex placed at position k. */
void rcm(int nv, const int* xadj, const int* adj, int* perm) {
    int* deg = (int*)malloc(sizeof(int) * nv);
    char* seen = (char*)calloc(nv, 1);
    int* q = (int*)malloc(sizeof(int) * nv);
    for (int v = 0; v < nv; ++v) deg[v] = xadj[v + 1] - xadj[v];
    int filled = 0;
    while (filled < nv) {
        /* start: unvisited vertex of minimum degree, then one BFS sweep to a far vertex */
        int start = -1;
        for (int v = 0; v < nv; ++v)
            if (!seen[v] && (start < 0 || deg[v] < deg[start])) start = v;
        for (int sweep = 0; sweep < 2; ++sweep) {
            char* s2 = (char*)calloc(nv, 1);
            int h = 0, t = 0;
            q[t++] = start; s2[start] = 1;
            int last = start;
            while (h < t) {
                int v = q[h++]; last = v;
                for (int k = xadj[v]; k < xadj[v + 1]; ++k)
                    if (!s2[adj[k]] && !seen[adj[k]]) { s2[adj[k]] = 1; q[t++] = adj[k]; }
            }
            free(s2);
            start = last;
        }
        int h = filled, t = filled;
        perm[t++] = start; seen[start] = 1;
        while (h < t) {
            int v = perm[h++];
            int b = t;
            for (int k = xadj[v]; k < xadj[v + 1]; ++k)
                if (!seen[adj[k]]) { seen[adj[k]] = 1; perm[t++] = adj[k]; }
            /* neighbours in increasing degree (insertion sort) */
            for (int i = b + 1; i < t; ++i) {
                int x = perm[i], j = i - 1;
                while (j >= b && deg[perm[j]] > deg[x]) { perm[j + 1] = perm[j]; --j; }
                perm[j + 1] = x;
            }
        }
        filled = t;
    }
    for (int i = 0; i < nv / 2; ++i) { int x = perm[i]; perm[i] = perm[nv - 1 - i]; perm[nv - 1 - i] = x; }
    free(deg); free(seen); free(q);
}

