/* sparse.h -- oracle-internal skyline LDL^T and RCM (test infrastructure only). */
#ifndef FEHMM_ORACLE_SPARSE_H
#define FEHMM_ORACLE_SPARSE_H
#include <stdint.h>

/* Symmetric matrix of order N: row i stores columns fc[i]..i at val[ptr[i] + (j - fc[i])]. */
typedef struct {
    int N;
    int* fc;
    int64_t* ptr;
    double* val;
    double* D;
} skyline;

int sky_alloc(skyline* s, int N, const int* fc);
void sky_free(skyline* s);
void sky_add(skyline* s, int i, int j, double v);   /* requires fc[max(i,j)] <= min(i,j) */
int sky_ldlt(skyline* s);                            /* 0, or 3 (singular: pivot <= 0 or not finite) */
void sky_solve(const skyline* s, double* x);         /* x <- K^{-1} x using the factor */
void rcm(int nv, const int* xadj, const int* adj, int* perm); /* perm[k] = vertex at position k */

#endif
