// mesh_common.h -- numbering of the structured periodic grid (host and device).
//
// Node (i,j[,k]) -> i + n j [+ n^2 k] (indices mod n).  Element (i,j[,k]) has the
// same id; its local node a sits at offset o(a) in {0,1}^d: counter-clockwise
// (0,0),(1,0),(1,1),(0,1) in 2D, that square at z = 0 then at z = 1 in 3D.
#pragma once

#if defined(__HIPCC__)
#define FEHMM_HD __host__ __device__ inline
#else
#define FEHMM_HD inline
#endif

namespace fehmm {

FEHMM_HD void local_offset(int d, int a, int* o) {
    o[0] = ((a & 3) == 1 || (a & 3) == 2) ? 1 : 0;
    o[1] = ((a & 3) >= 2) ? 1 : 0;
    if (d == 3) o[2] = a >> 2;
}

FEHMM_HD void element_nodes(int d, int n, int e, int* nodes) {
    int c[3] = {0, 0, 0}, t = e;
    for (int k = 0; k < d; ++k) { c[k] = t % n; t /= n; }
    for (int a = 0; a < (1 << d); ++a) {
        int o[3] = {0, 0, 0};
        local_offset(d, a, o);
        int id = 0, s = 1;
        for (int k = 0; k < d; ++k) { id += ((c[k] + o[k]) % n) * s; s *= n; }
        nodes[a] = id;
    }
}

// the element in which node v is local node a
FEHMM_HD int element_of_node(int d, int n, int v, int a) {
    int o[3] = {0, 0, 0};
    local_offset(d, a, o);
    int id = 0, s = 1, t = v;
    for (int k = 0; k < d; ++k) {
        int c = t % n;
        t /= n;
        id += ((c - o[k] + n) % n) * s;
        s *= n;
    }
    return id;
}

// the nodes whose fluctuation is held at zero: node 0 under periodic coupling
// (bc 0); under linear displacements (bc 1, KUBC) the boundary, i.e. on the n^d
// numbering every node with some grid index 0 (the faces x_k = 1 wrap onto them)
FEHMM_HD bool plan_pinned(int bc, int d, int n, int v) {
    if (bc == 0) return v == 0;
    for (int k = 0; k < d; ++k) {
        if (v % n == 0) return true;
        v /= n;
    }
    return false;
}

}  // namespace fehmm
