// plan.h -- symbolic factorization plan of the periodic RVE stiffness matrix.
//
// The sparsity of the free-free tangent K_ff depends only on (d, n): every node
// couples to its 3^d periodic neighbours and node 0 is pinned.  One plan per
// (d, n) therefore serves every RVE of that size.  The plan holds a geometric
// nested-dissection ordering of the periodic grid (two parallel planes cut a
// periodic direction, one plane cuts an open one), the supernodal elimination
// tree with one dense front per separator / leaf box, the maps that assemble
// element matrices and children's update matrices into each front, and the
// per-slot workspace layout of the batched multifrontal LDL^T.
#pragma once
#include <cstdint>
#include <vector>

namespace fehmm {

constexpr int kMaxNrhs = 10;  // the Newton residual beside the d^2 columns of the condensation (3D)

struct FrontHost {
    int m = 0, p = 0;           // dofs in the front, pivot dofs (leading)
    int parent = -1;
    int64_t rows_off = 0;       // into rows[]: m global dof ids (node*d + comp)
    int64_t relind_off = 0;     // into relind[]: (m-p) positions in the parent front
    int64_t L_off = 0;          // panel m x p, column-major, leading dimension m
    int64_t D_off = 0;          // p pivots
    int64_t y_off = 0;          // p x kMaxNrhs forward-substituted right-hand sides
    int64_t U_off = 0;          // update matrix (m-p)^2 + (m-p)*kMaxNrhs on the stack
    int child_begin = 0, child_end = 0;  // into children[]
    int kmap_begin = 0, kmap_end = 0;    // into kpair[]
    int asm_begin = 0, asm_end = 0;      // into asm_rc[] (lower-triangle targets of original entries)
    int64_t ea_off = 0;                  // into ea_dst[]: this front's packed update entries -> packed parent offsets
    int wave = 0;                        // 1: small front (m <= 64, subtree small) processed by one wave
    int height = 0;                      // 0 for leaves, 1 + max over children
};

// original-matrix block K(b, a) of a pivot node a: d x d block at front rows of
// node b (row_node) and pivot node a (col_node), sum over contributions
struct KPair {
    int32_t row_node;  // front-local node index of b (row block = row_node*d)
    int32_t col_node;  // front-local node index of a (< p/d)
    int32_t c_begin, c_count;  // into kcontrib[]
};

struct KContrib {
    int32_t elem;      // element id
    int32_t la, lb;    // local node numbers of a and b in that element
    int32_t pad;
};

struct PlanHost {
    int d = 0, n = 0, bc = 0;
    int nnode = 0, nelem = 0, nfree = 0;
    std::vector<FrontHost> fronts;     // postorder (children before parents)
    std::vector<int32_t> rows, relind, children;
    std::vector<KPair> kpair;
    std::vector<KContrib> kcontrib;
    // flat gather list of the original entries: target (row << 16 | col) in the
    // front and up to 2^d element-matrix sources (flat index into the element
    // matrices [elem][2^d d][2^d d], -1 = none), asm_src[t * 2^d + q]
    std::vector<int32_t> asm_rc, asm_src;
    // extend-add map: for every entry t of a front's packed update matrix
    // (column-major lower, (m-p)(m-p+1)/2 entries) the offset of its target in
    // the parent's packed front, cpk(C, m_par) + R - C
    std::vector<int32_t> ea_dst;
    // fronts processed wave-per-front before the workgroup fronts, grouped by
    // height (all fronts of one height are independent)
    std::vector<int32_t> wave_list, wave_hbeg;
    // the other (workgroup) fronts in processing order, kStepFronts entries per
    // step (-1 padded): one front on the whole workgroup, or 2 or 4 independent
    // fronts (equal height, pivot and child counts) side by side on equal parts
    // of it
    std::vector<int32_t> wg_steps;
    int64_t wave_slice = 0;    // doubles of one wave's LDS slice (packed front + rhs rows)
    bool lds_path = false;     // every front fits the LDS front buffer
    int64_t L_size = 0;        // doubles of L + D + y storage
    int64_t U_stack = 0;       // doubles of the update-matrix stack
    int64_t U_scratch = 0;     // doubles of the largest update matrix (+ rhs)
    int max_m = 0, max_p = 0;
    double factor_flops = 0;   // LDL^T flops of one factorization (fronts, exact)
    int64_t nnz_L = 0;
};

// LDS budget of the front buffer (packed front + its m x d^2 rhs rows)
constexpr int64_t kLdsFrontBytes = 148 * 1024;
constexpr int kWaveFrontMaxM = 64;
constexpr int kStepFronts = 4;  // fronts per workgroup-front step at most

// Builds the plan; throws std::runtime_error on unsupported (d, n).
// structural parameters of a plan (the autotuner's plan-level knobs)
struct PlanParams {
    int leaf = 0;        // largest leaf box of the nested dissection (nodes); 0: 16 in 2D, 27 in 3D
    int wave_max_m = kWaveFrontMaxM;  // largest front factored by one wave (0: none)
    int bc = 0;          // 0 periodic (node 0 pinned), 1 linear displacements (every node with a grid index 0 pinned)
};


PlanHost build_plan(int d, int n, const PlanParams& prm = PlanParams{});

}  // namespace fehmm
