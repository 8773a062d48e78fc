// solver_dev.h -- device-side data structures of the batched RVE solver.
#pragma once
#include <cstdint>

#include "plan.h"

namespace fehmm {

struct DevFront {
    int32_t m, p, parent, child_begin, child_end, kmap_begin, kmap_end, asm_begin, asm_end, wave;
    int64_t rows_off, relind_off, L_off, D_off, y_off, U_off, ea_off;
};

struct DevPlan {
    int32_t d, n, nnode, nelem, nfront, lds_ok;  // lds_ok: every front fits the LDS front buffer
    const DevFront* fronts;
    const int32_t* rows;
    const int32_t* relind;
    const int32_t* children;
    const KPair* kpair;
    const KContrib* kcontrib;
    const int32_t* asm_rc;
    const int32_t* asm_src;
    const int32_t* ea_dst;
    const int32_t* wave_list;
    const int32_t* wave_hbeg;
    int32_t nwave_h;       // number of heights in the wave phase
    int32_t wave_slice;    // doubles per wave slice
    const int32_t* wg_steps;  // [nwg_steps][kStepFronts] workgroup-front steps (-1 padded)
    int32_t nwg_steps;
    int32_t bc;               // micro boundary conditions: 0 periodic, 1 linear displacements
};

// offsets (in doubles) of the per-slot workspace regions
struct SlotLayout {
    int64_t w, wt, R, rhs, x, fe, ke, re, L, U, S, ir1, ir2, stride;
};

struct SolveArgs {
    const DevPlan* plans;        // [nplan]
    const int32_t* rve_plan;     // [B]
    const int64_t* rve_phase;    // [B] offset into phase_pool
    const uint8_t* phase_pool;
    const int32_t* rve_lame;     // [B] offset (in doubles) into lame_pool
    const int32_t* rve_kind;     // [B] RVE_LAW_* | RVE_ELEM_* << 8 of each RVE's mesh
    const double* lame_pool;
    const int64_t* state_off;    // [B+1]
    const double* rve_atol;      // [B] default absolute tolerance
    const int32_t* order;        // [B] queue order (longest first), or a subset list
    const int32_t* count_dev;    // length of a subset list (device), or null for the whole batch
    const int* skip;             // device flag: when set, the launch solves nothing (graph-captured steps)
    int64_t B;
    double* ws;
    SlotLayout lay;
    unsigned int* counter;
    const double* F;
    double* P;
    double* A;
    double* wstate;
    int32_t* status;
    int32_t* iters;
    double rtol, atol;
    int32_t max_iter, backtrack, want_A, dim;
    int32_t lds_front;           // elements (of the front type) of the LDS front region; rhs rows follow
    int32_t flags;               // RVE_FLAG_* of the options
    int32_t wave_slice;          // elements of one wave's LDS slice in the wave phase
    int32_t ir_max;              // refinement sweeps per Newton step (FP32 factors)
    int32_t ir_max_tan;          // refinement sweeps of the tangent solves
    int32_t tan64;               // FP32 factors: the condensation factorization of LDS plans in FP64
    int32_t lds_front64;         // FP64 elements of the front region for that factorization
    int32_t reuse_tan;           // 2D LDS plans: the condensation from the last Newton factorization
    double ir_eta;               // stop refining when ||b - K x|| <= ir_eta ||R||
    double ir_eta_tan;           // same for the d^2 tangent columns (Frobenius)
};

// LDS available to the front buffer (packed front + m x d^2 rhs rows)
constexpr int kLdsBytesMax = 160 * 1024;

// tiles of the global-front updates: kTileM rows x (64 or 128) columns per
// pass; two LDS buffers of a 16-column slab of A (kTileM rows) and B (up to
// 128 rows), row stride 144 elements (= 16 mod 32: the four lane groups of an
// MFMA operand read hit distinct LDS banks)
constexpr int kTileM = 128, kTileSlab = 16, kTileStride = 144;
constexpr int kTileLdsElems = 2 * kTileSlab * 2 * kTileStride;

}  // namespace fehmm
