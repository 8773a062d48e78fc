// rve_abi.cpp -- C ABI of the batched RVE solver (include/rve.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rve.h"
#include "plan.h"
#include "solver_dev.h"

namespace fehmm {
// the solver compiled with 256-thread (four-wave) and 512-thread (eight-wave) workgroups
namespace nt256 {
hipError_t launch_rve_solve(const SolveArgs& a, int nslots, size_t dyn_bytes, bool fp32, hipStream_t stream);
hipError_t launch_rve_assembly(const SolveArgs& a, int nslots, hipStream_t stream);
hipError_t prepare_rve_solve();
int lds_static_bytes();
}
namespace nt512 {
hipError_t launch_rve_solve(const SolveArgs& a, int nslots, size_t dyn_bytes, bool fp32, hipStream_t stream);
hipError_t launch_rve_assembly(const SolveArgs& a, int nslots, hipStream_t stream);
hipError_t prepare_rve_solve();
int lds_static_bytes();
}
constexpr int NWAVE_ = 4;  // waves per workgroup of the default solver
}

using namespace fehmm;

namespace {

// caller-provided workspaces: the queue counter takes the first 256 bytes (the
// slots that follow stay 256-byte aligned)
constexpr size_t kExtCounterBytes = 256;

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_OR(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(RVE_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- plan cache
using PlanKey = std::tuple<int, int, int, int, int>;  // d, n, leaf, wave_max_m, bc

struct PlanEntry {
    PlanKey key;
    PlanHost host;
    DevPlan dev{};          // device pointers inside
    DevFront* d_fronts = nullptr;
    int32_t* d_rows = nullptr;
    int32_t* d_relind = nullptr;
    int32_t* d_children = nullptr;
    KPair* d_kpair = nullptr;
    KContrib* d_kcontrib = nullptr;
    int32_t* d_asm_rc = nullptr;
    int32_t* d_asm_src = nullptr;
    int32_t* d_ea_dst = nullptr;
    int32_t* d_wave_list = nullptr;
    int32_t* d_wave_hbeg = nullptr;
    int32_t* d_wg_steps = nullptr;
    int refs = 0;
    int device = -1;
    int64_t lds_bytes = 0;            // FP64 fronts: dynamic LDS bytes
    int64_t front_elems[2] = {0, 0};  // LDS front region (elements of FP64 / FP32)
    int64_t rl_elems = 0;             // rhs rows following it
};

std::mutex g_mu;
std::map<PlanKey, std::unique_ptr<PlanEntry>> g_plans;
// tuned choices per (d, n): plan parameters and persistent workgroups
std::map<std::pair<int, int>, rve_tuning> g_tuning;

PlanParams params_for(int d, int n) {
    PlanParams p;
    auto it = g_tuning.find(std::make_pair(d, n));
    if (it != g_tuning.end()) {
        p.leaf = it->second.leaf;
        p.wave_max_m = it->second.wave_max_m;
    }
    return p;
}

int tuned_slots(int d, int n) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tuning.find(std::make_pair(d, n));
    return it != g_tuning.end() ? it->second.slots : 0;
}

int tuned_threads(int d, int n) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tuning.find(std::make_pair(d, n));
    return it != g_tuning.end() ? it->second.threads : 0;
}

template <typename T>
int upload(const std::vector<T>& v, T** out) {
    size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
    HIP_OR(hipMalloc((void**)out, bytes));
    if (!v.empty()) HIP_OR(hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return RVE_OK;
}

void free_plan_dev(PlanEntry& e) {
    (void)hipFree(e.d_fronts); (void)hipFree(e.d_rows); (void)hipFree(e.d_relind);
    (void)hipFree(e.d_children); (void)hipFree(e.d_kpair); (void)hipFree(e.d_kcontrib);
    (void)hipFree(e.d_asm_rc); (void)hipFree(e.d_asm_src); (void)hipFree(e.d_ea_dst);
    (void)hipFree(e.d_wave_list); (void)hipFree(e.d_wave_hbeg); (void)hipFree(e.d_wg_steps);
    e.d_fronts = nullptr;
}

// the plan of (d, n) under the current tuning for micro boundary conditions bc
int get_plan(int d, int n, PlanEntry** out, int bc = RVE_BC_PERIODIC) {
    std::lock_guard<std::mutex> lk(g_mu);
    PlanParams prm = params_for(d, n);
    prm.bc = bc;
    const PlanKey key(d, n, prm.leaf, prm.wave_max_m, bc);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second.get();
        return RVE_OK;
    }
    auto e = std::make_unique<PlanEntry>();
    e->key = key;
    try {
        e->host = build_plan(d, n, prm);
    } catch (const std::exception& ex) {
        return fail(RVE_EINVAL, std::string("plan: ") + ex.what());
    }
    *out = e.get();
    g_plans[key] = std::move(e);
    return RVE_OK;
}

int plan_device(PlanEntry* e) {
    if (e->d_fronts) return RVE_OK;
    const PlanHost& P = e->host;
    std::vector<DevFront> fr(P.fronts.size());
    for (size_t s = 0; s < fr.size(); ++s) {
        const FrontHost& f = P.fronts[s];
        fr[s] = DevFront{f.m, f.p, f.parent, f.child_begin, f.child_end, f.kmap_begin, f.kmap_end, f.asm_begin,
                         f.asm_end, f.wave, f.rows_off, f.relind_off, f.L_off, f.D_off, f.y_off, f.U_off, f.ea_off};
    }
    int st;
    if ((st = upload(fr, &e->d_fronts)) || (st = upload(P.rows, &e->d_rows)) || (st = upload(P.relind, &e->d_relind)) ||
        (st = upload(P.children, &e->d_children)) || (st = upload(P.kpair, &e->d_kpair)) ||
        (st = upload(P.kcontrib, &e->d_kcontrib)) || (st = upload(P.asm_rc, &e->d_asm_rc)) ||
        (st = upload(P.asm_src, &e->d_asm_src)) || (st = upload(P.ea_dst, &e->d_ea_dst)) ||
        (st = upload(P.wave_list, &e->d_wave_list)) || (st = upload(P.wave_hbeg, &e->d_wave_hbeg)) ||
        (st = upload(P.wg_steps, &e->d_wg_steps))) {
        free_plan_dev(*e);
        return st;
    }
    e->dev = DevPlan{P.d, P.n, P.nnode, P.nelem, (int32_t)P.fronts.size(), 0,
                     e->d_fronts, e->d_rows, e->d_relind, e->d_children, e->d_kpair, e->d_kcontrib,
                     e->d_asm_rc, e->d_asm_src, e->d_ea_dst, e->d_wave_list, e->d_wave_hbeg,
                     (int32_t)P.wave_hbeg.size() - 1, (int32_t)P.wave_slice, e->d_wg_steps,
                     (int32_t)(P.wg_steps.size() / kStepFronts)};
    if (P.wave_hbeg.empty()) e->dev.nwave_h = 0;
    e->dev.bc = P.bc;
    // whole fronts in LDS when the largest packed front plus its rhs rows fit;
    // the front region also hosts the FP64 scratch of the triangular solves
    // (m d^2 + 3 m doubles)
    const int64_t mm = P.max_m;
    int64_t scratch = 0;
    for (const FrontHost& fr : P.fronts) scratch = std::max<int64_t>(scratch, (int64_t)fr.m * (P.d * P.d + 3));
    e->front_elems[0] = std::max<int64_t>(mm * (mm + 1) / 2, scratch);
    e->front_elems[1] = std::max<int64_t>(mm * (mm + 1) / 2, 2 * scratch);
    // rhs rows (d^2 + 1 in 2D: the Newton residual beside the condensation's
    // columns, see rve_solve_kernel), then the original diagonal
    e->rl_elems = mm * (P.d * P.d + (P.d == 2 ? 2 : 1));
    const int64_t need = std::max<int64_t>(e->front_elems[0] + e->rl_elems, NWAVE_ * P.wave_slice) *
                         (int64_t)sizeof(double);
    e->lds_bytes = need;
    // (one thread per front row in the pivot sweep: m <= 256; the plan decides)
    e->dev.lds_ok = (P.lds_path && need + nt256::lds_static_bytes() + 1024 <= kLdsBytesMax) ? 1 : 0;
    return RVE_OK;
}

}  // namespace

int rve_internal_set_error(int code, const std::string& msg) { return fail(code, msg); }

// rve_solve_batch(_subset) whose launch does nothing while *skip is set on the
// device (the two-scale driver's graph-captured load steps)
int rve_internal_solve(rve_batch b, const int32_t* subset, const int32_t* count, const double* F, double* P,
                       double* A, double* w_state, int32_t* status, int32_t* iters, const rve_opts* opts,
                       void* hip_stream, const int* skip);

struct rve_mesh_s {
    int d = 0, n = 0, nphase = 0;
    std::vector<double> lame;
    std::vector<uint8_t> phase;
    PlanEntry* plan = nullptr;
    double mu_max = 0;
    int law = RVE_LAW_NEOHOOKE;
    int bc = RVE_BC_PERIODIC;
    int elem = RVE_ELEM_Q1;
    bool alive = true;
};

struct rve_batch_s {
    int d = 0;
    int64_t B = 0;
    int nslots = 0;
    int64_t lds_front[2] = {0, 0};  // front region of the dynamic LDS (FP64 / FP32 elements)
    int64_t wave_slice = 0;         // elements per wave slice
    size_t dyn_bytes[2] = {0, 0};
    // per precision: launch the eight-wave solver (2D LDS plans whose fronts leave
    // room for one four-wave workgroup per CU only) with its dynamic LDS size
    bool wide[2] = {false, false};
    size_t dyn_bytes_wide[2] = {0, 0};
    SlotLayout lay{};
    std::vector<int64_t> state_off;
    // device
    DevPlan* d_plans = nullptr;
    int32_t* d_rve_plan = nullptr;
    int64_t* d_rve_phase = nullptr;
    uint8_t* d_phase_pool = nullptr;
    int32_t* d_rve_lame = nullptr;
    int32_t* d_rve_kind = nullptr;
    double* d_lame_pool = nullptr;
    int64_t* d_state_off = nullptr;
    double* d_atol = nullptr;
    int32_t* d_order = nullptr;
    double* d_ws = nullptr;
    unsigned int* d_counter = nullptr;
    int device = -1;  // the device the batch's memory lives on
    bool alive = true;
};

extern "C" {

int rve_lame(double E, double nu, double* lam, double* mu) {
    if (!lam || !mu) return fail(RVE_EINVAL, "rve_lame: NULL output");
    if (!(E > 0) || !(nu > -1.0 && nu < 0.5)) return fail(RVE_EINVAL, "rve_lame: need E > 0 and -1 < nu < 0.5");
    *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    *mu = E / (2.0 * (1.0 + nu));
    return RVE_OK;
}

void rve_opts_default(rve_opts* o) {
    if (!o) return;
    o->rtol = 1e-10;
    o->atol = -1.0;
    o->max_iter = 25;
    o->precision = RVE_PREC_FP64;
    o->det_backtrack = 8;
    o->flags = 0;
}

const char* rve_strerror(int code) {
    switch (code) {
        case RVE_OK: return "ok";
        case RVE_EPARTIAL: return "some RVEs failed (see status)";
        case RVE_EINVAL: return "invalid argument";
        case RVE_ENOMEM: return "out of memory";
        case RVE_EHIP: return "HIP runtime error";
        case RVE_EUNSUPPORTED: return "unsupported";
        default: return "unknown error";
    }
}

int rve_last_error(char* buf, size_t n) {
    if (!buf || n == 0) return RVE_EINVAL;
    std::snprintf(buf, n, "%s", g_err.c_str());
    return RVE_OK;
}

int rve_plan_info(int32_t ndim, int32_t n, double* flops, int64_t* nnz, int32_t* nfronts, int32_t* max_front) {
    PlanEntry* e = nullptr;
    int st = get_plan(ndim, n, &e);
    if (st) return st;
    if (flops) *flops = e->host.factor_flops;
    if (nnz) *nnz = e->host.nnz_L;
    if (nfronts) *nfronts = (int32_t)e->host.fronts.size();
    if (max_front) *max_front = e->host.max_m;
    return RVE_OK;
}

int rve_mesh_create(const rve_mesh_desc* d, rve_mesh* out) {
    if (!d || !out) return fail(RVE_EINVAL, "rve_mesh_create: NULL argument");
    *out = nullptr;
    if (!(d->ndim == 2 || d->ndim == 3)) return fail(RVE_EINVAL, "rve_mesh_create: ndim must be 2 or 3");
    const int nmax = d->ndim == 2 ? 64 : 24;
    if (d->n < 2 || d->n > nmax) return fail(RVE_EINVAL, "rve_mesh_create: n out of range");
    if (d->nphase < 1 || d->nphase > 255 || !d->lame) return fail(RVE_EINVAL, "rve_mesh_create: bad phase table");
    for (int q = 0; q < d->nphase; ++q) {
        double lam = d->lame[2 * q], mu = d->lame[2 * q + 1];
        if (!std::isfinite(lam) || !std::isfinite(mu) || !(mu > 0))
            return fail(RVE_EINVAL, "rve_mesh_create: lame parameters must be finite with mu > 0");
    }
    if (d->law < RVE_LAW_NEOHOOKE || d->law > RVE_LAW_LINEAR)
        return fail(RVE_EINVAL, "rve_mesh_create: unknown constitutive law");
    if (d->bc != RVE_BC_PERIODIC && d->bc != RVE_BC_LINEAR)
        return fail(RVE_EINVAL, "rve_mesh_create: unknown micro boundary conditions");
    if (d->elem != RVE_ELEM_Q1 && d->elem != RVE_ELEM_P1)
        return fail(RVE_EINVAL, "rve_mesh_create: unknown element kind");
    auto m = std::make_unique<rve_mesh_s>();
    m->law = d->law;
    m->bc = d->bc;
    m->elem = d->elem;
    m->d = d->ndim;
    m->n = d->n;
    m->nphase = d->nphase;
    m->lame.assign(d->lame, d->lame + 2 * d->nphase);
    int ne = 1;
    for (int k = 0; k < m->d; ++k) ne *= m->n;
    m->phase.resize(ne);
    if (d->phase) {
        for (int e = 0; e < ne; ++e) {
            if (d->phase[e] >= d->nphase) return fail(RVE_EINVAL, "rve_mesh_create: phase id >= nphase");
            m->phase[e] = d->phase[e];
        }
    } else {
        if (d->incl_phase < 0 || d->incl_phase >= d->nphase)
            return fail(RVE_EINVAL, "rve_mesh_create: incl_phase out of range");
        const double h = 1.0 / m->n;
        for (int e = 0; e < ne; ++e) {
            int t = e;
            double r2 = 0;
            for (int k = 0; k < m->d; ++k) {
                double x = ((t % m->n) + 0.5) * h - d->incl_center[k];
                r2 += x * x;
                t /= m->n;
            }
            m->phase[e] = (std::sqrt(r2) < d->incl_radius) ? (uint8_t)d->incl_phase : 0;
        }
    }
    for (int q = 0; q < m->nphase; ++q) m->mu_max = std::max(m->mu_max, m->lame[2 * q + 1]);
    int st = get_plan(m->d, m->n, &m->plan, m->bc);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        m->plan->refs++;
    }
    *out = m.release();
    return RVE_OK;
}

int rve_mesh_destroy(rve_mesh m) {
    if (!m || !m->alive) return fail(RVE_EINVAL, "rve_mesh_destroy: invalid handle");
    m->alive = false;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (--m->plan->refs == 0) {
            free_plan_dev(*m->plan);
            g_plans.erase(m->plan->key);
        }
    }
    // the husk stays allocated so that a second destroy is detected
    m->lame.clear();
    m->phase.clear();
    return RVE_OK;
}

int rve_mesh_get_phase(rve_mesh m, uint8_t* host_phase) {
    if (!m || !m->alive || !host_phase) return fail(RVE_EINVAL, "rve_mesh_get_phase: invalid argument");
    std::memcpy(host_phase, m->phase.data(), m->phase.size());
    return RVE_OK;
}

static void free_batch(rve_batch_s* b) {
    (void)hipFree(b->d_plans); (void)hipFree(b->d_rve_plan); (void)hipFree(b->d_rve_phase); (void)hipFree(b->d_phase_pool);
    (void)hipFree(b->d_rve_lame); (void)hipFree(b->d_rve_kind); (void)hipFree(b->d_lame_pool); (void)hipFree(b->d_state_off); (void)hipFree(b->d_atol);
    (void)hipFree(b->d_order); (void)hipFree(b->d_ws); (void)hipFree(b->d_counter);
    b->d_ws = nullptr;
}

// kernel attributes (dynamic LDS limits), set once per process before the first
// launch -- at batch creation, so that no attribute call falls inside a graph
// capture of a later solve
static int ensure_prepared() {
    static bool prepared = false;
    if (!prepared) {
        hipError_t pe = nt256::prepare_rve_solve();
        if (pe == hipSuccess) pe = nt512::prepare_rve_solve();
        if (pe != hipSuccess) return fail(RVE_EHIP, std::string("rve kernels: ") + hipGetErrorString(pe));
        prepared = true;
    }
    return RVE_OK;
}

int rve_batch_create(const rve_mesh* meshes, int64_t B, rve_batch* out) {
    if (!meshes || !out || B <= 0) return fail(RVE_EINVAL, "rve_batch_create: invalid argument");
    *out = nullptr;
    for (int64_t r = 0; r < B; ++r)
        if (!meshes[r] || !meshes[r]->alive) return fail(RVE_EINVAL, "rve_batch_create: invalid mesh handle");
    {
        const int pst = ensure_prepared();
        if (pst) return pst;
    }
    const int d = meshes[0]->d;
    for (int64_t r = 0; r < B; ++r)
        if (meshes[r]->d != d) return fail(RVE_EUNSUPPORTED, "rve_batch_create: all meshes of a batch must share ndim");
    auto b = std::make_unique<rve_batch_s>();
    b->d = d;
    b->B = B;
    HIP_OR(hipGetDevice(&b->device));
    // distinct plans and meshes
    std::vector<PlanEntry*> plans;
    std::map<PlanEntry*, int> plan_id;
    std::map<rve_mesh, std::pair<int64_t, int32_t>> mesh_off;  // phase offset, lame offset
    std::vector<uint8_t> phase_pool;
    std::vector<double> lame_pool;
    std::vector<int32_t> rve_plan(B), rve_lame(B), rve_kind(B);
    std::vector<int64_t> rve_phase(B);
    std::vector<double> atol(B);
    b->state_off.resize(B + 1);
    b->state_off[0] = 0;
    std::vector<double> cost(B);
    for (int64_t r = 0; r < B; ++r) {
        rve_mesh m = meshes[r];
        if (!plan_id.count(m->plan)) {
            plan_id[m->plan] = (int)plans.size();
            plans.push_back(m->plan);
        }
        auto it = mesh_off.find(m);
        if (it == mesh_off.end()) {
            std::pair<int64_t, int32_t> off((int64_t)phase_pool.size(), (int32_t)lame_pool.size());
            phase_pool.insert(phase_pool.end(), m->phase.begin(), m->phase.end());
            lame_pool.insert(lame_pool.end(), m->lame.begin(), m->lame.end());
            it = mesh_off.emplace(m, off).first;
        }
        rve_plan[r] = plan_id[m->plan];
        rve_phase[r] = it->second.first;
        rve_lame[r] = it->second.second;
        rve_kind[r] = m->law | (m->elem << 8);
        atol[r] = 1e-12 * m->mu_max * std::pow(1.0 / m->n, d - 1);
        b->state_off[r + 1] = b->state_off[r] + (int64_t)d * m->plan->host.nnode;
        cost[r] = m->plan->host.factor_flops;
    }
    std::vector<int32_t> order(B);
    for (int64_t r = 0; r < B; ++r) order[r] = (int32_t)r;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
    // workspace layout: max over the distinct plans
    int64_t nn = 0, ne = 0, Lsz = 0, Ust = 0, Usc = 0;
    const int nen = 1 << d, nd = nen * d, d2 = d * d;
    for (PlanEntry* p : plans) {
        int st = plan_device(p);
        if (st) return st;
        nn = std::max<int64_t>(nn, p->host.nnode);
        ne = std::max<int64_t>(ne, p->host.nelem);
        Lsz = std::max(Lsz, p->host.L_size);
        Ust = std::max(Ust, p->host.U_stack);
        Usc = std::max(Usc, p->host.U_scratch);
    }
    for (PlanEntry* p : plans)
        if (p->dev.lds_ok) {
            for (int k = 0; k < 2; ++k) b->lds_front[k] = std::max(b->lds_front[k], p->front_elems[k]);
            b->wave_slice = std::max(b->wave_slice, p->host.wave_slice);
        }
    {
        int64_t rl = 0;
        for (PlanEntry* p : plans)
            if (p->dev.lds_ok) rl = std::max(rl, p->rl_elems);
        bool glb = false;
        for (PlanEntry* p : plans) glb = glb || !p->dev.lds_ok;
        const int threads = tuned_threads(d, meshes[0]->n);
        for (int k = 0; k < 2; ++k) {
            const int64_t es = k == 0 ? 8 : 4;
            int64_t elems = std::max(b->lds_front[k] + rl, NWAVE_ * b->wave_slice);
            int64_t bytes = elems * es;
            // global fronts: staged tile slabs, FP64-sized in both kernels (the
            // condensation factorization of global-front plans is FP64)
            if (glb) bytes = std::max<int64_t>(bytes, (int64_t)kTileLdsElems * 8);
            b->dyn_bytes[k] = (size_t)bytes;
            // eight waves: 2D plans with fronts in LDS, by default where the
            // fronts leave room for one four-wave workgroup per CU only
            const int64_t wide_bytes = std::max(b->lds_front[k] + rl, 2 * NWAVE_ * b->wave_slice) * es;
            const bool wide_fits = d == 2 && !glb && wide_bytes + nt512::lds_static_bytes() + 1024 <= kLdsBytesMax;
            const bool wide_rule = bytes + nt256::lds_static_bytes() > kLdsBytesMax / 2;
            b->wide[k] = wide_fits && (threads == 512 || (threads == 0 && wide_rule));
            b->dyn_bytes_wide[k] = (size_t)wide_bytes;
        }
    }
    auto rnd = [](int64_t x) { return (x + 31) / 32 * 32; };
    SlotLayout& L = b->lay;
    int64_t o = 0;
    L.w = o; o += rnd(nn * d);
    L.wt = o; o += rnd(nn * d);
    L.R = o; o += rnd(nn * d);
    L.rhs = o; o += rnd(nn * d * (d2 + 1));
    L.x = o; o += rnd(nn * d);
    L.fe = o; o += rnd(ne * nd);
    L.ke = o; o += rnd(ne * nd * nd);
    L.re = o; o += rnd(ne * nd * d2);
    L.L = o; o += rnd(Lsz);
    L.U = o; o += rnd(std::max<int64_t>(Ust, 1));
    L.S = o; o += rnd(std::max<int64_t>(Usc, 1));
    L.ir1 = o; o += rnd(nn * d * d2);
    L.ir2 = o; o += rnd(nn * d * d2);
    L.stride = o;
    size_t free_b = 0, total_b = 0;
    HIP_OR(hipMemGetInfo(&free_b, &total_b));
    const double slot_bytes = (double)L.stride * sizeof(double);
    int64_t cap = (int64_t)(0.5 * (double)free_b / slot_bytes);
    const int tslots = tuned_slots(d, meshes[0]->n);
    int64_t nslots = std::min<int64_t>({B, tslots > 0 ? (int64_t)tslots : (int64_t)1024, cap});
    if (nslots < 1) return fail(RVE_ENOMEM, "rve_batch_create: not enough device memory for one workspace slot");
    b->nslots = (int)nslots;
    std::vector<DevPlan> dplans;
    for (PlanEntry* p : plans) dplans.push_back(p->dev);
    int st;
    if ((st = upload(dplans, &b->d_plans)) || (st = upload(rve_plan, &b->d_rve_plan)) ||
        (st = upload(rve_phase, &b->d_rve_phase)) || (st = upload(phase_pool, &b->d_phase_pool)) ||
        (st = upload(rve_lame, &b->d_rve_lame)) || (st = upload(rve_kind, &b->d_rve_kind)) ||
        (st = upload(lame_pool, &b->d_lame_pool)) ||
        (st = upload(b->state_off, &b->d_state_off)) || (st = upload(atol, &b->d_atol)) ||
        (st = upload(order, &b->d_order))) {
        free_batch(b.get());
        return st;
    }
    hipError_t e1 = hipMalloc((void**)&b->d_ws, (size_t)L.stride * nslots * sizeof(double));
    hipError_t e2 = hipMalloc((void**)&b->d_counter, 256);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        free_batch(b.get());
        return fail(RVE_ENOMEM, "rve_batch_create: workspace allocation failed");
    }
    *out = b.release();
    return RVE_OK;
}

int rve_batch_destroy(rve_batch b) {
    if (!b || !b->alive) return fail(RVE_EINVAL, "rve_batch_destroy: invalid handle");
    free_batch(b);
    b->alive = false;
    return RVE_OK;
}

int rve_batch_state_offsets(rve_batch b, int64_t* host_off) {
    if (!b || !b->alive || !host_off) return fail(RVE_EINVAL, "rve_batch_state_offsets: invalid argument");
    std::memcpy(host_off, b->state_off.data(), sizeof(int64_t) * (b->B + 1));
    return RVE_OK;
}

// ext_ws: optional caller-provided device memory (queue counter in its first
// 256 bytes, then workspace slots) of ext_bytes bytes used instead of the
// batch's own workspace; the number of persistent workgroups is then limited to
// the slots that fit
static int solve_batch_impl(rve_batch b, const int32_t* subset, const int32_t* subset_count, const double* F,
                            double* P, double* A, double* w_state, int32_t* status, int32_t* iters,
                            const rve_opts* opts, void* hip_stream, const int* skip, void* ext_ws = nullptr,
                            size_t ext_bytes = 0) {
    if (!b || !b->alive) return fail(RVE_EINVAL, "rve_solve_batch: invalid batch handle");
    if (!F || !P) return fail(RVE_EINVAL, "rve_solve_batch: F and P are required");
    int nslots = b->nslots;
    double* ws = b->d_ws;
    unsigned int* counter = b->d_counter;
    if (ext_ws) {
        const size_t slot_bytes = (size_t)b->lay.stride * sizeof(double);
        const size_t fit = ext_bytes > kExtCounterBytes ? (ext_bytes - kExtCounterBytes) / slot_bytes : 0;
        if (fit < 1)
            return fail(RVE_EINVAL, "rve_solve_batch_static: one workspace slot of this batch (" +
                                        std::to_string(slot_bytes) + " bytes) does not fit the static scratch (" +
                                        std::to_string(ext_bytes) + " bytes)");
        nslots = (int)std::min<size_t>((size_t)nslots, fit);
        counter = reinterpret_cast<unsigned int*>(ext_ws);
        ws = reinterpret_cast<double*>(reinterpret_cast<char*>(ext_ws) + kExtCounterBytes);
    }
    rve_opts o;
    rve_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.rtol >= 0) || o.max_iter < 0 || o.max_iter > 1000 || o.det_backtrack < 0 || o.det_backtrack > 60)
        return fail(RVE_EINVAL, "rve_solve_batch: options out of range");
    if (o.precision != RVE_PREC_FP64 && o.precision != RVE_PREC_FP32_IR)
        return fail(RVE_EINVAL, "rve_solve_batch: unknown precision");
    int pst = ensure_prepared();
    if (pst) return pst;
    const bool fp32 = o.precision == RVE_PREC_FP32_IR;
    SolveArgs a{};
    a.plans = b->d_plans;
    a.rve_plan = b->d_rve_plan;
    a.rve_phase = b->d_rve_phase;
    a.phase_pool = b->d_phase_pool;
    a.rve_lame = b->d_rve_lame;
    a.rve_kind = b->d_rve_kind;
    a.lame_pool = b->d_lame_pool;
    a.state_off = b->d_state_off;
    a.rve_atol = b->d_atol;
    a.order = subset ? subset : b->d_order;
    a.count_dev = subset ? subset_count : nullptr;
    a.skip = skip;
    a.B = b->B;
    a.ws = ws;
    a.lay = b->lay;
    a.counter = counter;
    a.F = F;
    a.P = P;
    a.A = A;
    a.wstate = w_state;
    a.status = status;
    a.iters = iters;
    a.rtol = o.rtol;
    a.atol = o.atol;
    a.max_iter = o.max_iter;
    a.backtrack = o.det_backtrack;
    a.want_A = A != nullptr;
    a.dim = b->d;
    a.flags = o.flags;
    const int k = fp32 ? 1 : 0;
    a.lds_front = (int32_t)b->lds_front[k];
    a.wave_slice = (int32_t)b->wave_slice;
    const bool wide = b->wide[k];
    size_t dyn = wide ? b->dyn_bytes_wide[k] : b->dyn_bytes[k];
    // FP32 factors: where the FP64 front region keeps two workgroups per CU (the
    // register limit), the condensation factorization runs in FP64 and the direct
    // Schur form replaces the refined FP32 solves
    a.tan64 = 0;
    a.lds_front64 = (int32_t)b->lds_front[0];
    if (fp32 && !wide && (int64_t)b->dyn_bytes[0] + nt256::lds_static_bytes() <= kLdsBytesMax / 2) {
        a.tan64 = 1;
        dyn = std::max(dyn, b->dyn_bytes[0]);
    }
    // FP32 factors: a Newton step is refined only when ||b - K64 x|| > 1e-2 ||b||
    // (inexact Newton; convergence is judged on the FP64 residual); the tangent
    // takes the second-order (stationary) form straight from the FP32 solve: its
    // error is quadratic in the solve's (about 1e-11 relative at 32 x 32, where a
    // refinement sweep bought 2e-12 for 12 % of the batch time)
    a.ir_max = 2;
    a.ir_max_tan = 0;
    a.reuse_tan = (A != nullptr && !(o.flags & RVE_FLAG_DIRECT_TANGENT)) ? 1 : 0;
    a.ir_eta = 1e-2;
    a.ir_eta_tan = 0.0;
    hipError_t e = wide ? nt512::launch_rve_solve(a, nslots, dyn, fp32, (hipStream_t)hip_stream)
                        : nt256::launch_rve_solve(a, nslots, dyn, fp32, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(RVE_EHIP, std::string("rve_solve_batch launch: ") + hipGetErrorString(e));
    return RVE_OK;
}

int rve_solve_batch(rve_batch b, const double* F, double* P, double* A, double* w_state, int32_t* status,
                    int32_t* iters, const rve_opts* opts, void* hip_stream) {
    return solve_batch_impl(b, nullptr, nullptr, F, P, A, w_state, status, iters, opts, hip_stream, nullptr);
}

int rve_solve_batch_subset(rve_batch b, const int32_t* idx, const int32_t* count, const double* F, double* P,
                           double* A, double* w_state, int32_t* status, int32_t* iters, const rve_opts* opts,
                           void* hip_stream) {
    if (!idx || !count) return fail(RVE_EINVAL, "rve_solve_batch_subset: idx and count are required");
    return solve_batch_impl(b, idx, count, F, P, A, w_state, status, iters, opts, hip_stream, nullptr);
}

int rve_assemble_batch(rve_batch b, const double* F, const double* w_state, int32_t* status, void* hip_stream) {
    if (!b || !b->alive || !F) return fail(RVE_EINVAL, "rve_assemble_batch: invalid argument");
    int pst = ensure_prepared();
    if (pst) return pst;
    SolveArgs a{};
    a.plans = b->d_plans;
    a.rve_plan = b->d_rve_plan;
    a.rve_phase = b->d_rve_phase;
    a.phase_pool = b->d_phase_pool;
    a.rve_lame = b->d_rve_lame;
    a.rve_kind = b->d_rve_kind;
    a.lame_pool = b->d_lame_pool;
    a.state_off = b->d_state_off;
    a.rve_atol = b->d_atol;
    a.order = b->d_order;
    a.B = b->B;
    a.ws = b->d_ws;
    a.lay = b->lay;
    a.counter = b->d_counter;
    a.F = F;
    a.wstate = const_cast<double*>(w_state);
    a.status = status;
    a.dim = b->d;
    a.atol = -1.0;
    hipError_t e = nt256::launch_rve_assembly(a, b->nslots, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(RVE_EHIP, std::string("rve_assemble_batch launch: ") + hipGetErrorString(e));
    return RVE_OK;
}

int rve_solve_batch_sync(rve_batch b, const double* F, double* P, double* A, double* w_state, int32_t* status,
                         int32_t* iters, const rve_opts* opts, void* hip_stream) {
    if (!status) return fail(RVE_EINVAL, "rve_solve_batch_sync: status is required");
    int st = rve_solve_batch(b, F, P, A, w_state, status, iters, opts, hip_stream);
    if (st) return st;
    HIP_OR(hipStreamSynchronize((hipStream_t)hip_stream));
    std::vector<int32_t> h(b->B);
    HIP_OR(hipMemcpy(h.data(), status, sizeof(int32_t) * b->B, hipMemcpyDeviceToHost));
    for (int32_t s : h)
        if (s != RVE_S_CONVERGED) return RVE_EPARTIAL;
    return RVE_OK;
}

}  // extern "C"

extern "C" int rve_plan_schedule(int32_t ndim, int32_t n, int64_t* nsteps, int32_t* steps, int32_t* wave) {
    PlanEntry* e = nullptr;
    int st = get_plan(ndim, n, &e);
    if (st) return st;
    const PlanHost& P = e->host;
    if (!nsteps) return fail(RVE_EINVAL, "rve_plan_schedule: nsteps is required");
    *nsteps = P.lds_path ? (int64_t)(P.wg_steps.size() / kStepFronts) : 0;
    if (steps && P.lds_path) std::memcpy(steps, P.wg_steps.data(), P.wg_steps.size() * sizeof(int32_t));
    if (wave)
        for (size_t s = 0; s < P.fronts.size(); ++s) wave[s] = P.lds_path ? P.fronts[s].wave : 0;
    return RVE_OK;
}

extern "C" int rve_plan_export(int32_t ndim, int32_t n, int64_t* sizes, int32_t* fronts, int32_t* rows,
                               int32_t* relind, int32_t* children, int32_t* kpair, int32_t* kcontrib) {
    PlanEntry* e = nullptr;
    int st = get_plan(ndim, n, &e);
    if (st) return st;
    const PlanHost& P = e->host;
    if (!sizes) return fail(RVE_EINVAL, "rve_plan_export: sizes is required");
    sizes[0] = (int64_t)P.fronts.size();
    sizes[1] = (int64_t)P.rows.size();
    sizes[2] = (int64_t)P.relind.size();
    sizes[3] = (int64_t)P.children.size();
    sizes[4] = (int64_t)P.kpair.size();
    sizes[5] = (int64_t)P.kcontrib.size();
    if (fronts)
        for (size_t s = 0; s < P.fronts.size(); ++s) {
            const FrontHost& f = P.fronts[s];
            int32_t* o = fronts + 8 * s;
            o[0] = f.m; o[1] = f.p; o[2] = f.parent; o[3] = (int32_t)f.rows_off; o[4] = (int32_t)f.relind_off;
            o[5] = f.child_begin; o[6] = f.child_end; o[7] = f.kmap_begin;
        }
    if (rows) std::memcpy(rows, P.rows.data(), P.rows.size() * sizeof(int32_t));
    if (relind) std::memcpy(relind, P.relind.data(), P.relind.size() * sizeof(int32_t));
    if (children) std::memcpy(children, P.children.data(), P.children.size() * sizeof(int32_t));
    if (kpair)
        for (size_t q = 0; q < P.kpair.size(); ++q) {
            kpair[4 * q] = P.kpair[q].row_node; kpair[4 * q + 1] = P.kpair[q].col_node;
            kpair[4 * q + 2] = P.kpair[q].c_begin; kpair[4 * q + 3] = P.kpair[q].c_count;
        }
    if (kcontrib)
        for (size_t q = 0; q < P.kcontrib.size(); ++q) {
            kcontrib[3 * q] = P.kcontrib[q].elem; kcontrib[3 * q + 1] = P.kcontrib[q].la;
            kcontrib[3 * q + 2] = P.kcontrib[q].lb;
        }
    return RVE_OK;
}

int rve_internal_solve(rve_batch b, const int32_t* subset, const int32_t* count, const double* F, double* P,
                       double* A, double* w_state, int32_t* status, int32_t* iters, const rve_opts* opts,
                       void* hip_stream, const int* skip) {
    return solve_batch_impl(b, subset, count, F, P, A, w_state, status, iters, opts, hip_stream, skip);
}

int rve_internal_solve_ext(rve_batch b, const double* F, double* P, double* A, double* w_state, int32_t* status,
                           int32_t* iters, const rve_opts* opts, void* hip_stream, void* ext_ws, size_t ext_bytes,
                           int device) {
    if (!ext_ws) return fail(RVE_EINVAL, "rve_solve_batch_static: no scratch");
    if (!b || !b->alive) return fail(RVE_EINVAL, "rve_solve_batch_static: invalid batch handle");
    if (b->device != device)
        return fail(RVE_EINVAL, "rve_solve_batch_static: the batch lives on another device than the current one");
    return solve_batch_impl(b, nullptr, nullptr, F, P, A, w_state, status, iters, opts, hip_stream, nullptr, ext_ws,
                            ext_bytes);
}

extern "C" {

int rve_tuning_get(int32_t ndim, int32_t n, rve_tuning* out) {
    if (!out || !(ndim == 2 || ndim == 3) || n < 2) return fail(RVE_EINVAL, "rve_tuning_get: invalid argument");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tuning.find(std::make_pair((int)ndim, (int)n));
    if (it != g_tuning.end()) {
        *out = it->second;
    } else {
        *out = rve_tuning{0, kWaveFrontMaxM, 0, 0, 0.0};
    }
    return RVE_OK;
}

int rve_tuning_set(int32_t ndim, int32_t n, const rve_tuning* t) {
    if (!t || !(ndim == 2 || ndim == 3) || n < 2) return fail(RVE_EINVAL, "rve_tuning_set: invalid argument");
    if (t->leaf < 0 || t->leaf > 4096 || t->wave_max_m < 0 || t->wave_max_m > kWaveFrontMaxM || t->slots < 0 ||
        t->slots > 65536 || !(t->threads == 0 || t->threads == 256 || t->threads == 512))
        return fail(RVE_EINVAL, "rve_tuning_set: value out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuning[std::make_pair((int)ndim, (int)n)] = *t;
    return RVE_OK;
}

int rve_tuning_reset(int32_t ndim, int32_t n) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (n == 0) {
        g_tuning.clear();
    } else {
        g_tuning.erase(std::make_pair((int)ndim, (int)n));
    }
    return RVE_OK;
}

int rve_autotune(rve_mesh m, const double* F, int64_t nF, const rve_opts* o, rve_tuning* best, void* hip_stream) {
    if (!m || !m->alive || !F || nF < 1 || !best) return fail(RVE_EINVAL, "rve_autotune: invalid argument");
    const int d = m->d, n = m->n, d2 = d * d;
    hipStream_t st = (hipStream_t)hip_stream;
    rve_tuning saved{};
    bool had = false;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_tuning.find(std::make_pair(d, n));
        if (it != g_tuning.end()) {
            saved = it->second;
            had = true;
        }
    }
    const std::vector<int> leaves = d == 2 ? std::vector<int>{8, 16, 32} : std::vector<int>{8, 27, 64};
    const std::vector<int> waves = {0, 32, 64};
    const std::vector<int> slots = {512, 1024};
    double *P = nullptr, *A = nullptr;
    int32_t* status = nullptr;
    HIP_OR(hipMalloc((void**)&P, sizeof(double) * d2 * nF));
    HIP_OR(hipMalloc((void**)&A, sizeof(double) * d2 * d2 * nF));
    HIP_OR(hipMalloc((void**)&status, sizeof(int32_t) * nF));
    hipEvent_t e0, e1;
    HIP_OR(hipEventCreate(&e0));
    HIP_OR(hipEventCreate(&e1));
    rve_tuning win{0, kWaveFrontMaxM, 0, 0, 1e300};
    int err = RVE_OK;
    for (int leaf : leaves) {
        // the wave limit matters only where whole fronts fit LDS
        bool lds = false;
        try {
            PlanParams pp;
            pp.leaf = leaf;
            pp.bc = m->bc;
            lds = build_plan(d, n, pp).lds_path;
        } catch (const std::exception& ex) {
            err = fail(RVE_EINVAL, std::string("rve_autotune: ") + ex.what());
            break;
        }
        // eight-wave workgroups exist for 2D plans with fronts in LDS only
        const std::vector<int> threads = lds && d == 2 ? std::vector<int>{256, 512} : std::vector<int>{0};
        for (int wave : waves) {
            if (!lds && wave != kWaveFrontMaxM) continue;
            for (size_t c = 0; c < slots.size() * threads.size() && !err; ++c) {
                const int sl = slots[c / threads.size()], th = threads[c % threads.size()];
                rve_tuning cand{leaf, wave, sl, th, 0.0};
                if ((err = rve_tuning_set(d, n, &cand))) break;
                rve_mesh_desc md{};
                md.ndim = d;
                md.n = n;
                md.nphase = m->nphase;
                md.lame = m->lame.data();
                md.phase = m->phase.data();
                md.law = m->law;
                md.bc = m->bc;
                md.elem = m->elem;
                rve_mesh cm = nullptr;
                if ((err = rve_mesh_create(&md, &cm))) break;
                std::vector<rve_mesh> ms((size_t)nF, cm);
                rve_batch cb = nullptr;
                if ((err = rve_batch_create(ms.data(), nF, &cb))) {
                    rve_mesh_destroy(cm);
                    break;
                }
                float ms_best = 1e30f;
                for (int rep = 0; rep < 2 && !err; ++rep) {  // first run warms up
                    (void)hipEventRecord(e0, st);
                    err = rve_solve_batch(cb, F, P, A, nullptr, status, nullptr, o, hip_stream);
                    (void)hipEventRecord(e1, st);
                    if (hipEventSynchronize(e1) != hipSuccess) err = fail(RVE_EHIP, "rve_autotune: solve failed");
                    float t = 0.f;
                    (void)hipEventElapsedTime(&t, e0, e1);
                    if (rep == 1) ms_best = t;
                }
                rve_batch_destroy(cb);
                rve_mesh_destroy(cm);
                if (err) break;
                if (ms_best < win.ms) win = rve_tuning{leaf, wave, sl, th, (double)ms_best};
            }
            if (err) break;
        }
        if (err) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(P);
    (void)hipFree(A);
    (void)hipFree(status);
    if (err) {
        if (had) rve_tuning_set(d, n, &saved);
        else rve_tuning_reset(d, n);
        return err;
    }
    rve_tuning_set(d, n, &win);
    *best = win;
    return RVE_OK;
}

}  // extern "C"
