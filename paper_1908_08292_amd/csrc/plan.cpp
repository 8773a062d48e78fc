// plan.cpp -- symbolic analysis shared by all RVEs of one (d, n).
#include "plan.h"

#include <algorithm>
#include <map>
#include <set>
#include <climits>
#include <cstdint>
#include <stdexcept>

#include "mesh_common.h"

namespace fehmm {
namespace {

struct Box {
    int lo[3], hi[3];
    bool per[3];
};

struct NDBuilder {
    int d, n, leaf;
    std::vector<std::vector<int>> sup;  // supernodes in postorder

    int node_id(const int* c) const {
        int id = 0, s = 1;
        for (int k = 0; k < d; ++k) {
            id += (((c[k] % n) + n) % n) * s;
            s *= n;
        }
        return id;
    }

    std::vector<int> nodes_of(const Box& b) const {
        std::vector<int> out;
        int c[3] = {0, 0, 0};
        int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
        for (int k = 0; k < d; ++k) { lo[k] = b.lo[k]; hi[k] = b.hi[k]; }
        for (c[2] = lo[2]; c[2] < hi[2]; ++c[2])
            for (c[1] = lo[1]; c[1] < hi[1]; ++c[1])
                for (c[0] = lo[0]; c[0] < hi[0]; ++c[0]) out.push_back(node_id(c));
        return out;
    }

    static int64_t volume(const Box& b, int d) {
        int64_t v = 1;
        for (int k = 0; k < d; ++k) v *= std::max(0, b.hi[k] - b.lo[k]);
        return v;
    }

    void rec(const Box& b) {
        int64_t vol = volume(b, d);
        if (vol == 0) return;
        if (vol <= leaf) {
            sup.push_back(nodes_of(b));
            return;
        }
        // cut direction: a periodic direction first, then the longest
        int k = 0;
        auto key = [&](int q) { return std::make_pair(b.per[q] ? 1 : 0, b.hi[q] - b.lo[q]); };
        for (int q = 1; q < d; ++q)
            if (key(q) > key(k)) k = q;
        int size = b.hi[k] - b.lo[k];
        if (b.per[k]) {
            int a = b.lo[k], c = b.lo[k] + size / 2;
            Box b1 = b, b2 = b;
            b1.lo[k] = a + 1; b1.hi[k] = c; b1.per[k] = false;
            b2.lo[k] = c + 1; b2.hi[k] = b.hi[k]; b2.per[k] = false;
            rec(b1);
            rec(b2);
            Box s1 = b, s2 = b;
            s1.lo[k] = a; s1.hi[k] = a + 1; s1.per[k] = false;
            s2.lo[k] = c; s2.hi[k] = c + 1; s2.per[k] = false;
            std::vector<int> sep = nodes_of(s1);
            if (c != a) {
                std::vector<int> t = nodes_of(s2);
                sep.insert(sep.end(), t.begin(), t.end());
            }
            sup.push_back(sep);
        } else {
            int mid = b.lo[k] + size / 2;
            Box b1 = b, b2 = b, s = b;
            b1.hi[k] = mid;
            b2.lo[k] = mid + 1;
            s.lo[k] = mid; s.hi[k] = mid + 1;
            rec(b1);
            rec(b2);
            sup.push_back(nodes_of(s));
        }
    }
};

std::vector<int> periodic_neighbours(int d, int n, int v) {
    int nb = 1;
    for (int k = 0; k < d; ++k) nb *= 3;
    int c[3] = {0, 0, 0}, t = v;
    for (int k = 0; k < d; ++k) { c[k] = t % n; t /= n; }
    std::vector<int> out;
    for (int o = 0; o < nb; ++o) {
        int oo = o, id = 0, s = 1;
        for (int k = 0; k < d; ++k) {
            int dk = oo % 3 - 1;
            oo /= 3;
            id += ((c[k] + dk + n) % n) * s;
            s *= n;
        }
        out.push_back(id);
    }
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
    return out;
}

// parent of every supernode (owner of the earliest node of its structure)
std::vector<int> supernode_parents(int d, int n, const std::vector<std::vector<int>>& sup) {
    int nn = 1;
    for (int k = 0; k < d; ++k) nn *= n;
    const int ns = (int)sup.size();
    std::vector<int> pos(nn, -1), owner(nn, -1), endp(ns);
    int cur = 0;
    for (int s = 0; s < ns; ++s) {
        for (int v : sup[s]) { pos[v] = cur++; owner[v] = s; }
        endp[s] = cur;
    }
    std::vector<std::set<int>> st(ns);
    std::vector<int> parent(ns, -1);
    std::vector<int> node_at(cur);
    for (int v = 0; v < nn; ++v) if (pos[v] >= 0) node_at[pos[v]] = v;
    for (int s = 0; s < ns; ++s) {
        for (int v : sup[s])
            for (int u : periodic_neighbours(d, n, v))
                if (pos[u] >= endp[s]) st[s].insert(pos[u]);
        if (!st[s].empty()) {
            int par = owner[node_at[*st[s].begin()]];
            parent[s] = par;
            for (int q : st[s])
                if (q >= endp[par]) st[par].insert(q);
        }
    }
    return parent;
}

std::vector<std::vector<int>> postorder(const std::vector<std::vector<int>>& sup, const std::vector<int>& parent) {
    const int ns = (int)sup.size();
    std::vector<std::vector<int>> kids(ns);
    std::vector<int> roots;
    for (int s = 0; s < ns; ++s) {
        if (parent[s] < 0) roots.push_back(s);
        else kids[parent[s]].push_back(s);
    }
    std::vector<std::vector<int>> out;
    // iterative DFS: children in their original order, node after its children
    std::vector<std::pair<int, size_t>> stk;
    for (int r : roots) {
        stk.push_back({r, 0});
        while (!stk.empty()) {
            auto& top = stk.back();
            if (top.second < kids[top.first].size()) {
                int c = kids[top.first][top.second++];
                stk.push_back({c, 0});
            } else {
                out.push_back(sup[top.first]);
                stk.pop_back();
            }
        }
    }
    return out;
}

}  // namespace

PlanHost build_plan(int d, int n, const PlanParams& prm) {
    if (!(d == 2 || d == 3) || n < 2) throw std::runtime_error("unsupported mesh size");
    if (prm.leaf < 0 || prm.wave_max_m < 0 || prm.wave_max_m > kWaveFrontMaxM)
        throw std::runtime_error("plan parameters out of range");
    if (prm.bc != 0 && prm.bc != 1) throw std::runtime_error("unknown micro boundary conditions");
    PlanHost P;
    P.d = d;
    P.n = n;
    P.bc = prm.bc;
    int nn = 1;
    for (int k = 0; k < d; ++k) nn *= n;
    P.nnode = nn;
    P.nelem = nn;
    std::vector<char> pinned(nn);
    int nfree_nodes = 0;
    for (int v = 0; v < nn; ++v) {
        pinned[v] = plan_pinned(prm.bc, d, n, v) ? 1 : 0;
        nfree_nodes += pinned[v] ? 0 : 1;
    }
    if (nfree_nodes == 0) throw std::runtime_error("no free node");
    P.nfree = d * nfree_nodes;

    NDBuilder nd{d, n, prm.leaf > 0 ? prm.leaf : (d == 2 ? 16 : 27), {}};
    Box root;
    for (int k = 0; k < 3; ++k) { root.lo[k] = 0; root.hi[k] = (k < d) ? n : 1; root.per[k] = k < d; }
    nd.rec(root);

    // drop the pinned nodes
    std::vector<std::vector<int>> sup0;
    for (auto& s : nd.sup) {
        std::vector<int> t;
        for (int v : s) if (!pinned[v]) t.push_back(v);
        if (!t.empty()) sup0.push_back(t);
    }
    // the supernodal tree of the dissection order, then a depth-first postorder
    // of it, so that each front's children sit on top of the update stack
    std::vector<int> par0 = supernode_parents(d, n, sup0);
    std::vector<std::vector<int>> sup = postorder(sup0, par0);
    const int ns = (int)sup.size();
    std::vector<int> pos(nn, -1), owner(nn, -1), first(ns), endp(ns);
    int cur = 0;
    for (int s = 0; s < ns; ++s) {
        first[s] = cur;
        for (int v : sup[s]) { pos[v] = cur++; owner[v] = s; }
        endp[s] = cur;
    }
    if (cur != nfree_nodes) throw std::runtime_error("nested dissection lost nodes");

    auto neighbours = [&](int v) { return periodic_neighbours(d, n, v); };

    std::vector<int> node_at(nfree_nodes);
    for (int v = 0; v < nn; ++v)
        if (!pinned[v]) node_at[pos[v]] = v;
    auto node_at_pos = [&](int q) { return node_at[q]; };

    // symbolic factorization over supernodes (structures kept as sorted positions)
    std::vector<std::set<int>> st(ns);
    std::vector<int> parent(ns, -1);
    std::vector<std::vector<int>> kids(ns);
    for (int s = 0; s < ns; ++s) {
        for (int v : sup[s])
            for (int u : neighbours(v))
                if (!pinned[u] && pos[u] >= endp[s]) st[s].insert(pos[u]);
        for (int c : kids[s])
            for (int q : st[c])
                if (q >= endp[s]) st[s].insert(q);
        if (!st[s].empty()) {
            int par = owner[node_at_pos(*st[s].begin())];
            parent[s] = par;
            kids[par].push_back(s);
        }
    }
    P.fronts.resize(ns);
    int64_t Loff = 0, top = 0, maxtop = 0, scratch = 0;
    for (int s = 0; s < ns; ++s) {
        FrontHost& F = P.fronts[s];
        int pn = (int)sup[s].size();
        std::vector<int> fnodes(sup[s].begin(), sup[s].end());
        std::sort(fnodes.begin(), fnodes.end(), [&](int a, int b) { return pos[a] < pos[b]; });
        for (int q : st[s]) fnodes.push_back(node_at[q]);
        F.m = (int)fnodes.size() * d;
        F.p = pn * d;
        F.parent = parent[s];
        F.rows_off = (int64_t)P.rows.size();
        for (int v : fnodes)
            for (int k = 0; k < d; ++k) P.rows.push_back(v * d + k);
        // front-local node index
        std::map<int, int> loc;
        for (int i = 0; i < (int)fnodes.size(); ++i) loc[fnodes[i]] = i;
        // children and their relind into this front
        F.child_begin = (int)P.children.size();
        for (int c : kids[s]) P.children.push_back(c);
        F.child_end = (int)P.children.size();
        for (int c : kids[s]) {
            FrontHost& C = P.fronts[c];
            C.relind_off = (int64_t)P.relind.size();
            for (int q : st[c]) {
                auto it = loc.find(node_at[q]);
                if (it == loc.end()) throw std::runtime_error("child structure not in parent front");
                for (int k = 0; k < d; ++k) P.relind.push_back(it->second * d + k);
            }
        }
        // original entries: pivot node a, neighbour b eliminated no earlier than a
        F.kmap_begin = (int)P.kpair.size();
        for (int ia = 0; ia < pn; ++ia) {
            int a = fnodes[ia];
            for (int b : neighbours(a)) {
                if (pinned[b] || pos[b] < pos[a]) continue;
                KPair kp;
                kp.row_node = loc.at(b);
                kp.col_node = ia;
                kp.c_begin = (int)P.kcontrib.size();
                // elements containing a: a is local node la of element (a - offset(la))
                for (int la = 0; la < (1 << d); ++la) {
                    int e = element_of_node(d, n, a, la);
                    int en[8];
                    element_nodes(d, n, e, en);
                    for (int lb = 0; lb < (1 << d); ++lb)
                        if (en[lb] == b) P.kcontrib.push_back(KContrib{e, la, lb, 0});
                }
                kp.c_count = (int)P.kcontrib.size() - kp.c_begin;
                P.kpair.push_back(kp);
            }
        }
        F.kmap_end = (int)P.kpair.size();
        F.asm_begin = (int)P.asm_rc.size();
        {
            const int nen = 1 << d, ndl = nen * d;
            for (int q = F.kmap_begin; q < F.kmap_end; ++q) {
                const KPair& kp = P.kpair[q];
                for (int k = 0; k < d; ++k)
                    for (int l = 0; l < d; ++l) {
                        int r = kp.row_node * d + k, col = kp.col_node * d + l;
                        if (r < col) continue;
                        if (r >= 32768 || col >= 32768) throw std::runtime_error("front too large for the gather list");
                        P.asm_rc.push_back((r << 16) | col);
                        for (int t = 0; t < nen; ++t) {
                            int src = -1;
                            if (t < kp.c_count) {
                                const KContrib& cb = P.kcontrib[kp.c_begin + t];
                                int64_t flat = ((int64_t)cb.elem * ndl + cb.lb * d + k) * ndl + cb.la * d + l;
                                if (flat > INT32_MAX) throw std::runtime_error("element matrix index overflow");
                                src = (int)flat;
                            }
                            P.asm_src.push_back(src);
                        }
                    }
            }
        }
        F.asm_end = (int)P.asm_rc.size();
        // storage
        F.L_off = Loff;
        Loff += (int64_t)F.m * F.p;
        F.D_off = Loff;
        Loff += F.p;
        F.y_off = Loff;
        Loff += (int64_t)F.p * kMaxNrhs;
        int64_t usz = (int64_t)(F.m - F.p) * (F.m - F.p) + (int64_t)(F.m - F.p) * kMaxNrhs;
        scratch = std::max(scratch, usz);
        // update-matrix stack: children are the top entries; U_s replaces them
        if (F.child_end > F.child_begin) {
            int64_t expect = P.fronts[P.children[F.child_begin]].U_off;
            for (int q = F.child_begin; q < F.child_end; ++q) {
                const FrontHost& C = P.fronts[P.children[q]];
                if (C.U_off != expect) throw std::runtime_error("children are not on top of the update stack");
                expect += (int64_t)(C.m - C.p) * (C.m - C.p) + (int64_t)(C.m - C.p) * kMaxNrhs;
            }
            if (expect != top) throw std::runtime_error("update stack out of order");
            top = P.fronts[P.children[F.child_begin]].U_off;
        }
        F.U_off = top;
        top += usz;
        maxtop = std::max(maxtop, top);
        P.max_m = std::max(P.max_m, F.m);
        P.max_p = std::max(P.max_p, F.p);
        for (int j = 0; j < F.p; ++j) {
            double r = F.m - j - 1;
            P.factor_flops += r * (r + 2.0);
            P.nnz_L += F.m - j;
        }
    }
    if (P.fronts.back().parent != -1) throw std::runtime_error("plan root is not last");
    for (int s = 0; s < ns; ++s) {
        FrontHost& F = P.fronts[s];
        F.ea_off = (int64_t)P.ea_dst.size();
        if (F.parent < 0) continue;
        const int mc = F.m - F.p, mp = P.fronts[F.parent].m;
        const int32_t* rel = &P.relind[F.relind_off];
        for (int k = 0; k < mc; ++k)
            for (int i = k; i < mc; ++i) {
                const int64_t R = rel[i], C = rel[k];
                const int64_t off = C * mp - (C * (C - 1)) / 2 + R - C;
                if (off > INT32_MAX) throw std::runtime_error("extend-add offset overflow");
                P.ea_dst.push_back((int32_t)off);
            }
    }
    P.L_size = Loff;
    P.U_stack = maxtop;
    P.U_scratch = scratch;
    // LDS path: whole fronts fit the LDS buffer; then update matrices get static
    // slots (any processing order) and small subtrees run wave-per-front
    {
        const int64_t mm = P.max_m;
        P.lds_path = mm <= 256 && (mm * (mm + 1) / 2 + mm * d * d) * 8 <= kLdsFrontBytes;
    }
    if (P.lds_path) {
        int64_t off = 0;
        for (int s = 0; s < ns; ++s) {
            FrontHost& F = P.fronts[s];
            const int64_t mu = F.m - F.p;
            F.U_off = off;
            off += mu * mu + mu * kMaxNrhs;  // room for either update-matrix format
        }
        P.U_stack = std::max<int64_t>(off, 1);
        int maxh = 0;
        for (int s = 0; s < ns; ++s) {
            FrontHost& F = P.fronts[s];
            F.wave = F.m <= prm.wave_max_m ? 1 : 0;
            F.height = 0;
            for (int q = F.child_begin; q < F.child_end; ++q) {
                const FrontHost& C = P.fronts[P.children[q]];
                if (!C.wave) F.wave = 0;
                F.height = std::max(F.height, C.height + 1);
            }
            if (F.wave) {
                maxh = std::max(maxh, F.height);
                // packed front, rhs rows, original diagonal (m <= 64) within the 256 spare
                P.wave_slice = std::max<int64_t>(P.wave_slice, (int64_t)F.m * (F.m + 1) / 2 + (int64_t)F.m * d * d + 256);
            }
        }
        for (int h = 0; h <= maxh; ++h) {
            P.wave_hbeg.push_back((int32_t)P.wave_list.size());
            for (int s = 0; s < ns; ++s)
                if (P.fronts[s].wave && P.fronts[s].height == h) P.wave_list.push_back(s);
        }
        P.wave_hbeg.push_back((int32_t)P.wave_list.size());
        P.wave_slice = (P.wave_slice + 31) / 32 * 32;
        // workgroup fronts by height (children first).  Fronts of one height are
        // independent; with equal p and child counts they pass the same barriers,
        // so up to kStepFronts of them can share a step (each on a group of at
        // least 128 threads, one per front row: m <= 128) when together they fit
        // the front region: the packed fronts with their rhs rows and diagonals,
        // and in the backward substitution the staged panels with their FP64
        // scratch (d^2 m + 3 p doubles, i.e. twice as many FP32 elements).
        // (rhs rows: d^2 + 1 columns in 2D, where the last Newton factorization
        // and its backward substitution carry the condensation's columns beside
        // the residual; then the original diagonal)
        const int64_t rr = d * d + (d == 2 ? 2 : 1);
        const int64_t mm = P.max_m, region = mm * (mm + 1) / 2 + mm * rr;
        auto fneed = [&](const FrontHost& X) { return (int64_t)X.m * (X.m + 1) / 2 + (int64_t)X.m * rr; };
        const int64_t bc = d * d + (d == 2 ? 1 : 0);  // backward-substituted columns
        auto bneed = [&](const FrontHost& X) {
            return (int64_t)X.p * X.m - (int64_t)X.p * (X.p - 1) / 2 + 2 * (bc * X.m + 3 * (int64_t)X.p) + 1;
        };
        int hmax = 0;
        for (const FrontHost& F : P.fronts) hmax = std::max(hmax, F.height);
        for (int h = 0; h <= hmax; ++h) {
            std::vector<int> lst;
            for (int s = 0; s < ns; ++s)
                if (!P.fronts[s].wave && P.fronts[s].height == h) lst.push_back(s);
            std::vector<char> used(lst.size(), 0);
            for (size_t a = 0; a < lst.size(); ++a) {
                if (used[a]) continue;
                used[a] = 1;
                const FrontHost& A = P.fronts[lst[a]];
                std::vector<int> grp = {lst[a]};
                int64_t fsum = fneed(A), bsum = bneed(A);
                for (size_t b = a + 1; b < lst.size() && A.m <= 128 && (int)grp.size() < kStepFronts; ++b) {
                    const FrontHost& Bf = P.fronts[lst[b]];
                    if (!used[b] && Bf.m <= 128 && Bf.p == A.p &&
                        Bf.child_end - Bf.child_begin == A.child_end - A.child_begin &&
                        fsum + fneed(Bf) <= region && bsum + bneed(Bf) <= region) {
                        grp.push_back(lst[b]);
                        fsum += fneed(Bf);
                        bsum += bneed(Bf);
                        used[b] = 1;
                    }
                }
                // 1, 2 or 4 fronts per step (the kernel splits the workgroup evenly)
                while (grp.size() == 3) {
                    used[std::find(lst.begin(), lst.end(), grp.back()) - lst.begin()] = 0;
                    grp.pop_back();
                }
                for (int k = 0; k < kStepFronts; ++k) P.wg_steps.push_back(k < (int)grp.size() ? grp[k] : -1);
            }
        }
    }
    return P;
}

}  // namespace fehmm
