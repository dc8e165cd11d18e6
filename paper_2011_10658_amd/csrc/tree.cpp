// Tree geometry and leg-sector allocation.
//
// Sector rule (the paper draws the sector distribution at random; this
// deterministic rule lets independent implementations agree bit for bit):
//  * dS(q): number of product states of the subtree with charge q, dC(q)
//    the same for the complement; saturating int64 counts (cap 2^62).
//  * charge q is allowed on a link if dS(q) > 0 and dC(Q - q) > 0;
//    cap(q) = min(dS(q), dC(Q - q)) (Schmidt-rank bound).
//  * if sum cap <= chi the link is exact; otherwise chi is split with
//    weights W(q) = floor(2^30 w(q)/max w + 1/2), w(q) = pS(q) pC(Q-q),
//    pS/pC the charge distributions of uniformly drawn product states
//    (binary64 convolutions, charges ascending, subtree / complement as
//    the left operand), by integer largest remainder (ties: smaller
//    |q N - Q |S||, then smaller q), freezing charges at their cap and
//    re-splitting the rest.
//  * consistency with every QR of a node toward a leg (the sector must not
//    be wider than its rows), enforced by min-passes to the fixed point.
#include "tree.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>

#pragma clang fp contract(off)

namespace qed {

void Tree::build(const Lattice& lat) {
    N = lat.N;
    if (N < 2) fail(QED_ERR_INVALID_ARG, "the lattice needs at least two sites");
    struct Blk { int o[3]; int sz[3]; int link; };
    std::vector<Blk> blocks;
    for (int k = 0; k < lat.L[2]; ++k)
        for (int j = 0; j < lat.L[1]; ++j)
            for (int i = 0; i < lat.L[0]; ++i) {
                int c[3] = {i, j, k};
                blocks.push_back(Blk{{i, j, k}, {1, 1, 1}, lat.index(c)});
            }
    nodes.clear();
    sites_of.assign(N, {});
    for (int s = 0; s < N; ++s) sites_of[s] = {s};
    int axis = 0, layer = 0;
    while (blocks.size() > 1) {
        for (int t = 0; t < 3; ++t) {
            if (blocks[0].sz[axis] < lat.L[axis]) break;
            axis = (axis + 1) % 3;
        }
        int a = axis;
        std::map<std::array<int, 3>, int> byorig;
        for (int b = 0; b < (int)blocks.size(); ++b)
            byorig[{blocks[b].o[0], blocks[b].o[1], blocks[b].o[2]}] = b;
        std::vector<Blk> nb;
        for (const Blk& b : blocks) {
            if (b.o[a] % (2 * b.sz[a])) continue;
            std::array<int, 3> o2 = {b.o[0], b.o[1], b.o[2]};
            o2[a] += b.sz[a];
            const Blk& b2 = blocks[byorig.at(o2)];
            int nid = (int)nodes.size();
            int link = N + nid;
            Node nd;
            nd.l = b.link;
            nd.r = b2.link;
            nd.p = link;
            nd.layer = layer;
            for (int t = 0; t < 3; ++t) nd.origin[t] = b.o[t];
            nodes.push_back(nd);
            std::vector<int> st = sites_of[b.link];
            st.insert(st.end(), sites_of[b2.link].begin(), sites_of[b2.link].end());
            std::sort(st.begin(), st.end());
            sites_of.push_back(st);
            Blk n2 = b;
            n2.sz[a] *= 2;
            n2.link = link;
            nb.push_back(n2);
        }
        std::sort(nb.begin(), nb.end(), [](const Blk& x, const Blk& y) {
            if (x.o[2] != y.o[2]) return x.o[2] < y.o[2];
            if (x.o[1] != y.o[1]) return x.o[1] < y.o[1];
            return x.o[0] < y.o[0];
        });
        blocks = nb;
        axis = (a + 1) % 3;
        ++layer;
    }
    root = (int)nodes.size() - 1;
    top = N + root;
    parent_node.assign(nlinks(), -1);
    parent_side.assign(nlinks(), -1);
    for (int n = 0; n < (int)nodes.size(); ++n) {
        parent_node[nodes[n].l] = n;
        parent_side[nodes[n].l] = 0;
        parent_node[nodes[n].r] = n;
        parent_side[nodes[n].r] = 1;
    }
}

std::vector<int> Tree::path(int a, int b) const {
    auto anc = [&](int n) {
        std::vector<int> out = {n};
        while (n != root) {
            n = parent_node[nodes[n].p];
            out.push_back(n);
        }
        return out;
    };
    std::vector<int> pa = anc(a), pb = anc(b);
    int lca = -1;
    size_t ia = 0, ib = 0;
    for (ia = 0; ia < pa.size(); ++ia) {
        auto it = std::find(pb.begin(), pb.end(), pa[ia]);
        if (it != pb.end()) {
            lca = pa[ia];
            ib = it - pb.begin();
            break;
        }
    }
    std::vector<int> out(pa.begin(), pa.begin() + ia + 1);
    for (size_t k = ib; k-- > 0;) out.push_back(pb[k]);
    (void)lca;
    return out;
}

namespace {

const int64_t SAT = (int64_t)1 << 62;

using IMap = std::map<int, int64_t>;
using FMap = std::map<int, double>;

int64_t sat_mul(int64_t a, int64_t b) {
    if (a == 0 || b == 0) return 0;
    if (a > SAT / b) return SAT;
    return std::min(SAT, a * b);
}

IMap conv_int(const IMap& a, const IMap& b) {
    IMap out;
    for (auto& x : a)
        for (auto& y : b) {
            int64_t v = sat_mul(x.second, y.second);
            int64_t& o = out[x.first + y.first];
            o = (o > SAT - v) ? SAT : o + v;
        }
    return out;
}

FMap conv_float(const FMap& a, const FMap& b) {
    std::vector<int> keys;
    for (auto& x : a)
        for (auto& y : b) keys.push_back(x.first + y.first);
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    FMap out;
    for (int q : keys) {
        double acc = 0.0;
        for (auto& x : a) {
            auto it = b.find(q - x.first);
            if (it == b.end()) continue;
            double prod = x.second * it->second;
            acc = acc + prod;
        }
        out[q] = acc;
    }
    return out;
}

}  // namespace

std::vector<Leg> allocate_sectors(const Tree& tree, const std::vector<Leg>& site_legs, int Q,
                                  int chi) {
    const int N = tree.N;
    const int nl = tree.nlinks();
    std::vector<IMap> dS(nl), dC(nl);
    std::vector<FMap> pS(nl), pC(nl);
    for (int s = 0; s < N; ++s) {
        const Leg& g = site_legs[s];
        int64_t tot = 0;
        for (int v : g.n) tot += v;
        for (int i = 0; i < g.nsec(); ++i) {
            dS[s][g.q[i]] = g.n[i];
            pS[s][g.q[i]] = (double)g.n[i] / (double)tot;
        }
    }
    for (const auto& nd : tree.nodes) {
        dS[nd.p] = conv_int(dS[nd.l], dS[nd.r]);
        pS[nd.p] = conv_float(pS[nd.l], pS[nd.r]);
    }
    dC[tree.top] = {{0, 1}};
    pC[tree.top] = {{0, 1.0}};
    for (int n = (int)tree.nodes.size() - 1; n >= 0; --n) {
        const auto& nd = tree.nodes[n];
        dC[nd.l] = conv_int(dC[nd.p], dS[nd.r]);
        pC[nd.l] = conv_float(pC[nd.p], pS[nd.r]);
        dC[nd.r] = conv_int(dC[nd.p], dS[nd.l]);
        pC[nd.r] = conv_float(pC[nd.p], pS[nd.l]);
    }
    std::vector<Leg> legs(nl);
    for (int s = 0; s < N; ++s) legs[s] = site_legs[s];
    legs[tree.top].q = {Q};
    legs[tree.top].n = {1};
    for (const auto& nd : tree.nodes) {
        const int e = nd.p;
        if (e == tree.top) continue;
        std::vector<int> qs;
        std::map<int, int64_t> cap;
        for (auto& x : dS[e]) {
            auto it = dC[e].find(Q - x.first);
            if (x.second > 0 && it != dC[e].end() && it->second > 0) {
                qs.push_back(x.first);
                cap[x.first] = std::min(x.second, it->second);
            }
        }
        int64_t capsum = 0;
        for (int q : qs) capsum = (capsum > SAT - cap[q]) ? SAT : capsum + cap[q];
        Leg leg;
        if (capsum <= chi) {
            for (int q : qs) {
                leg.q.push_back(q);
                leg.n.push_back((int)cap[q]);
            }
            legs[e] = leg;
            continue;
        }
        std::map<int, double> w;
        double wmax = 0.0;
        for (int q : qs) {
            w[q] = pS[e][q] * pC[e][Q - q];
            wmax = std::max(wmax, w[q]);
        }
        std::map<int, int64_t> W;
        for (int q : qs) {
            double scaled = w[q] / wmax * 1073741824.0 + 0.5;
            W[q] = (int64_t)std::floor(scaled);
        }
        const int64_t size = (int64_t)tree.sites_of[e].size();
        auto tie = [&](int q) { return std::llabs((int64_t)q * N - (int64_t)Q * size); };
        std::map<int, int64_t> alloc_final;
        std::vector<int> freeq;
        for (int q : qs)
            if (cap[q] > 0 && W[q] > 0) freeq.push_back(q);
        int64_t budget = chi;
        while (!freeq.empty() && budget > 0) {
            int64_t wsum = 0;
            for (int q : freeq) wsum += W[q];
            std::map<int, int64_t> al, rem;
            int64_t used = 0;
            for (int q : freeq) {
                al[q] = budget * W[q] / wsum;
                rem[q] = budget * W[q] % wsum;
                used += al[q];
            }
            int64_t left = budget - used;
            std::vector<int> order = freeq;
            std::sort(order.begin(), order.end(), [&](int a, int b) {
                if (rem[a] != rem[b]) return rem[a] > rem[b];
                if (tie(a) != tie(b)) return tie(a) < tie(b);
                return a < b;
            });
            for (int64_t i = 0; i < left; ++i) al[order[i]] += 1;
            std::vector<int> over;
            for (int q : freeq)
                if (al[q] >= cap[q]) over.push_back(q);
            if (over.empty()) {
                for (int q : freeq) alloc_final[q] = al[q];
                break;
            }
            for (int q : over) {
                alloc_final[q] = cap[q];
                budget -= cap[q];
                freeq.erase(std::find(freeq.begin(), freeq.end(), q));
            }
        }
        for (auto& x : alloc_final)
            if (x.second > 0) {
                leg.q.push_back(x.first);
                leg.n.push_back((int)x.second);
            }
        legs[e] = leg;
    }
    // consistency with the QR of every node toward each of its legs
    auto rows_sum = [](const Leg& A, const Leg& B, int q, int sgnA, int sgnB) {
        // sum over sectors a of A, b of B with sgnA qa + sgnB qb = q
        int64_t s = 0;
        for (int i = 0; i < A.nsec(); ++i) {
            int need = (q - sgnA * A.q[i]) * sgnB;  // sgnB = +-1
            int j = B.find(need);
            if (j >= 0) s += (int64_t)A.n[i] * B.n[j];
        }
        return s;
    };
    bool changed = true;
    while (changed) {
        changed = false;
        for (const auto& nd : tree.nodes) {
            const Leg L0 = legs[nd.l], R0 = legs[nd.r], P0 = legs[nd.p];
            Leg nL, nR, nP;
            for (int i = 0; i < P0.nsec(); ++i) {
                int64_t v = std::min<int64_t>(P0.n[i], rows_sum(L0, R0, P0.q[i], 1, 1));
                if (v > 0) { nP.q.push_back(P0.q[i]); nP.n.push_back((int)v); }
            }
            for (int i = 0; i < L0.nsec(); ++i) {
                // q_l = q_p - q_r: rows over (r, p) with q_p - q_r = q
                int64_t v = std::min<int64_t>(L0.n[i], rows_sum(R0, P0, L0.q[i], -1, 1));
                if (v > 0) { nL.q.push_back(L0.q[i]); nL.n.push_back((int)v); }
            }
            for (int i = 0; i < R0.nsec(); ++i) {
                int64_t v = std::min<int64_t>(R0.n[i], rows_sum(L0, P0, R0.q[i], -1, 1));
                if (v > 0) { nR.q.push_back(R0.q[i]); nR.n.push_back((int)v); }
            }
            if (nd.l >= N && !(nL == legs[nd.l])) { legs[nd.l] = nL; changed = true; }
            if (nd.r >= N && !(nR == legs[nd.r])) { legs[nd.r] = nR; changed = true; }
            if (nd.p >= N && !(nP == legs[nd.p])) { legs[nd.p] = nP; changed = true; }
        }
    }
    return legs;
}

}  // namespace qed
