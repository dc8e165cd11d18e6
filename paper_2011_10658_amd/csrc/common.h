// Shared host-side definitions of the qedttn library.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/qedttn.h"

namespace qed {

// Error carried across internal calls and turned into a status code at
// the C boundary.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

// One tree leg: strictly ascending charges, sizes > 0.
struct Leg {
    std::vector<int> q;
    std::vector<int> n;
    int nsec() const { return (int)q.size(); }
    int dim() const {
        int d = 0;
        for (int v : n) d += v;
        return d;
    }
    // sector index of charge c, or -1
    int find(int c) const {
        int lo = 0, hi = (int)q.size() - 1;
        while (lo <= hi) {
            int mid = (lo + hi) / 2;
            if (q[mid] == c) return mid;
            if (q[mid] < c) lo = mid + 1; else hi = mid - 1;
        }
        return -1;
    }
    bool operator==(const Leg& o) const { return q == o.q && n == o.n; }
};

// Allowed blocks of a three-leg tensor, canonical order: (q_l, q_r)
// ascending, q_p = q_l + q_r - flux must be a sector of p.
struct BlockTable {
    std::vector<int> s[3];          // sector indices per leg
    std::vector<int64_t> off;       // nblk + 1 prefix sums
    int nblk() const { return (int)s[0].size(); }
    int64_t size() const { return off.empty() ? 0 : off.back(); }
};

inline BlockTable make_table(const Leg& l, const Leg& r, const Leg& p, int flux) {
    BlockTable t;
    t.off.push_back(0);
    for (int a = 0; a < l.nsec(); ++a)
        for (int b = 0; b < r.nsec(); ++b) {
            int c = p.find(l.q[a] + r.q[b] - flux);
            if (c < 0) continue;
            t.s[0].push_back(a);
            t.s[1].push_back(b);
            t.s[2].push_back(c);
            t.off.push_back(t.off.back() + (int64_t)l.n[a] * r.n[b] * p.n[c]);
        }
    return t;
}

// Packed layout of a block-sparse operator on one leg with charge shift
// delta: one dense row-major (n_out x n_in) block per input sector whose
// shifted charge exists, in ascending input order.
struct OpLayout {
    int delta = 0;
    std::vector<int> out_of_in;     // per input sector: output sector or -1
    std::vector<int64_t> off;       // per input sector: offset or -1
    int64_t size = 0;
};

inline OpLayout make_op_layout(const Leg& leg, int delta) {
    OpLayout L;
    L.delta = delta;
    L.out_of_in.assign(leg.nsec(), -1);
    L.off.assign(leg.nsec(), -1);
    for (int s = 0; s < leg.nsec(); ++s) {
        int o = leg.find(leg.q[s] + delta);
        if (o < 0) continue;
        L.out_of_in[s] = o;
        L.off[s] = L.size;
        L.size += (int64_t)leg.n[o] * leg.n[s];
    }
    return L;
}

}  // namespace qed
