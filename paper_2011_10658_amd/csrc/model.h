// Lattice QED on dressed sites: geometry, gauge-invariant local bases,
// site-local operators and the Hamiltonian as a list of product terms.
#pragma once

#include <array>
#include <cstdint>
#include <vector>

#include "common.h"

namespace qed {

// Half-link order of a dressed site: 0:-x 1:-y 2:-z 3:+x 4:+y 5:+z.
struct Lattice {
    int L[3] = {0, 0, 0};
    int bc = QED_BC_OPEN_ZERO_FLUX;
    int N = 0;
    void coords(int s, int c[3]) const {
        c[0] = s % L[0];
        c[1] = (s / L[0]) % L[1];
        c[2] = s / (L[0] * L[1]);
    }
    int index(const int c[3]) const { return c[0] + L[0] * (c[1] + L[1] * c[2]); }
    int parity(int s) const {
        int c[3];
        coords(s, c);
        return (c[0] + c[1] + c[2]) & 1;
    }
    // neighbour across half-link h, or -1 at an open boundary; periodic
    // lattices wrap every axis of extent >= 2 (with extent 2 the wrapped
    // link is a second link between the same two sites)
    int neighbour(int s, int h) const {
        int c[3];
        coords(s, c);
        int a = h % 3;
        c[a] += h >= 3 ? 1 : -1;
        if (bc == QED_BC_PERIODIC && L[a] >= 2) c[a] = (c[a] + L[a]) % L[a];
        if (c[a] < 0 || c[a] >= L[a]) return -1;
        return index(c);
    }
};

// Site-local operator: dense d x d row-major FP64 with a U(1) shift.
struct SiteOp {
    int delta = 0;
    std::vector<double> m;
};

struct Site {
    int parity = 0;
    std::vector<std::array<int8_t, 7>> rows;   // (phi, k_0..k_5), canonical order
    Leg leg;                                   // charge sectors of the basis
    std::vector<SiteOp> ops;                   // op table of this site
    int d() const { return (int)rows.size(); }
};

struct Factor {
    int site;
    int op;   // index into Site::ops
};

enum { CLS_PHYS = 0, CLS_PEN = 1 };

struct Term {
    double coef;
    int cls;
    std::vector<Factor> f;   // sites ascending
};

struct Model {
    Lattice lat;
    double t = 1, m = 1, g2e = 1, g2m = 1;
    std::vector<double> mu;   // local chemical potentials (one per site, or empty)
    std::vector<Site> sites;
    std::vector<Term> terms;
    double offset[2] = {0.0, 0.0};   // constant parts per class
    int nlinks = 0;

    void build();
};

}  // namespace qed
