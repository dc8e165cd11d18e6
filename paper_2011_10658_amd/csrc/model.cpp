// Dressed-site lattice QED model (arXiv:2011.10658, Results Eq. 1 and the
// Methods sections on the fermionic compact representation and on the
// link penalty).
//
// Local basis: (phi, k_0..k_5) with phi + sum k = 6 + p (Gauss law in
// rishon form), lexicographic order, sign factor
// sigma = (-1)^{[k_0=2] + [k_1=2] + [k_2=2]} on the negative half-links.
// Operators are written down directly from the mode algebra:
//   psi lowers phi (first mode of the site, no string sign);
//   eta^dag_j raises k_j by one with unit amplitude and the string sign
//   (-1)^{phi + sum_{i<j} k_i} of the modes placed before half-link j;
//   eta_j is its transpose.
// Hamiltonian terms (products of site-local matrices):
//   hopping   -t (M^dag_{x,+mu} M_{x+mu,-mu} + h.c.),   M_j = eta^dag_j psi
//   plaquette box = -C_A C_B C_C C_D with C = eta^dag eta on the four
//             corners; -(g_m^2/2)(box + box^dag)
//   onsite    m (-1)^x phi + (g_e^2/2) sum (1 - k_{+mu})^2 over the
//             site's +mu links (+ dangling half-links under free flux)
//             [+ mu_x phi with local chemical potentials]
//   penalty   nu (1 - sum_a P^a_{x,+mu} P^{2-a}_{x+mu,-mu}) per link, built
//             as nu sum_a P^a_{x,+mu} (1 - P^{2-a}_{x+mu,-mu}) (equal, since
//             sum_a P^a = 1): three nonnegative terms that vanish on links
//             obeying the rishon constraint, and no constant part, so no
//             large cancellation is left to the reduced-precision GEMMs.
#include "model.h"

#include <algorithm>
#include <map>

namespace qed {

namespace {

int encode(const std::array<int8_t, 7>& r) {
    int v = r[0];
    for (int j = 1; j < 7; ++j) v = v * 3 + r[j];
    return v;
}

void build_site(Site& st, int parity, const bool present[6], int bc) {
    st.parity = parity;
    st.rows.clear();
    for (int phi = 0; phi <= 1; ++phi)
        for (int code = 0; code < 729; ++code) {
            std::array<int8_t, 7> r;
            r[0] = (int8_t)phi;
            int c = code, sum = phi;
            // most significant digit first -> lexicographic enumeration
            for (int j = 6; j >= 1; --j) {
                r[j] = (int8_t)(c % 3);
                c /= 3;
            }
            bool ok = true;
            for (int j = 0; j < 6; ++j) {
                sum += r[1 + j];
                if (bc != QED_BC_OPEN_FREE_FLUX && !present[j] && r[1 + j] != 1) ok = false;
            }
            if (ok && sum == 6 + parity) st.rows.push_back(r);
        }
    // sectors: phi = 0 rows first (charge -p), then phi = 1 (charge 1 - p)
    st.leg.q.clear();
    st.leg.n.clear();
    for (auto& r : st.rows) {
        int q = r[0] - parity;
        if (st.leg.q.empty() || st.leg.q.back() != q) {
            st.leg.q.push_back(q);
            st.leg.n.push_back(0);
        }
        st.leg.n.back()++;
    }
}

struct SiteBuilder {
    Site& st;
    std::map<int, int> idx;
    explicit SiteBuilder(Site& s) : st(s) {
        for (int i = 0; i < s.d(); ++i) idx[encode(s.rows[i])] = i;
    }
    int d() const { return st.d(); }
    int sigma(const std::array<int8_t, 7>& r) const {
        int e = (r[1] == 2) + (r[2] == 2) + (r[3] == 2);
        return (e & 1) ? -1 : 1;
    }
    int find(const std::array<int8_t, 7>& r) const {
        auto it = idx.find(encode(r));
        return it == idx.end() ? -1 : it->second;
    }
    // string sign of the modes before half-link j
    static int string_sign(const std::array<int8_t, 7>& r, int j) {
        int s = r[0];
        for (int i = 0; i < j; ++i) s += r[1 + i];
        return (s & 1) ? -1 : 1;
    }
    int add(SiteOp op) {
        st.ops.push_back(std::move(op));
        return (int)st.ops.size() - 1;
    }
    SiteOp zero(int delta) const {
        SiteOp o;
        o.delta = delta;
        o.m.assign((size_t)d() * d(), 0.0);
        return o;
    }
    // M_j = eta^dag_j psi
    int M(int j) {
        SiteOp o = zero(-1);
        for (int s = 0; s < d(); ++s) {
            auto r = st.rows[s];
            if (r[0] != 1 || r[1 + j] >= 2) continue;
            auto r2 = r;
            r2[0] = 0;               // psi: first mode, no string sign
            int sg = string_sign(r2, j);
            r2[1 + j] += 1;          // eta^dag_j on the phi = 0 state
            int t = find(r2);
            if (t < 0) continue;     // frozen boundary half-link
            o.m[(size_t)t * d() + s] = sigma(r) * sigma(r2) * sg;
        }
        return add(o);
    }
    int transpose(int id, int delta) {
        SiteOp o = zero(delta);
        const auto& a = st.ops[id].m;
        for (int i = 0; i < d(); ++i)
            for (int k = 0; k < d(); ++k) o.m[(size_t)k * d() + i] = a[(size_t)i * d() + k];
        return add(o);
    }
    // C_ij = eta^dag_i eta_j  (i != j)
    int C(int i, int j) {
        SiteOp o = zero(0);
        for (int s = 0; s < d(); ++s) {
            auto r = st.rows[s];
            if (r[1 + j] == 0) continue;
            auto r1 = r;
            r1[1 + j] -= 1;
            int sg1 = string_sign(r1, j);   // prefix of the lower state
            if (r1[1 + i] >= 2) continue;
            int sg2 = string_sign(r1, i);
            auto r2 = r1;
            r2[1 + i] += 1;
            int t = find(r2);
            if (t < 0) continue;
            o.m[(size_t)t * d() + s] = sigma(r) * sigma(r2) * sg1 * sg2;
        }
        return add(o);
    }
    int proj(int j, int a) {
        SiteOp o = zero(0);
        for (int s = 0; s < d(); ++s)
            if (st.rows[s][1 + j] == a) o.m[(size_t)s * d() + s] = 1.0;
        return add(o);
    }
    int notproj(int j, int a) {   // 1 - P^a on half-link j
        SiteOp o = zero(0);
        for (int s = 0; s < d(); ++s)
            if (st.rows[s][1 + j] != a) o.m[(size_t)s * d() + s] = 1.0;
        return add(o);
    }
};

}  // namespace

void Model::build() {
    const Lattice& L = lat;
    if (L.bc != QED_BC_OPEN_ZERO_FLUX && L.bc != QED_BC_OPEN_FREE_FLUX && L.bc != QED_BC_PERIODIC)
        fail(QED_ERR_INVALID_ARG, "unknown boundary condition");
    sites.assign(L.N, Site());
    terms.clear();
    offset[0] = offset[1] = 0.0;
    nlinks = 0;
    std::vector<SiteBuilder*> sb;
    // per-site operator ids
    std::vector<std::array<int, 6>> Mid(L.N), Mdid(L.N);
    std::vector<std::array<std::array<int, 6>, 6>> Cid(L.N);
    std::vector<std::array<std::array<int, 3>, 6>> Pid(L.N), Nid(L.N);
    std::vector<int> Hid(L.N);
    std::vector<SiteBuilder> builders;
    builders.reserve(L.N);
    for (int s = 0; s < L.N; ++s) {
        bool present[6];
        for (int h = 0; h < 6; ++h) present[h] = L.neighbour(s, h) >= 0;
        build_site(sites[s], L.parity(s), present, L.bc);
        builders.emplace_back(sites[s]);
        SiteBuilder& b = builders.back();
        const int p = sites[s].parity;
        // onsite diagonal: staggered mass + electric energy
        SiteOp h = b.zero(0);
        for (int i = 0; i < b.d(); ++i) {
            const auto& r = sites[s].rows[i];
            double v = m * (1 - 2 * p) * r[0];
            if (!mu.empty()) v += mu[s] * r[0];
            for (int j = 0; j < 6; ++j) {
                double E = 1.0 - r[1 + j];
                if ((j >= 3 && present[j]) || (L.bc == QED_BC_OPEN_FREE_FLUX && !present[j]))
                    v += 0.5 * g2e * E * E;
            }
            h.m[(size_t)i * b.d() + i] = v;
        }
        Hid[s] = b.add(h);
        for (int j = 0; j < 6; ++j) {
            Mid[s][j] = Mdid[s][j] = -1;
            for (int a = 0; a < 3; ++a) Pid[s][j][a] = Nid[s][j][a] = -1;
            for (int i = 0; i < 6; ++i) Cid[s][i][j] = -1;
            if (!present[j]) continue;
            Mid[s][j] = b.M(j);
            Mdid[s][j] = b.transpose(Mid[s][j], +1);
            for (int a = 0; a < 3; ++a) {
                if (j >= 3) Pid[s][j][a] = b.proj(j, a);
                else Nid[s][j][a] = b.notproj(j, a);
            }
        }
    }
    auto Cop = [&](int s, int i, int j) {
        if (Cid[s][i][j] < 0) Cid[s][i][j] = builders[s].C(i, j);
        return Cid[s][i][j];
    };
    auto cop_t = [&](int s, int id) { return builders[s].transpose(id, 0); };
    auto two = [&](double c, int cls, int s1, int o1, int s2, int o2) {
        Term t;
        t.coef = c;
        t.cls = cls;
        if (s1 < s2) t.f = {{s1, o1}, {s2, o2}};
        else t.f = {{s2, o2}, {s1, o1}};
        terms.push_back(t);
    };
    for (int s = 0; s < L.N; ++s) terms.push_back(Term{1.0, CLS_PHYS, {{s, Hid[s]}}});
    // hopping: psi^dag_x U_{x,mu} psi_y = M^dag_{x,+mu} M_{y,-mu}
    for (int x = 0; x < L.N; ++x)
        for (int mu = 0; mu < 3; ++mu) {
            int y = L.neighbour(x, 3 + mu);
            if (y < 0) continue;
            ++nlinks;
            two(-t, CLS_PHYS, x, Mdid[x][3 + mu], y, Mid[y][mu]);
            two(-t, CLS_PHYS, y, Mdid[y][mu], x, Mid[x][3 + mu]);
        }
    // plaquettes
    for (int x = 0; x < L.N; ++x)
        for (int al = 0; al < 3; ++al)
            for (int be = al + 1; be < 3; ++be) {
                int xa = L.neighbour(x, 3 + al), xb = L.neighbour(x, 3 + be);
                if (xa < 0 || xb < 0) continue;
                int xab = L.neighbour(xa, 3 + be);
                if (xab < 0) continue;
                int cA = Cop(x, 3 + be, 3 + al);
                int cB = Cop(xa, al, 3 + be);
                int cC = Cop(xab, be, al);
                int cD = Cop(xb, 3 + al, be);
                std::vector<Factor> f = {{x, cA}, {xa, cB}, {xab, cC}, {xb, cD}};
                std::vector<Factor> fd = {{x, cop_t(x, cA)}, {xa, cop_t(xa, cB)},
                                          {xab, cop_t(xab, cC)}, {xb, cop_t(xb, cD)}};
                auto by_site = [](const Factor& a, const Factor& b) { return a.site < b.site; };
                std::sort(f.begin(), f.end(), by_site);
                std::sort(fd.begin(), fd.end(), by_site);
                // -(g_m^2/2)(box + box^dag) with box = -C_A C_B C_C C_D
                terms.push_back(Term{0.5 * g2m, CLS_PHYS, f});
                terms.push_back(Term{0.5 * g2m, CLS_PHYS, fd});
            }
    // penalty: sum_a P^a(x,+mu) (1 - P^{2-a}(y,-mu)) = 1 - sum_a P^a P^{2-a}
    for (int x = 0; x < L.N; ++x)
        for (int mu = 0; mu < 3; ++mu) {
            int y = L.neighbour(x, 3 + mu);
            if (y < 0) continue;
            for (int a = 0; a < 3; ++a) two(1.0, CLS_PEN, x, Pid[x][3 + mu][a], y, Nid[y][mu][2 - a]);
        }
}

}  // namespace qed
