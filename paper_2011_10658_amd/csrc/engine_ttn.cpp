// Tree tensor network ground-state sweep on the device (Methods, "Tensor
// Networks": single-tensor optimisation from the lowest to the highest
// layer; "Numerical Convergence": driven penalty nu).
//
// Environments.  For every tree link and each of its two sides the engine
// keeps the operators of that side in the basis of the link: one block
// Hamiltonian per class (physics, penalty with unit coefficient) holding
// every term inside the side, and the open factor of every term that
// straddles the link.  They are rebuilt whenever the isometry centre moves
// across the link (renormalisation with the fresh isometry).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "engine.h"

namespace qed {

constexpr double LZ_TOL_FLOOR_FP32 = 2e-6;
// BF16 operands carry 8 significant bits (unit roundoff u = 2^-9): a
// matvec is accurate to a few u relative, and Krylov residuals stall near
// that level; the floor is 2u
constexpr double LZ_TOL_FLOOR_BF16 = 3.9e-3;
// with the FP64 residual correction (refine >= 2) the residual is exact at
// every restart; the floors are those that carry the energy to well below
// 1e-8 relative (the energy error is second order in the residual)
constexpr double LZ_TOL_FLOOR_FIX_FP32 = 1e-8;
constexpr double LZ_TOL_FLOOR_FIX_BF16 = 1e-6;

namespace {

uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

double sym_uniform(uint64_t key, uint64_t i) {
    uint64_t w = mix64(key + (i + 1) * 0x9E3779B97F4A7C15ULL);
    double u = (double)(w >> 11) * (1.0 / 9007199254740992.0);
    return 2.0 * u - 1.0;
}

}  // namespace

void Engine::build(Ctx* c) {
    ctx = c;
    const Params& P = c->prm;
    model = Model();
    model.lat.L[0] = P.Lx;
    model.lat.L[1] = P.Ly;
    model.lat.L[2] = P.Lz;
    model.lat.bc = P.bc;
    model.lat.N = P.Lx * P.Ly * P.Lz;
    model.t = P.t;
    model.m = P.m;
    model.g2e = P.g2e;
    model.g2m = P.g2m;
    model.mu = P.mu;
    model.build();
    if (P.bc != QED_BC_OPEN_FREE_FLUX && P.Q != 0)
        fail(QED_ERR_INVALID_ARG, "zero-flux and periodic boundaries admit only total charge Q = 0");
    tree = Tree();
    tree.build(model.lat);
    std::vector<Leg> sl;
    for (auto& s : model.sites) sl.push_back(s.leg);
    legs = allocate_sectors(tree, sl, P.Q, P.chi);
    alloc_legs = legs;
    // the charge sector must be reachable: every leg non-empty
    for (int e = 0; e < tree.nlinks(); ++e)
        if (legs[e].nsec() == 0)
            fail(QED_ERR_INVALID_ARG, "the total charge is not reachable on this lattice");
    for (const auto& nd : tree.nodes) {
        BlockTable t = make_table(legs[nd.l], legs[nd.r], legs[nd.p], 0);
        if (t.nblk() == 0) fail(QED_ERR_INVALID_ARG, "a tree node has no allowed block");
    }
    const int N = tree.N;
    inside.assign(tree.nlinks(), std::vector<char>(N, 0));
    for (int e = 0; e < tree.nlinks(); ++e)
        for (int s : tree.sites_of[e]) inside[e][s] = 1;
    tsites.clear();
    for (const Term& t : model.terms) {
        std::vector<int> s;
        for (const Factor& f : t.f) s.push_back(f.site);
        tsites.push_back(s);
    }
    nodes.clear();
    siteops.clear();
    up.assign(tree.nlinks(), EnvD());
    dn.assign(tree.nlinks(), EnvD());
    centre = -1;
    sweeps_done = 0;
    sweep_energies.clear();
    have_energy = false;
}

void Engine::init_nodes(uint64_t seed) {
    Dev* dev = &ctx->dev;
    legs = alloc_legs;
    n_expand = 0;
    last_updated = -1;
    nodes.assign(tree.nodes.size(), TensorD());
    for (int n = 0; n < (int)tree.nodes.size(); ++n) {
        const auto& nd = tree.nodes[n];
        TensorD& T = nodes[n];
        T.legs[0] = legs[nd.l];
        T.legs[1] = legs[nd.r];
        T.legs[2] = legs[nd.p];
        T.tab = make_table(T.legs[0], T.legs[1], T.legs[2], 0);
        const int64_t sz = T.tab.size();
        std::vector<double> h(sz);
        const uint64_t key = mix64(seed ^ mix64((uint64_t)n + 0x632BE59BD9B4E019ULL));
        for (int64_t i = 0; i < sz; ++i) h[i] = sym_uniform(key, (uint64_t)i);
        T.d = std::make_shared<DBuf>(dev, sz * sizeof(double));
        dev->upload(T.d->p, h.data(), sz * sizeof(double));
    }
    sweep_energies.assign(sweeps_done, NAN);
    invalidate();
}

// Driven penalty (Methods, "Numerical Convergence"): linear growth from
// nu_max/20 to nu_max/4 over n_lin sweeps, quadratic growth to nu_max over
// n_quad sweeps, then constant.  With the adaptive switch the linear phase
// ends early, after the first linear sweep t >= 1 whose energy rose above
// that of sweep t - 1 (by more than 1e-10 |E_t|), and the quadratic phase
// starts from the nu of that sweep.
double Engine::nu_for(int s) const {
    const Params& P = ctx->prm;
    const double numax = P.nu_max, lo = numax / 20.0, mid = numax / 4.0;
    auto linear = [&](int t) {
        if (P.n_lin == 1) return mid;
        return lo + (mid - lo) * t / (P.n_lin - 1);
    };
    int sw = P.n_lin;
    if (P.pen_adaptive) {
        const int nh = std::min<int>({P.n_lin, (int)sweep_energies.size(), s});
        for (int t = 1; t < nh; ++t)
            if (sweep_energies[t] > sweep_energies[t - 1] + 1e-10 * std::fabs(sweep_energies[t])) {
                sw = t + 1;
                break;
            }
    }
    if (s < sw) return linear(s);
    const double start = sw > 0 ? linear(sw - 1) : mid;
    const int k = s - sw;
    if (k < P.n_quad) {
        const double u = (double)(k + 1) / P.n_quad;
        return start + (numax - start) * u * u;
    }
    return numax;
}

// ---------------------------------------------------------------------
// QR of node n toward leg `which`; returns R (sector-preserving op)
// ---------------------------------------------------------------------
// QEDTTN_QR=cholesky takes the shifted CholeskyQR3 route for the centre
// moves, where it applies; by default every move takes the Householder
// route.  On the 2x2x2 free-flux lattice at chi = 64 the sector matrices
// of the bottom nodes toward their parent become numerically rank
// deficient as the state converges (Schmidt weights far below 1e-8), where
// the Cholesky route has to hand over to Householder after its passes:
// measured 103 against 99 ms per FP32 sweep, so it is not the default.
static bool use_cholqr() {
    const char* v = std::getenv("QEDTTN_QR");
    return v && !std::strcmp(v, "cholesky");
}

OpP Engine::qr_toward(int n, int which) {
    Dev* dev = &ctx->dev;
    TensorD& T = nodes[n];
    const Leg& L = T.legs[which];
    const int ns = L.nsec();
    std::vector<int64_t> rows(ns, 0);
    for (int b = 0; b < T.tab.nblk(); ++b) {
        const int s = T.tab.s[which][b];
        int64_t sz = T.tab.off[b + 1] - T.tab.off[b];
        rows[s] += sz / L.n[s];
    }
    std::vector<int64_t> mat(ns, 0);
    int64_t tot = 0;
    for (int s = 0; s < ns; ++s) {
        if (rows[s] < L.n[s]) fail(QED_ERR_BAD_STATE, "a sector is wider than its rows (QR)");
        mat[s] = tot;
        tot += rows[s] * L.n[s];
    }
    OpP R = make_op(dev, L, 0, false);
    std::vector<PackBlk> pb;
    std::vector<int64_t> row0(ns, 0);
    int64_t maxsize = 0;
    for (int b = 0; b < T.tab.nblk(); ++b) {
        PackBlk B{};
        B.off = T.tab.off[b];
        for (int e = 0; e < 3; ++e) B.n[e] = T.legs[e].n[T.tab.s[e][b]];
        const int s = T.tab.s[which][b];
        B.leg = which;
        B.mat = mat[s];
        B.rows = (int)rows[s];
        B.row0 = (int)row0[s];
        const int64_t sz = (int64_t)B.n[0] * B.n[1] * B.n[2];
        row0[s] += sz / L.n[s];
        maxsize = std::max(maxsize, sz);
        pb.push_back(B);
    }
    DBuf dpb(dev, pb.size() * sizeof(PackBlk));
    dev->upload(dpb.p, pb.data(), pb.size() * sizeof(PackBlk));
    DBuf packed(dev, tot * sizeof(double));
    launch_pack(dpb.as<PackBlk>(), (int)pb.size(), maxsize, T.ptr(), packed.as<double>(), 0, dev->stream);
    // every sector of the leg at once: CholeskyQR2 on the block GEMM, or,
    // for sectors it cannot take (too wide, rank deficient), the batched
    // level-synchronous Householder QR
    std::vector<QRTask> tasks;
    for (int s = 0; s < ns; ++s)
        tasks.push_back(QRTask{packed.as<double>() + mat[s], rows[s], L.n[s],
                               (double*)R->d64->p + R->lay.off[s], L.n[s], 1});
    if (!use_cholqr() || !cholqr_multi(dev, tasks)) {
        if (use_cholqr() && std::getenv("QEDTTN_TRACE"))
            std::fprintf(stderr, "[qedttn] QR of node %d toward leg %d: Householder route\n", n, which);
        tsqr_multi(dev, tasks);
    }
    launch_pack(dpb.as<PackBlk>(), (int)pb.size(), maxsize, T.ptr(), packed.as<double>(), 1, dev->stream);
    dev->check(hipGetLastError(), "qr launch");
    return R;
}

void Engine::absorb(int m, int e, const OpP& R) {
    Dev* dev = &ctx->dev;
    TensorD& T = nodes[m];
    auto out = std::make_shared<DBuf>(dev, T.tab.size() * sizeof(double));
    Plan P = plan_mode(T, e, R, out->as<double>());
    P.upload(dev);
    P.run(dev, nullptr, nullptr, nullptr);
    T.d = out;
}

EnvD& Engine::env_for(int n, int which) {
    const auto& nd = tree.nodes[n];
    EnvD& e = which == 0 ? up[nd.l] : which == 1 ? up[nd.r] : dn[nd.p];
    if (!e.valid) fail(QED_ERR_BAD_STATE, "environment used before it was rebuilt");
    return e;
}

// side membership: 0 = subtree of l, 1 = subtree of r, 2 = outside node n
static inline bool in_side(const Engine& E, int n, int side, int site) {
    const auto& nd = E.tree.nodes[n];
    if (side == 0) return E.inside[nd.l][site];
    if (side == 1) return E.inside[nd.r][site];
    return !E.inside[nd.p][site];
}

void Engine::build_env(int n, int which, EnvD& out) {
    Dev* dev = &ctx->dev;
    const TensorD& T = nodes[n];
    const int f1 = which == 0 ? 1 : 0;
    const int f2 = which == 2 ? 1 : 2;
    EnvD& e1 = env_for(n, f1);
    EnvD& e2 = env_for(n, f2);
    const Leg& leg = T.legs[which];
    std::vector<OpP> outs;
    std::vector<RTerm> rt;
    EnvD res;
    for (int cls = 0; cls < 2; ++cls) {
        res.H[cls] = make_op(dev, leg, 0, false);
        outs.push_back(res.H[cls]);
        rt.push_back(RTerm{1.0, e1.H[cls], nullptr, cls});
        rt.push_back(RTerm{1.0, nullptr, e2.H[cls], cls});
    }
    for (int i = 0; i < (int)model.terms.size(); ++i) {
        const Term& t = model.terms[i];
        if (t.coef == 0.0) continue;
        int c1 = 0, c2 = 0;
        const int tot = (int)tsites[i].size();
        for (int s : tsites[i]) {
            c1 += in_side(*this, n, f1, s);
            c2 += in_side(*this, n, f2, s);
        }
        if (c1 + c2 == 0) continue;
        if (c1 == tot || c2 == tot) continue;   // inside one side: in its H
        OpP a = c1 ? e1.open.at(i) : nullptr;
        OpP b = c2 ? e2.open.at(i) : nullptr;
        if (c1 + c2 == tot) {
            rt.push_back(RTerm{t.coef, a, b, t.cls});
            continue;
        }
        const int da = a ? a->lay.delta : 0, db = b ? b->lay.delta : 0;
        const int delta = which == 2 ? da + db : db - da;
        OpP o = make_op(dev, leg, delta, false);
        res.open[i] = o;
        rt.push_back(RTerm{1.0, a, b, (int)outs.size()});
        outs.push_back(o);
    }
    // terms whose factor is known to be zero are dropped
    std::vector<RTerm> keep;
    for (auto& r : rt) {
        if (r.a && !r.a->lay.size) continue;
        if (r.b && !r.b->lay.size) continue;
        keep.push_back(r);
    }
    Plan P = plan_renorm(T, which, keep, outs);
    P.upload(dev);
    void* w = ws.get(dev, std::max<int64_t>(1, P.ws_elems) * sizeof(double));
    P.run(dev, w, nullptr, nullptr);
    res.valid = true;
    out = res;
}

void Engine::move(int a, int b) {
    const auto& ta = tree.nodes[a];
    const auto& tb = tree.nodes[b];
    if (tb.l == ta.p || tb.r == ta.p) {
        OpP R = qr_toward(a, 2);
        absorb(b, tb.l == ta.p ? 0 : 1, R);
        build_env(a, 2, up[ta.p]);
    } else {
        const int side = ta.l == tb.p ? 0 : 1;
        OpP R = qr_toward(a, side);
        absorb(b, 2, R);
        build_env(a, side, dn[side == 0 ? ta.l : ta.r]);
    }
    centre = b;
}

void Engine::move_to(int target) {
    std::vector<int> p = tree.path(centre, target);
    for (size_t i = 0; i + 1 < p.size(); ++i) {
        if (ctx->prm.exp_on) move_svd(p[i], p[i + 1], p[i] == last_updated);
        else move(p[i], p[i + 1]);
        last_updated = -1;
    }
}

// ---------------------------------------------------------------------
// Subspace expansion (Methods: single-tensor optimisation with subspace
// expansion, bond dimensions growing and sectors adapting).  On the first
// move after node a was updated, from a to its neighbour b across link e
// (a's leg w):
//   1. e is extended: every charge Q that a's other legs can carry gets
//      min(n(Q) + delta, rows_a(Q)) columns (never fewer than n(Q)), the
//      old ones first; a is zero-padded to the extended leg;
//   2. Z = sum_k c_k (A_k (x) B_k (x) Omega_k) a+ over the terms of a's
//      H_eff that reach across e, Omega_k a random map on the extended leg
//      with the term's charge shift, nonzero from old into padded columns
//      only (counter-based SplitMix64 uniforms in [-1, 1), stream
//      65536 * (expansion count) + term index, canonical operator layout);
//   3. M = a+ + alpha (|a+| / |Z|) Z: b does not see the padded columns,
//      so the state is unchanged;
//   4. per sector, M matricised against w is factored M = U S V^T (QR, then
//      one-sided Jacobi on R^T; Jacobi on M^T directly for sectors with
//      fewer rows than columns); the largest singular values over all
//      sectors are kept, at most chi_max and none below 1e-12 of the
//      largest; a := U_keep, b := (U_keep^T M) b on the kept leg;
//   5. the environment of e from a's side is rebuilt; the one from b's side
//      is invalid until the centre crosses e back.
// Every other move in expansion mode is the same SVD move without 1-3.
// ---------------------------------------------------------------------
namespace {

// rows per charge of a node matricised against leg `which`, over all
// sector pairs of its other two legs
std::map<int, int64_t> rows_by_charge(const Leg L[3], int which) {
    std::map<int, int64_t> r;
    const int o1 = which == 0 ? 1 : 0, o2 = which == 2 ? 1 : 2;
    for (int a = 0; a < L[o1].nsec(); ++a)
        for (int b = 0; b < L[o2].nsec(); ++b) {
            const int Q = which == 2 ? L[0].q[a] + L[1].q[b] : L[2].q[b] - L[o1].q[a];
            r[Q] += (int64_t)L[o1].n[a] * L[o2].n[b];
        }
    return r;
}

int64_t get0(const std::map<int, int64_t>& m, int q) {
    auto it = m.find(q);
    return it == m.end() ? 0 : it->second;
}

// node with leg `which` replaced (table rebuilt, data uninitialised)
TensorD with_leg(Dev* dev, const TensorD& T, int which, const Leg& L) {
    TensorD R;
    for (int e = 0; e < 3; ++e) R.legs[e] = T.legs[e];
    R.legs[which] = L;
    R.tab = make_table(R.legs[0], R.legs[1], R.legs[2], 0);
    R.d = std::make_shared<DBuf>(dev, std::max<int64_t>(1, R.tab.size()) * sizeof(double));
    return R;
}

// pack descriptors of T matricised against `which`: the sector of charge q
// is a rows(q) x n(q) column-major matrix at mat(q)
struct PackList {
    std::vector<PackBlk> blks;
    int64_t maxsize = 0;
};

PackList pack_list(const TensorD& T, int which, const std::map<int, int64_t>& mat,
                   const std::map<int, int64_t>& rows) {
    PackList pl;
    std::map<int, int64_t> row0;
    const Leg& L = T.legs[which];
    for (int b = 0; b < T.tab.nblk(); ++b) {
        PackBlk B{};
        B.off = T.tab.off[b];
        for (int e = 0; e < 3; ++e) B.n[e] = T.legs[e].n[T.tab.s[e][b]];
        const int q = L.q[T.tab.s[which][b]];
        B.leg = which;
        B.mat = mat.at(q);
        B.rows = (int)rows.at(q);
        B.row0 = (int)row0[q];
        const int64_t sz = (int64_t)B.n[0] * B.n[1] * B.n[2];
        row0[q] += sz / B.n[which];
        pl.maxsize = std::max(pl.maxsize, sz);
        pl.blks.push_back(B);
    }
    return pl;
}

// host-side bounds check of a pack list against its buffers (element counts)
void check_pack(const PackList& pl, int64_t tensor_elems, int64_t packed_elems) {
    for (const PackBlk& B : pl.blks) {
        const int64_t sz = (int64_t)B.n[0] * B.n[1] * B.n[2];
        const int64_t brows = sz / B.n[B.leg];
        if (B.off < 0 || B.off + sz > tensor_elems || B.row0 < 0 || B.row0 + brows > B.rows ||
            B.mat < 0 || B.mat + (int64_t)(B.n[B.leg] - 1) * B.rows + B.rows > packed_elems)
            fail(QED_ERR_BAD_STATE, "internal: sector packing out of bounds");
    }
}

void run_pack(Dev* dev, const PackList& pl, double* tensor, double* packed, int dir) {
    if (pl.blks.empty()) return;
    DBuf d(dev, pl.blks.size() * sizeof(PackBlk));
    dev->upload(d.p, pl.blks.data(), pl.blks.size() * sizeof(PackBlk));
    launch_pack(d.as<PackBlk>(), (int)pl.blks.size(), pl.maxsize, tensor, packed, dir, dev->stream);
    dev->check(hipGetLastError(), "pack");
}

// sector-matrix offsets of a leg with the given rows per charge
std::map<int, int64_t> sector_offsets(const Leg& L, const std::map<int, int64_t>& rows, int64_t& tot) {
    std::map<int, int64_t> mat;
    tot = 0;
    for (int s = 0; s < L.nsec(); ++s) {
        mat[L.q[s]] = tot;
        tot += get0(rows, L.q[s]) * L.n[s];
    }
    return mat;
}

// C (col-major rows x k, ld rows) = A (col-major rows x kin, ld rows) *
// Bm (col-major kin x k, ld kin), as the row-major product C^T = Bm^T A^T
void push_colmajor_gemm(Plan& pl, double* C, const double* A, const double* Bm, int64_t rows, int kin,
                        int k) {
    if (rows <= 0 || kin <= 0 || k <= 0 || rows > INT32_MAX)
        fail(QED_ERR_BAD_STATE, "internal: empty or oversized sector product");
    GProd pr{};
    pr.A = GRef{Bm, 0, TAG_ABS, 0};
    pr.lda = kin;
    pr.B = GRef{A, 0, TAG_ABS, 0};
    pr.ldb = (int)rows;
    pr.K = kin;
    pr.alpha = 1.0;
    pr.nred = 1;
    GJob j{};
    j.C = GRef{C, 0, TAG_ABS, 0};
    j.M = k;
    j.N = (int)rows;
    j.ldc = (int)rows;
    j.batch = 1;
    j.p0 = (int)pl.prods[0].size();
    pl.prods[0].push_back(pr);
    j.p1 = j.p0 + 1;
    pl.jobs[0].push_back(j);
    pl.stage_flops[0] += 2.0 * rows * kin * k;
    pl.flops += 2.0 * rows * kin * k;
}

}  // namespace

void Engine::move_svd(int a, int b, bool grow) {
    Dev* dev = &ctx->dev;
    const Params& P = ctx->prm;
    hipStream_t st = dev->stream;
    const auto& ta = tree.nodes[a];
    const auto& tb = tree.nodes[b];
    int w, wb, link;
    if (tb.l == ta.p || tb.r == ta.p) {
        w = 2;
        wb = tb.l == ta.p ? 0 : 1;
        link = ta.p;
    } else {
        w = ta.l == tb.p ? 0 : 1;
        wb = 2;
        link = w == 0 ? ta.l : ta.r;
    }
    const Leg old = legs[link];
    std::map<int, int> oldn;
    for (int s = 0; s < old.nsec(); ++s) oldn[old.q[s]] = old.n[s];
    auto nold = [&](int q) { auto it = oldn.find(q); return it == oldn.end() ? 0 : it->second; };
    // 1. extended leg and the padded node
    const std::map<int, int64_t> rows = rows_by_charge(nodes[a].legs, w);
    std::map<int, int> sz = oldn;
    if (grow)
        for (const auto& kv : rows) {
            const int n0 = nold(kv.first);
            const int64_t n = std::max<int64_t>(n0, std::min<int64_t>((int64_t)n0 + P.exp_delta, kv.second));
            if (n > 0) sz[kv.first] = (int)n;
        }
    Leg plus;
    for (const auto& kv : sz) {
        plus.q.push_back(kv.first);
        plus.n.push_back(kv.second);
    }
    TensorD M = with_leg(dev, nodes[a], w, plus);
    int64_t tot = 0;
    const std::map<int, int64_t> mat = sector_offsets(plus, rows, tot);
    DBuf packed(dev, std::max<int64_t>(1, tot) * sizeof(double));
    launch_fill(packed.as<double>(), tot, 0.0, st);
    const PackList pl_old = pack_list(nodes[a], w, mat, rows);
    const PackList pl_m = pack_list(M, w, mat, rows);
    check_pack(pl_old, nodes[a].tab.size(), tot);
    check_pack(pl_m, M.tab.size(), tot);
    run_pack(dev, pl_old, nodes[a].ptr(), packed.as<double>(), 0);
    run_pack(dev, pl_m, M.ptr(), packed.as<double>(), 1);
    const int64_t nm = M.tab.size();
    // 2-3. expansion term
    if (grow && P.exp_alpha > 0.0 && nm > 0) {
        std::vector<HTerm> zt;
        EnvD* E[3] = {&env_for(a, 0), &env_for(a, 1), &env_for(a, 2)};
        for (int i = 0; i < (int)model.terms.size(); ++i) {
            const Term& t = model.terms[i];
            if (t.coef == 0.0) continue;
            bool touch[3] = {false, false, false};
            for (int s : tsites[i])
                for (int side = 0; side < 3; ++side)
                    if (in_side(*this, a, side, s)) touch[side] = true;
            if (!touch[w] || touch[0] + touch[1] + touch[2] < 2) continue;
            OpP om = make_op(dev, plus, E[w]->open.at(i)->lay.delta, false);
            if (!om->lay.size) continue;
            std::vector<double> h(om->lay.size, 0.0);
            const uint64_t stream = (uint64_t)n_expand * 65536ULL + (uint64_t)i;
            const uint64_t key = mix64(P.exp_seed ^ mix64(stream + 0x632BE59BD9B4E019ULL));
            bool any = false;
            for (int s = 0; s < plus.nsec(); ++s) {
                const int o = om->lay.out_of_in[s];
                if (o < 0) continue;
                const int ni = plus.n[s], no = plus.n[o];
                for (int r = nold(plus.q[o]); r < no; ++r)
                    for (int c = 0; c < nold(plus.q[s]); ++c) {
                        const int64_t idx = om->lay.off[s] + (int64_t)r * ni + c;
                        h[idx] = sym_uniform(key, (uint64_t)idx);
                        any = true;
                    }
            }
            if (!any) continue;
            dev->upload(om->d64->p, h.data(), h.size() * sizeof(double));
            HTerm ht{t.coef * (t.cls == CLS_PEN ? cur_nu : 1.0), {nullptr, nullptr, nullptr}};
            for (int k = 0; k < 3; ++k)
                if (k != w && touch[k]) ht.op[k] = E[k]->open.at(i);
            ht.op[w] = om;
            zt.push_back(ht);
        }
        if (!zt.empty()) {
            Plan pz = plan_matvec(M.legs, M.tab, zt, QED_FP64);
            pz.upload(dev);
            DBuf z(dev, nm * sizeof(double));
            void* wsp = ws.get(dev, std::max<int64_t>(1, pz.ws_elems) * sizeof(double));
            pz.run(dev, wsp, M.ptr(), z.p);
            DBuf part(dev, 512 * sizeof(double)), nr(dev, 2 * sizeof(double));
            launch_dots(M.ptr(), nm, 1, M.ptr(), nm, part.as<double>(), nr.as<double>(), 1, nullptr, 0, st);
            launch_dots(z.as<double>(), nm, 1, z.as<double>(), nm, part.as<double>(), nr.as<double>() + 1, 1,
                        nullptr, 0, st);
            double h2[2];
            dev->download(h2, nr.p, sizeof(h2));
            if (h2[1] > 0.0 && std::isfinite(h2[1])) {
                launch_axpy(M.ptr(), z.as<double>(), P.exp_alpha * h2[0] / h2[1], nm, st);
                // the padded columns now carry the expansion: repack M
                run_pack(dev, pl_m, M.ptr(), packed.as<double>(), 0);
            }
        }
    }
    // 4. per-sector SVD
    struct Sec {
        int q, r, c, m;        // charge, rows, columns, Jacobi columns
        bool qr;
        int64_t x, v, s;       // offsets of X (c x m), V (m x m), sigma (m)
    };
    std::vector<Sec> secs;
    int64_t xs = 0, vs = 0, ss = 0;
    for (int s = 0; s < plus.nsec(); ++s) {
        Sec S{};
        S.q = plus.q[s];
        S.r = (int)get0(rows, S.q);
        S.c = plus.n[s];
        if (S.r == 0) continue;
        S.qr = S.r >= S.c;
        S.m = S.qr ? S.c : S.r;
        S.x = xs;
        S.v = vs;
        S.s = ss;
        xs += (int64_t)S.c * S.m;
        vs += (int64_t)S.m * S.m;
        ss += S.m;
        secs.push_back(S);
    }
    DBuf X(dev, std::max<int64_t>(1, xs) * sizeof(double));
    DBuf V(dev, std::max<int64_t>(1, vs) * sizeof(double));
    DBuf SG(dev, std::max<int64_t>(1, ss) * sizeof(double));
    std::vector<QRTask> tasks;
    std::vector<int64_t> tblk;
    for (const Sec& S : secs) {
        if (mat.at(S.q) + (int64_t)S.r * S.c > tot || S.x + (int64_t)S.c * S.m > xs ||
            S.v + (int64_t)S.m * S.m > vs || S.s + S.m > ss)
            fail(QED_ERR_BAD_STATE, "internal: sector decomposition out of bounds");
        double* Mq = packed.as<double>() + mat.at(S.q);
        if (S.qr) {
            // R row-major (rrs = c, rcs = 1) is R^T column-major: X directly
            tasks.push_back(QRTask{Mq, S.r, S.c, X.as<double>() + S.x, S.c, 1});
        } else {
            // M_q (column-major r x c) is row-major c x r; its transpose is
            // X = M_q^T column-major (c x r)
            tblk.insert(tblk.end(), {mat.at(S.q), S.x, (int64_t)S.c, (int64_t)S.r});
        }
    }
    if (!tasks.empty()) tsqr_multi(dev, tasks);
    if (!tblk.empty()) {
        DBuf d(dev, tblk.size() * sizeof(int64_t));
        dev->upload(d.p, tblk.data(), tblk.size() * sizeof(int64_t));
        launch_transpose_blocks(packed.as<double>(), X.as<double>(), d.as<int64_t>(), (int)tblk.size() / 4, st);
    }
    std::vector<SvdMat> sm;
    for (const Sec& S : secs)
        sm.push_back(SvdMat{X.as<double>() + S.x, V.as<double>() + S.v, SG.as<double>() + S.s, S.c, S.m});
    if (!sm.empty()) {
        DBuf d(dev, sm.size() * sizeof(SvdMat));
        dev->upload(d.p, sm.data(), sm.size() * sizeof(SvdMat));
        launch_jacobi_svd(d.as<SvdMat>(), (int)sm.size(), st);
        dev->check(hipGetLastError(), "jacobi svd");
    }
    std::vector<double> hX(xs), hV(vs), hS(ss);
    if (xs) dev->download(hX.data(), X.p, xs * sizeof(double));
    if (vs) dev->download(hV.data(), V.p, vs * sizeof(double));
    if (ss) dev->download(hS.data(), SG.p, ss * sizeof(double));
    // kept singular values: the largest over all sectors, at most chi_max,
    // none below 1e-12 of the largest (ties: charge, then position)
    struct Cand {
        double s;
        int sec, j;
    };
    double smax = 0.0;
    for (double v : hS) smax = std::max(smax, v);
    std::vector<Cand> cand;
    for (int k = 0; k < (int)secs.size(); ++k) {
        std::vector<int> js(secs[k].m);
        for (int j = 0; j < secs[k].m; ++j) js[j] = j;
        std::stable_sort(js.begin(), js.end(),
                         [&](int x, int y) { return hS[secs[k].s + x] > hS[secs[k].s + y]; });
        for (int j : js)
            if (hS[secs[k].s + j] > 1e-12 * smax) cand.push_back(Cand{hS[secs[k].s + j], k, j});
    }
    std::stable_sort(cand.begin(), cand.end(), [](const Cand& x, const Cand& y) { return x.s > y.s; });
    const int chimax = P.exp_chimax > 0 ? P.exp_chimax : P.chi;
    if ((int)cand.size() > chimax) cand.resize(chimax);
    if (cand.empty()) fail(QED_ERR_NONFINITE, "subspace expansion: the node has no nonzero singular value");
    std::map<int, std::vector<int>> keep;   // per section index: kept Jacobi columns, descending sigma
    for (const Cand& c : cand) keep[c.sec].push_back(c.j);
    Leg enew;
    for (int k = 0; k < (int)secs.size(); ++k)
        if (keep.count(k)) {
            enew.q.push_back(secs[k].q);
            enew.n.push_back((int)keep[k].size());
        }
    // a := U_keep; b := (U_keep^T M) b on the kept leg
    TensorD An = with_leg(dev, nodes[a], w, enew);
    TensorD Bn = with_leg(dev, nodes[b], wb, enew);
    int64_t tota = 0, totb_old = 0, totb = 0;
    const std::map<int, int64_t> mata = sector_offsets(enew, rows, tota);
    const std::map<int, int64_t> rowsb = rows_by_charge(nodes[b].legs, wb);
    const std::map<int, int64_t> matb_old = sector_offsets(old, rowsb, totb_old);
    const std::map<int, int64_t> matb = sector_offsets(enew, rowsb, totb);
    DBuf pa(dev, std::max<int64_t>(1, tota) * sizeof(double));
    DBuf pbo(dev, std::max<int64_t>(1, totb_old) * sizeof(double));
    DBuf pb(dev, std::max<int64_t>(1, totb) * sizeof(double));
    launch_fill(pb.as<double>(), totb, 0.0, st);
    const PackList pl_bo = pack_list(nodes[b], wb, matb_old, rowsb);
    check_pack(pl_bo, nodes[b].tab.size(), totb_old);
    run_pack(dev, pl_bo, nodes[b].ptr(), pbo.as<double>(), 0);
    std::vector<double> hU, hT;          // host copies of U_keep / T blocks
    std::vector<int64_t> uo, to;
    for (const auto& kv : keep) {
        const Sec& S = secs[kv.first];
        const std::vector<int>& js = kv.second;
        const int k = (int)js.size();
        uo.push_back((int64_t)hU.size());
        for (int j : js)
            for (int i = 0; i < S.m; ++i) hU.push_back(hV[S.v + (int64_t)j * S.m + i]);
        const int n0 = nold(S.q);
        to.push_back((int64_t)hT.size());
        for (int j : js)
            for (int i = 0; i < n0; ++i) hT.push_back(hX[S.x + (int64_t)j * S.c + i]);
        (void)k;
    }
    DBuf dU(dev, std::max<size_t>(1, hU.size()) * sizeof(double));
    DBuf dT(dev, std::max<size_t>(1, hT.size()) * sizeof(double));
    if (!hU.empty()) dev->upload(dU.p, hU.data(), hU.size() * sizeof(double));
    if (!hT.empty()) dev->upload(dT.p, hT.data(), hT.size() * sizeof(double));
    Plan pl;
    pl.dtype = QED_FP64;
    pl.jobs.emplace_back();
    pl.prods.emplace_back();
    pl.stage_flops.push_back(0.0);
    size_t idx = 0;
    for (const auto& kv : keep) {
        const Sec& S = secs[kv.first];
        const int k = (int)kv.second.size();
        double* Ca = pa.as<double>() + mata.at(S.q);
        const double* Uk = dU.as<double>() + uo[idx];
        if (mata.at(S.q) + (int64_t)S.r * k > tota || uo[idx] + (int64_t)S.m * k > (int64_t)hU.size())
            fail(QED_ERR_BAD_STATE, "internal: expansion output out of bounds");
        if (S.qr) {
            // a block = Q (r x c) U_keep (c x k)
            push_colmajor_gemm(pl, Ca, packed.as<double>() + mat.at(S.q), Uk, S.r, S.c, k);
        } else {
            // Q is the identity: a block = U_keep (r x k)
            dev->check(hipMemcpyAsync(Ca, Uk, (size_t)S.r * k * sizeof(double), hipMemcpyDeviceToDevice, st),
                       "expansion copy");
        }
        const int n0 = nold(S.q);
        const int64_t rb = get0(rowsb, S.q);
        if (n0 > 0 && rb > 0 &&
            (matb.at(S.q) + rb * k > totb || matb_old.at(S.q) + rb * n0 > totb_old ||
             to[idx] + (int64_t)n0 * k > (int64_t)hT.size()))
            fail(QED_ERR_BAD_STATE, "internal: expansion output out of bounds");
        if (n0 > 0 && rb > 0)
            push_colmajor_gemm(pl, pb.as<double>() + matb.at(S.q), pbo.as<double>() + matb_old.at(S.q),
                               dT.as<double>() + to[idx], rb, n0, k);
        ++idx;
    }
    if (!pl.jobs[0].empty()) {
        pl.upload(dev);
        pl.run(dev, nullptr, nullptr, nullptr);
    }
    const PackList pl_a = pack_list(An, w, mata, rows);
    const PackList pl_b = pack_list(Bn, wb, matb, rowsb);
    check_pack(pl_a, An.tab.size(), tota);
    check_pack(pl_b, Bn.tab.size(), totb);
    run_pack(dev, pl_a, An.ptr(), pa.as<double>(), 1);
    run_pack(dev, pl_b, Bn.ptr(), pb.as<double>(), 1);
    // 5. install, environments
    legs[link] = enew;
    nodes[a] = An;
    nodes[b] = Bn;
    build_env(a, w, w == 2 ? up[link] : dn[link]);
    (w == 2 ? dn[link] : up[link]) = EnvD();
    if (grow) ++n_expand;
    centre = b;
}

void Engine::adopt_legs(const std::vector<Leg>& nl) {
    Dev* dev = &ctx->dev;
    legs = nl;
    nodes.assign(tree.nodes.size(), TensorD());
    for (int n = 0; n < (int)tree.nodes.size(); ++n) {
        const auto& nd = tree.nodes[n];
        TensorD& T = nodes[n];
        T.legs[0] = legs[nd.l];
        T.legs[1] = legs[nd.r];
        T.legs[2] = legs[nd.p];
        T.tab = make_table(T.legs[0], T.legs[1], T.legs[2], 0);
        T.d = std::make_shared<DBuf>(dev, std::max<int64_t>(1, T.tab.size()) * sizeof(double));
    }
    invalidate();
}

void Engine::prepare() {
    Dev* dev = &ctx->dev;
    if (nodes.empty()) fail(QED_ERR_BAD_STATE, "no state: call qed_init_state or qed_set_node");
    // site operators on the device
    siteops.assign(tree.N, {});
    for (int s = 0; s < tree.N; ++s) {
        const Site& st = model.sites[s];
        const int d = st.d();
        for (const SiteOp& so : st.ops) {
            OpP o = make_op(dev, st.leg, so.delta, false);
            std::vector<double> h(o->lay.size, 0.0);
            int off_in = 0;
            std::vector<int> start(st.leg.nsec(), 0);
            for (int k = 1; k < st.leg.nsec(); ++k) start[k] = start[k - 1] + st.leg.n[k - 1];
            (void)off_in;
            for (int si = 0; si < st.leg.nsec(); ++si) {
                const int so_ = o->lay.out_of_in[si];
                if (so_ < 0) continue;
                const int ni = st.leg.n[si], no = st.leg.n[so_];
                for (int r = 0; r < no; ++r)
                    for (int c = 0; c < ni; ++c)
                        h[o->lay.off[si] + (int64_t)r * ni + c] =
                            so.m[(size_t)(start[so_] + r) * d + start[si] + c];
            }
            if (o->lay.size) dev->upload(o->d64->p, h.data(), h.size() * sizeof(double));
            siteops[s].push_back(o);
        }
    }
    // upward environments of the physical legs
    for (int s = 0; s < tree.N; ++s) {
        const Site& st = model.sites[s];
        EnvD e;
        std::vector<double> hsum[2];
        for (int cls = 0; cls < 2; ++cls) e.H[cls] = make_op(dev, st.leg, 0, true);
        std::vector<double> acc[2];
        for (int cls = 0; cls < 2; ++cls) acc[cls].assign(e.H[cls]->lay.size, 0.0);
        bool any[2] = {false, false};
        for (int i = 0; i < (int)model.terms.size(); ++i) {
            const Term& t = model.terms[i];
            if (t.coef == 0.0) continue;
            int fi = -1;
            for (int k = 0; k < (int)t.f.size(); ++k)
                if (t.f[k].site == s) fi = k;
            if (fi < 0) continue;
            const OpP& op = siteops[s][t.f[fi].op];
            if (t.f.size() == 1) {
                if (op->lay.delta != 0) fail(QED_ERR_BAD_STATE, "onsite term must conserve charge");
                // accumulate on the host from the dense site matrix
                const SiteOp& so = st.ops[t.f[fi].op];
                std::vector<int> start(st.leg.nsec(), 0);
                for (int k = 1; k < st.leg.nsec(); ++k) start[k] = start[k - 1] + st.leg.n[k - 1];
                for (int si = 0; si < st.leg.nsec(); ++si) {
                    const int ni = st.leg.n[si];
                    for (int r = 0; r < ni; ++r)
                        for (int c = 0; c < ni; ++c)
                            acc[t.cls][e.H[t.cls]->lay.off[si] + (int64_t)r * ni + c] +=
                                t.coef * so.m[(size_t)(start[si] + r) * st.d() + start[si] + c];
                }
                any[t.cls] = true;
            } else {
                e.open[i] = op;
            }
        }
        for (int cls = 0; cls < 2; ++cls)
            if (any[cls]) dev->upload(e.H[cls]->d64->p, acc[cls].data(), acc[cls].size() * sizeof(double));
        e.valid = true;
        up[s] = e;
    }
    // isometrise bottom-up; the centre ends at the root (a state restored
    // from a checkpoint taken with the centre at the root is isometric
    // already: only its environments are rebuilt)
    for (int n = 0; n < (int)tree.nodes.size(); ++n) {
        if (n == tree.root) continue;
        const auto& nd = tree.nodes[n];
        if (!isometric) {
            if (ctx->prm.exp_on) {
                // expansion mode: SVD moves throughout (they build the environment)
                move_svd(n, tree.parent_node[nd.p], false);
                continue;
            }
            OpP R = qr_toward(n, 2);
            absorb(tree.parent_node[nd.p], tree.parent_side[nd.p], R);
        }
        build_env(n, 2, up[nd.p]);
    }
    isometric = false;
    EnvD top;
    for (int cls = 0; cls < 2; ++cls) top.H[cls] = make_op(dev, legs[tree.top], 0, true);
    top.valid = true;
    dn[tree.top] = top;
    centre = tree.root;
}

// The FP32 path keeps its Krylov basis in FP32, the precision of its
// matvec: the matvec reads its input straight from the basis and every
// Gram-Schmidt pass reads half the bytes (dot products and updates still in
// FP64).  On the 2x2x2 free-flux lattice at chi = 64 its sweeps take 83
// against 86 ms with the FP64 basis, and its trajectory converges in 1930
// against 2171 matvecs.  QEDTTN_LZ_BASIS=fp64 selects the FP64 basis (with
// an FP32 copy of each new vector for the matvec).
static bool basis32_enabled() {
    const char* v = std::getenv("QEDTTN_LZ_BASIS");
    return !(v && !std::strcmp(v, "fp64"));
}

double Engine::update(int n, double nu, bool refine_here) {
    Dev* dev = &ctx->dev;
    const Params& P = ctx->prm;
    cur_nu = nu;
    TensorD& T = nodes[n];
    std::vector<HTerm> ht;
    EnvD* E[3] = {&env_for(n, 0), &env_for(n, 1), &env_for(n, 2)};
    for (int cls = 0; cls < 2; ++cls) {
        const double w = cls == CLS_PEN ? nu : 1.0;
        for (int e = 0; e < 3; ++e) {
            HTerm h{w, {nullptr, nullptr, nullptr}};
            h.op[e] = E[e]->H[cls];
            ht.push_back(h);
        }
    }
    for (int i = 0; i < (int)model.terms.size(); ++i) {
        const Term& t = model.terms[i];
        if (t.coef == 0.0) continue;
        bool touch[3] = {false, false, false};
        for (int s : tsites[i])
            for (int side = 0; side < 3; ++side)
                if (in_side(*this, n, side, s)) touch[side] = true;
        if (touch[0] + touch[1] + touch[2] < 2) continue;
        HTerm h{t.coef * (t.cls == CLS_PEN ? nu : 1.0), {nullptr, nullptr, nullptr}};
        for (int e = 0; e < 3; ++e)
            if (touch[e]) h.op[e] = E[e]->open.at(i);
        ht.push_back(h);
    }
    const int dtype = P.dtype;
    if (dtype == QED_FP32) {
        std::vector<LegOpD*> ops;
        for (const HTerm& h : ht)
            for (int e = 0; e < 3; ++e)
                if (h.op[e]) ops.push_back(h.op[e].get());
        prepare_f32_copies(dev, ops);
    }
    Plan plan = plan_matvec(T.legs, T.tab, ht, dtype);
    plan.upload(dev);
    plan.prof = &ctx->prof;
    const int64_t n_el = T.tab.size();
    BufP xc, yc;
    if (dtype != QED_FP64) {
        xc = std::make_shared<DBuf>(dev, n_el * dtype_size(dtype));
        yc = std::make_shared<DBuf>(dev, n_el * dtype_size(dtype));
    }
    void* w = ws.get(dev, std::max<int64_t>(1, plan.ws_elems) * dtype_size(dtype));
    // reduced precision with the FP64 residual correction: the FP64 plan
    // applies the first vector of every Lanczos cycle, so the exact residual
    // of the current vector enters the Krylov space and ends the run once it
    // is small enough; the other steps use the reduced-precision plan
    const bool fix = dtype != QED_FP64 && P.refine >= 2;
    Plan p64;
    void* w64 = nullptr;
    if (fix) {
        p64 = plan_matvec(T.legs, T.tab, ht, QED_FP64);
        p64.upload(dev);
        w64 = ws64.get(dev, std::max<int64_t>(1, p64.ws_elems) * 8);
    }
    long long exact_mv = 0;
    auto apply = [&](const double* v, const float* v32, double* y, double* part) {
        if (dtype == QED_FP64) {
            plan.run(dev, w, (void*)v, (void*)y);
            return false;
        }
        if (fix && v && v == lws.V->as<double>()) {
            p64.run(dev, w64, (void*)v, (void*)y);
            ++exact_mv;
            return false;
        }
        // the FP32 input: the FP32 basis vector itself, the FP32 copy the
        // previous step wrote, or a conversion of the FP64 vector
        const bool have32 = v32 && dtype == QED_FP32;
        if (!have32) to_compute(dtype, v, xc->p, n_el, dev->stream);
        plan.run(dev, w, have32 ? (void*)v32 : xc->p, yc->p);
        if (dtype == QED_FP32) {   // conversion back fused with the alpha dot
            if (v)
                launch_f32_to_f64_dot<double>((const float*)yc->p, y, v, n_el, part, lws.st->as<LState>(),
                                              dev->stream);
            else
                launch_f32_to_f64_dot<float>((const float*)yc->p, y, v32, n_el, part, lws.st->as<LState>(),
                                             dev->stream);
            return true;
        }
        from_compute(dtype, yc->p, y, n_el, dev->stream);
        return false;
    };
    // an FP32 Krylov recurrence cannot resolve residuals below ~eps32 |H|:
    // restarts past that point only repeat work (the FP64 Rayleigh quotient
    // below fixes the energy)
    // the precision schedule of the sweeps (raised sweep by sweep)
    double tol_s = P.lz_tol;
    if (P.lz_tol0 > 0.0) tol_s = std::max(tol_s, P.lz_tol0 * std::pow(P.lz_factor, (double)sweeps_done));
    double tol = tol_s;
    if (dtype != QED_FP64)
        tol = std::max(tol_s, fix ? (dtype == QED_BF16 ? LZ_TOL_FLOOR_FIX_BF16 : LZ_TOL_FLOOR_FIX_FP32)
                                  : (dtype == QED_BF16 ? LZ_TOL_FLOOR_BF16 : LZ_TOL_FLOOR_FP32));
    // the FP32 path takes each new basis vector's FP32 copy from the
    // Lanczos step that writes it
    LanczosResult R = lanczos(dev, lws, apply, T.ptr(), n_el, P.lz_steps, P.lz_cycles, tol,
                              dtype == QED_FP32 ? (float*)xc->p : nullptr, fix ? tol : 0.0,
                              dtype == QED_FP32 && !fix && basis32_enabled());
    // the Lanczos run ended in a synchronising download: every GEMM event
    // recorded so far has completed, and its pair can be reused
    if (ctx->prof.on) ctx->prof.harvest();
    matvecs += R.matvecs;
    flops += R.matvecs * plan.flops;
    ctx->mv_count += R.matvecs;
    ctx->mv_flops += R.matvecs * plan.flops;
    double theta = R.theta;
    if (dtype != QED_FP64 && P.refine && refine_here && !R.exact) {
        // FP64 Rayleigh quotient of the (normalised) Ritz vector
        if (!fix) {
            p64 = plan_matvec(T.legs, T.tab, ht, QED_FP64);
            p64.upload(dev);
            w64 = ws64.get(dev, std::max<int64_t>(1, p64.ws_elems) * 8);
        }
        DBuf y(dev, n_el * sizeof(double));
        p64.run(dev, w64, T.ptr(), y.p);
        DBuf part(dev, 512 * sizeof(double)), out(dev, sizeof(double));
        launch_dots(T.ptr(), n_el, 1, y.as<double>(), n_el, part.as<double>(), out.as<double>(), 0,
                    nullptr, 0, dev->stream);
        dev->download(&theta, out.p, sizeof(double));
        matvecs += 1;
        flops += p64.flops;
        ctx->mv_count += 1;
        ctx->mv_flops += p64.flops;
    }
    energy = theta + model.offset[CLS_PHYS] + nu * model.offset[CLS_PEN];
    have_energy = true;
    last_updated = n;
    if (std::getenv("QEDTTN_TRACE"))
        std::fprintf(stderr, "[qedttn] update node %d size %lld terms %zu theta %.15g resid %.3g%s E %.15g "
                     "(%lld matvecs, %lld FP64)\n", n, (long long)n_el, ht.size(), theta, R.resid,
                     R.exact ? " (exact)" : "", energy, R.matvecs, exact_mv);
    return energy;
}

void Engine::sweep(int s_index, qed_sweep_report* rep) {
    Dev* dev = &ctx->dev;
    const double nu = nu_for(sweeps_done);
    if (centre < 0) prepare();
    const double e_prev = have_energy ? energy : NAN;
    const long long mv0 = matvecs;
    const double fl0 = flops;
    dev->sync();
    auto t0 = std::chrono::steady_clock::now();
    const bool trace = std::getenv("QEDTTN_TRACE") != nullptr;
    for (int n = 0; n < (int)tree.nodes.size(); ++n) {
        auto a = std::chrono::steady_clock::now();
        move_to(n);
        if (trace) {
            dev->sync();
            auto b = std::chrono::steady_clock::now();
            std::fprintf(stderr, "[qedttn] move to node %d: %.3f s\n", n,
                         std::chrono::duration<double>(b - a).count());
            a = b;
        }
        // the energy of the sweep is that of its last update: only there
        // does the reduced-precision path add the FP64 Rayleigh quotient
        update(n, nu, n + 1 == (int)tree.nodes.size());
        if (trace) {
            dev->sync();
            std::fprintf(stderr, "[qedttn] update node %d: %.3f s\n", n,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count());
        }
    }
    dev->sync();
    auto t1 = std::chrono::steady_clock::now();
    ++sweeps_done;
    // energy history by sweep index (entries of sweeps run before a state
    // was set are NaN: they never count as a rise)
    if ((int)sweep_energies.size() < sweeps_done) sweep_energies.resize(sweeps_done, NAN);
    sweep_energies[sweeps_done - 1] = energy;
    if (rep) {
        std::vector<double> e7;
        observables(e7);
        double dL = 0.0, Q = 0.0;
        const Lattice& L = model.lat;
        for (int x = 0; x < L.N; ++x) {
            Q += e7[x * 7] - L.parity(x);
            for (int mu = 0; mu < 3; ++mu) {
                int y = L.neighbour(x, 3 + mu);
                if (y < 0) continue;
                dL += std::fabs(e7[x * 7 + 1 + 3 + mu] + e7[y * 7 + 1 + mu] - 2.0);
            }
        }
        rep->energy = energy;
        rep->dE = energy - e_prev;
        rep->nu = nu;
        rep->deltaL = dL;
        rep->Q = Q;
        rep->seconds = std::chrono::duration<double>(t1 - t0).count();
        rep->flops = flops - fl0;
        rep->matvecs = matvecs - mv0;
    }
    (void)s_index;
}

void Engine::observables(std::vector<double>& site7) {
    Dev* dev = &ctx->dev;
    if (centre < 0) prepare();
    move_to(tree.root);
    const int nl = tree.nlinks();
    std::vector<OpP> rho(nl);
    // top: 1 / |root|^2
    {
        TensorD& R = nodes[tree.root];
        DBuf part(dev, 512 * sizeof(double)), out(dev, sizeof(double));
        launch_dots(R.ptr(), R.tab.size(), 1, R.ptr(), R.tab.size(), part.as<double>(),
                    out.as<double>(), 0, nullptr, 0, dev->stream);
        double nrm2 = 0.0;
        dev->download(&nrm2, out.p, sizeof(double));
        OpP t = make_op(dev, legs[tree.top], 0, false);
        double v = 1.0 / nrm2;
        dev->upload(t->d64->p, &v, sizeof(double));
        rho[tree.top] = t;
    }
    for (int n = (int)tree.nodes.size() - 1; n >= 0; --n) {
        const auto& nd = tree.nodes[n];
        for (int side = 0; side < 2; ++side) {
            const int link = side == 0 ? nd.l : nd.r;
            OpP o = make_op(dev, legs[link], 0, false);
            std::vector<RTerm> rt = {RTerm{1.0, nullptr, rho[nd.p], 0}};
            Plan P = plan_renorm(nodes[n], side, rt, {o});
            P.upload(dev);
            void* w = ws.get(dev, std::max<int64_t>(1, P.ws_elems) * sizeof(double));
            P.run(dev, w, nullptr, nullptr);
            rho[link] = o;
        }
    }
    site7.assign((size_t)tree.N * 7, 0.0);
    DBuf out(dev, 7 * sizeof(double));
    for (int s = 0; s < tree.N; ++s) {
        const Site& st = model.sites[s];
        const OpP& r = rho[s];
        std::vector<int64_t> pos;
        std::vector<signed char> rows;
        for (int si = 0; si < st.leg.nsec(); ++si) {
            const int ni = st.leg.n[si];
            for (int i = 0; i < ni; ++i) pos.push_back(r->lay.off[si] + (int64_t)i * ni + i);
        }
        for (auto& row : st.rows)
            for (int c = 0; c < 7; ++c) rows.push_back(row[c]);
        DBuf dpos(dev, pos.size() * sizeof(int64_t)), drows(dev, rows.size());
        dev->upload(dpos.p, pos.data(), pos.size() * sizeof(int64_t));
        dev->upload(drows.p, rows.data(), rows.size());
        launch_site_expect(r->f64(), dpos.as<int64_t>(), drows.as<signed char>(), st.d(),
                           out.as<double>(), dev->stream);
        dev->download(&site7[(size_t)s * 7], out.p, 7 * sizeof(double));
    }
}

}  // namespace qed
