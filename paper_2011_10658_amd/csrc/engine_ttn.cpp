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

#include "engine.h"

namespace qed {

constexpr double LZ_TOL_FLOOR_FP32 = 2e-6;
// BF16 operands carry 8 significant bits (unit roundoff u = 2^-9): a
// matvec is accurate to a few u relative, and Krylov residuals stall near
// that level; the floor is 2u
constexpr double LZ_TOL_FLOOR_BF16 = 3.9e-3;

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
    have_energy = false;
}

void Engine::init_nodes(uint64_t seed) {
    Dev* dev = &ctx->dev;
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
    invalidate();
}

double Engine::nu_for(int s) const {
    const Params& P = ctx->prm;
    const double numax = P.nu_max, lo = numax / 20.0, mid = numax / 4.0;
    if (s < P.n_lin) {
        if (P.n_lin == 1) return mid;
        return lo + (mid - lo) * s / (P.n_lin - 1);
    }
    if (s < P.n_lin + P.n_quad) {
        double u = (double)(s - P.n_lin + 1) / P.n_quad;
        return mid + (numax - mid) * u * u;
    }
    return numax;
}

// ---------------------------------------------------------------------
// QR of node n toward leg `which`; returns R (sector-preserving op)
// ---------------------------------------------------------------------
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
    // every sector of the leg in one batched (level-synchronous) QR
    std::vector<QRTask> tasks;
    for (int s = 0; s < ns; ++s)
        tasks.push_back(QRTask{packed.as<double>() + mat[s], rows[s], L.n[s],
                               (double*)R->d64->p + R->lay.off[s], L.n[s], 1});
    tsqr_multi(dev, tasks);
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
    if (which == 0) return up[nd.l];
    if (which == 1) return up[nd.r];
    return dn[nd.p];
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
    for (size_t i = 0; i + 1 < p.size(); ++i) move(p[i], p[i + 1]);
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

double Engine::update(int n, double nu) {
    Dev* dev = &ctx->dev;
    const Params& P = ctx->prm;
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
    auto apply = [&](const double* v, double* y) {
        if (dtype == QED_FP64) {
            plan.run(dev, w, (void*)v, (void*)y);
        } else {
            to_compute(dtype, v, xc->p, n_el, dev->stream);
            plan.run(dev, w, xc->p, yc->p);
            from_compute(dtype, yc->p, y, n_el, dev->stream);
        }
    };
    // an FP32 Krylov recurrence cannot resolve residuals below ~eps32 |H|:
    // restarts past that point only repeat work (the FP64 Rayleigh quotient
    // below fixes the energy)
    // the precision schedule of the sweeps (raised sweep by sweep)
    double tol_s = P.lz_tol;
    if (P.lz_tol0 > 0.0) tol_s = std::max(tol_s, P.lz_tol0 * std::pow(P.lz_factor, (double)sweeps_done));
    const double tol = dtype == QED_FP64 ? tol_s
                       : std::max(tol_s, dtype == QED_BF16 ? LZ_TOL_FLOOR_BF16 : LZ_TOL_FLOOR_FP32);
    LanczosResult R = lanczos(dev, lws, apply, T.ptr(), n_el, P.lz_steps, P.lz_cycles, tol);
    matvecs += R.matvecs;
    flops += R.matvecs * plan.flops;
    ctx->mv_count += R.matvecs;
    ctx->mv_flops += R.matvecs * plan.flops;
    double theta = R.theta;
    if (dtype != QED_FP64 && P.refine) {
        // FP64 Rayleigh quotient of the (normalised) Ritz vector
        Plan p64 = plan_matvec(T.legs, T.tab, ht, QED_FP64);
        p64.upload(dev);
        void* w64 = ws.get(dev, std::max<int64_t>(1, p64.ws_elems) * 8);
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
    if (std::getenv("QEDTTN_TRACE"))
        std::fprintf(stderr, "[qedttn] update node %d size %lld terms %zu theta %.15g resid %.3g E %.15g\n",
                     n, (long long)n_el, ht.size(), theta, R.resid, energy);
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
        update(n, nu);
        if (trace) {
            dev->sync();
            std::fprintf(stderr, "[qedttn] update node %d: %.3f s\n", n,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count());
        }
    }
    dev->sync();
    auto t1 = std::chrono::steady_clock::now();
    ++sweeps_done;
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
