// Hand-written adjoint of the effective-Hamiltonian application (the
// reverse-mode derivative of y = sum_k c_k A_k (x) B_k (x) C_k x with
// respect to x, every factor and every coefficient).
#include <algorithm>
#include <cmath>

#include "engine.h"

namespace qed {

namespace {

OpP transpose_op(Dev* dev, const LegOpD& A) {
    OpP T = make_op(dev, A.leg, -A.lay.delta, false);
    std::vector<int64_t> blk;
    for (int s = 0; s < A.leg.nsec(); ++s) {
        const int o = A.lay.out_of_in[s];
        if (o < 0) continue;
        // transposed op maps sector o to sector s
        blk.insert(blk.end(), {A.lay.off[s], T->lay.off[o], (int64_t)A.leg.n[o], (int64_t)A.leg.n[s]});
    }
    if (!blk.empty()) {
        DBuf d(dev, blk.size() * sizeof(int64_t));
        dev->upload(d.p, blk.data(), blk.size() * sizeof(int64_t));
        launch_transpose_blocks(A.f64(), (double*)T->d64->p, d.as<int64_t>(), (int)blk.size() / 4,
                                dev->stream);
        dev->sync();
    }
    return T;
}

}  // namespace

void Heff::build_adjoint() {
    Dev* dev = &ctx->dev;
    Adjoint& J = adj;
    const int dtype = plan.dtype;
    const int es = dtype_size(dtype);
    // xbar: the same schedule with every factor transposed
    std::vector<HTerm> tt;
    J.opT.assign(terms.size(), {});
    for (size_t k = 0; k < terms.size(); ++k) {
        HTerm h{terms[k].coef, {nullptr, nullptr, nullptr}};
        for (int e = 0; e < 3; ++e)
            if (terms[k].op[e]) {
                h.op[e] = transpose_op(dev, *terms[k].op[e]);
                J.opT[k].push_back(h.op[e]);
            }
        tt.push_back(h);
    }
    J.xbar = Plan();
    J.xbar.dtype = dtype;
    append_matvec(J.xbar, legs, tab, tt, 0);
    J.xbar.upload(dev);
    // gradients: one output per present factor, unscaled (coefficient 1)
    J.goff.assign(terms.size(), {-1, -1, -1});
    J.gsize = 0;
    std::vector<std::vector<RTerm>> rt(3);
    std::vector<std::vector<ContractOut>> outs(3);
    for (size_t k = 0; k < terms.size(); ++k)
        for (int e = 0; e < 3; ++e) {
            const OpP& A = terms[k].op[e];
            if (!A || !A->lay.size) continue;
            J.goff[k][e] = J.gsize;
            J.gsize += (A->lay.size + 63) & ~(int64_t)63;
        }
    J.G = std::make_shared<DBuf>(dev, std::max<int64_t>(1, J.gsize) * es);
    J.G64 = std::make_shared<DBuf>(dev, std::max<int64_t>(1, J.gsize) * sizeof(double));
    for (size_t k = 0; k < terms.size(); ++k)
        for (int e = 0; e < 3; ++e) {
            if (J.goff[k][e] < 0) continue;
            const OpP& A = terms[k].op[e];
            const int f1 = e == 0 ? 1 : 0, f2 = e == 2 ? 1 : 2;
            GRef base{(const char*)J.G->p + J.goff[k][e] * es, 0, TAG_ABS, 0};
            outs[e].push_back(ContractOut{A->leg, A->lay, base});
            rt[e].push_back(RTerm{1.0, terms[k].op[f1], terms[k].op[f2], (int)outs[e].size() - 1});
        }
    J.grads = Plan();
    J.grads.dtype = dtype;
    // the three legs' contractions are independent: they share stages, so
    // each stage is one launch with the tiles of all three
    bool any = false;
    for (int e = 0; e < 3; ++e)
        if (!rt[e].empty()) {
            append_contract(J.grads, legs, tab, GRef{nullptr, 0, TAG_X, 0}, GRef{nullptr, 0, TAG_Y, 0},
                            e, rt[e], outs[e], false, 0);
            any = true;
        }
    if (any) split_long_reductions(J.grads, 2);
    J.grads.upload(dev);
    if (dtype != QED_FP64) J.ybc = std::make_shared<DBuf>(dev, tab.size() * es);
    // c_bar_k = <G_k, A_k> on the term's first present factor; a term with
    // no factor gets <ybar, x>, whose pointers are bound per call
    J.dots.clear();
    for (size_t k = 0; k < terms.size(); ++k) {
        int first = -1;
        for (int e = 0; e < 3 && first < 0; ++e)
            if (J.goff[k][e] >= 0) first = e;
        AdjSeg s{};
        s.dot = (int)k;
        if (first >= 0) {
            s.src = J.G64->as<double>() + J.goff[k][first];
            s.a = terms[k].op[first]->f64();
            s.n = terms[k].op[first]->lay.size;
        }
        J.dots.push_back(s);
    }
    J.ddots = std::make_shared<DBuf>(dev, std::max<size_t>(1, J.dots.size()) * sizeof(AdjSeg));
    J.cbar = std::make_shared<DBuf>(dev, std::max<size_t>(1, terms.size()) * sizeof(double));
    J.built = true;
}

void Heff::adjoint(const double* x, const double* ybar, double* xbar, double* const* opbar,
                   double* coefbar) {
    Dev* dev = &ctx->dev;
    if (!adj.built) build_adjoint();
    Adjoint& J = adj;
    const int dtype = plan.dtype;
    const int es = dtype_size(dtype);
    const int64_t n = tab.size();
    // segment lists of the gradient post-processing first: their uploads
    // synchronise the stream, which costs nothing before any work is queued
    std::vector<AdjSeg> sc;
    int64_t maxn = 0;
    if (opbar)
        for (size_t k = 0; k < terms.size(); ++k)
            for (int e = 0; e < 3; ++e) {
                if (J.goff[k][e] < 0 || !opbar[3 * k + e]) continue;
                AdjSeg sg{};
                sg.src = J.G64->as<double>() + J.goff[k][e];
                sg.dst = opbar[3 * k + e];
                sg.n = terms[k].op[e]->lay.size;
                sg.scale = terms[k].coef;
                sg.dot = -1;
                maxn = std::max(maxn, sg.n);
                sc.push_back(sg);
            }
    void* dsc = nullptr;
    if (!sc.empty()) {
        dsc = J.dscale.get(dev, sc.size() * sizeof(AdjSeg));
        dev->upload(dsc, sc.data(), sc.size() * sizeof(AdjSeg));
    }
    if (coefbar) {
        // terms without a factor contract ybar with x (bound per call)
        std::vector<AdjSeg> ds = J.dots;
        for (AdjSeg& sg : ds)
            if (!sg.src) {
                sg.src = ybar;
                sg.a = x;
                sg.n = n;
            }
        dev->upload(J.ddots->p, ds.data(), ds.size() * sizeof(AdjSeg));
    }
    // operands in the compute dtype
    const void* xc_ = x;
    const void* yb_ = ybar;
    if (dtype != QED_FP64) {
        to_compute(dtype, x, xc->p, n, dev->stream);
        to_compute(dtype, ybar, J.ybc->p, n, dev->stream);
        xc_ = xc->p;
        yb_ = J.ybc->p;
    }
    if (xbar) {
        void* w = J.ws.get(dev, std::max<int64_t>(1, J.xbar.ws_elems) * es);
        if (dtype == QED_FP64) {
            J.xbar.run(dev, w, (void*)ybar, xbar);
        } else {
            J.xbar.run(dev, w, J.ybc->p, yc->p);
            from_compute(dtype, yc->p, xbar, n, dev->stream);
        }
        ctx->mv_flops += J.xbar.flops;
        ctx->mv_count += 1;
    }
    bool need_grads = coefbar != nullptr;
    if (opbar)
        for (size_t k = 0; k < terms.size(); ++k)
            for (int e = 0; e < 3; ++e)
                if (opbar[3 * k + e] && J.goff[k][e] >= 0) need_grads = true;
    if (!need_grads) return;
    void* w = J.ws.get(dev, std::max<int64_t>(1, J.grads.ws_elems) * es);
    J.grads.run(dev, w, (void*)xc_, (void*)yb_);
    // unscaled gradients in FP64
    launch_scale_to_f64(J.G->p, dtype, J.G64->as<double>(), J.gsize, 1.0, dev->stream);
    // factor cotangents c_k G: one launch over every requested factor
    if (dsc) launch_adj_scale((const AdjSeg*)dsc, (int)sc.size(), maxn, dev->stream);
    if (coefbar) {
        launch_adj_dots(J.ddots->as<AdjSeg>(), (int)J.dots.size(), J.cbar->as<double>(), dev->stream);
        dev->download(coefbar, J.cbar->p, terms.size() * sizeof(double));
    }
    dev->check(hipGetLastError(), "adjoint");
}

}  // namespace qed
