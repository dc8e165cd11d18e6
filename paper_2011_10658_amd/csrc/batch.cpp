// Batched node updates: many independent tree nodes of uneven shape share
// one grouped block-GEMM launch per contraction stage and one segmented
// Lanczos (one recurrence per node, FP64 arithmetic; an FP32 plan keeps the
// basis in FP32).  A whole Lanczos cycle is
// captured once into a HIP graph and replayed.  The GEMM tile shape and
// operand pipeline of every stage can be chosen by timing (autotuner)
// instead of the padding and reduction-length heuristics.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <type_traits>

#include "engine.h"

namespace qed {

// ---------------------------------------------------------------------
// segmented Lanczos
// ---------------------------------------------------------------------
void SegLanczos::setup(Dev* dev, const std::vector<int64_t>& seg_off, int64_t NN, int mm, bool basis32) {
    nseg = (int)seg_off.size() - 1;
    N = NN;
    m = mm;
    b32 = basis32 && m + 1 <= 32;
    const int64_t CH = 4096;
    std::vector<SegChunk> ch;
    std::vector<int> c0;
    for (int s = 0; s < nseg; ++s) {
        c0.push_back((int)ch.size());
        for (int64_t lo = seg_off[s]; lo < seg_off[s + 1]; lo += CH)
            ch.push_back(SegChunk{s, 0, lo, std::min(lo + CH, seg_off[s + 1])});
    }
    c0.push_back((int)ch.size());
    nch = (int)ch.size();
    chunks = std::make_shared<DBuf>(dev, ch.size() * sizeof(SegChunk));
    seg_c0 = std::make_shared<DBuf>(dev, c0.size() * sizeof(int));
    dev->upload(chunks->p, ch.data(), ch.size() * sizeof(SegChunk));
    dev->upload(seg_c0->p, c0.data(), c0.size() * sizeof(int));
    V = std::make_shared<DBuf>(dev, (size_t)(m + 1) * N * (b32 ? sizeof(float) : sizeof(double)));
    w = std::make_shared<DBuf>(dev, (size_t)N * sizeof(double));
    const size_t ps = (size_t)nseg * LDS * sizeof(double);
    alpha = std::make_shared<DBuf>(dev, ps);
    beta = std::make_shared<DBuf>(dev, ps);
    coef = std::make_shared<DBuf>(dev, ps);
    coef2 = std::make_shared<DBuf>(dev, ps);
    sv = std::make_shared<DBuf>(dev, ps);
    work = std::make_shared<DBuf>(dev, (size_t)nseg * 256 * sizeof(double));
    st = std::make_shared<DBuf>(dev, (size_t)nseg * sizeof(LState));
    partial = std::make_shared<DBuf>(dev, (size_t)(LDS) * nch * sizeof(double));
    pv = std::make_shared<DBuf>(dev, (size_t)nch * sizeof(double));
    pi = std::make_shared<DBuf>(dev, (size_t)nch * sizeof(int64_t));
    nrm = std::make_shared<DBuf>(dev, (size_t)nseg * LDN * sizeof(double));
    fac = std::make_shared<DBuf>(dev, (size_t)nseg * sizeof(double));
}

void SegLanczos::cycle(const std::function<void(const double*, const float*, double*)>& apply, double* x,
                       hipStream_t s) {
    const SegChunk* ch = chunks->as<SegChunk>();
    const int* c0 = seg_c0->as<int>();
    double* wp = w->as<double>();
    double* al = alpha->as<double>();
    double* be = beta->as<double>();
    double* co = coef->as<double>();
    double* co2 = coef2->as<double>();
    double* part = partial->as<double>();
    double* nr = nrm->as<double>();
    LState* sp = st->as<LState>();
    auto run = [&](auto* Vp) {
        using TV = typename std::remove_pointer<decltype(Vp)>::type;
        constexpr bool F64 = std::is_same<TV, double>::value;
        seg_dots<double>(x, N, 1, x, ch, nch, c0, nseg, part, nr + 0, LDN, 1, sp, 0, s);
        seg_init(sp, nseg, m, nr + 0, LDN, s);
        seg_start<TV>(Vp, x, nr + 0, LDN, ch, nch, s);
        for (int j = 0; j < m; ++j) {
            TV* vj = Vp + (int64_t)j * N;
            if constexpr (F64) apply(vj, nullptr, wp);
            else apply(nullptr, vj, wp);
            seg_dots<TV>(vj, N, 1, wp, ch, nch, c0, nseg, part, al + j, LDS, 0, sp, 1, s);
            // three-term recurrence, classical Gram-Schmidt against V with a
            // second pass where a segment's first one removed more than half
            // of |w|^2, norm: three fused passes over the basis
            if (seg_fused<TV>(0, wp, Vp, N, 0, j, al, be, LDS, nullptr, nullptr, ch, nch, c0, nseg, part, co, LDS,
                              sp, s)) {
                seg_fused<TV>(1, wp, Vp, N, j + 1, j, al, be, LDS, co, co, ch, nch, c0, nseg, part, co2, LDS, sp, s);
                seg_fused<TV>(2, wp, Vp, N, j + 1, j, al, be, LDS, co2, co, ch, nch, c0, nseg, part, nr + 1, LDN, sp,
                              s);
            } else {
                // (an FP32 basis always fits the fused passes: m + 1 <= 32)
                if constexpr (F64) {
                    seg_three_term(wp, Vp, N, j, al, be, LDS, ch, nch, sp, s);
                    for (int pass = 0; pass < 2; ++pass) {
                        seg_dots<double>(Vp, N, j + 1, wp, ch, nch, c0, nseg, part, co, LDS, 0, sp, 1, s);
                        seg_subtract(wp, Vp, N, j + 1, co, LDS, ch, nch, sp, s);
                    }
                    seg_dots<double>(wp, N, 1, wp, ch, nch, c0, nseg, part, nr + 1, LDN, 0, sp, 1, s);
                }
            }
            seg_beta(nr + 1, LDN, al, be, LDS, j, sp, nseg, 1e-14, s);
            seg_next<TV>(Vp, N, j, wp, be, LDS, ch, nch, sp, s);
        }
        seg_tridiag(al, be, LDS, sv->as<double>(), sp, work->as<double>(), nseg, s);
        seg_ritz<TV>(x, Vp, N, sv->as<double>(), LDS, ch, nch, sp, s);
        seg_dots<double>(x, N, 1, x, ch, nch, c0, nseg, part, nr + 2, LDN, 1, sp, 0, s);
        seg_normalise_sign(x, ch, nch, c0, nseg, nr + 2, LDN, pv->as<double>(), pi->as<int64_t>(),
                           fac->as<double>(), s);
    };
    if (b32) run(V->as<float>());
    else run(V->as<double>());
}

// ---------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------
static std::string stage_key(const Plan& P, size_t s) {
    // shape signature: dtype, job count and the sums of extents (the
    // leading "p" marks entries that store tile shape + 4 pipeline)
    std::ostringstream o;
    int64_t jm = 0, jn = 0, jk = 0, jb = 0;
    for (const GJob& J : P.jobs[s]) {
        jm += J.M;
        jn += J.N;
        jb += J.batch;
        for (int p = J.p0; p < J.p1; ++p) jk += (int64_t)P.prods[s][p].K * P.prods[s][p].nred;
    }
    o << "p" << P.dtype << ":" << P.jobs[s].size() << ":" << jm << ":" << jn << ":" << jk << ":" << jb;
    return o.str();
}

void Tuner::load() {
    if (path.empty()) return;
    std::ifstream f(path);
    std::string k;
    int v;
    while (f >> k >> v) cache[k] = v;
}

void Tuner::save() const {
    if (path.empty()) return;
    std::ofstream f(path);
    for (auto& kv : cache) f << kv.first << " " << kv.second << "\n";
}

void Tuner::tune(Dev* dev, Plan& P, void* ws, void* x, void* y) {
    if (!on) return;
    bool changed = false;
    for (size_t s = 0; s < P.jobs.size(); ++s) {
        if (!P.ntiles[s] || P.sumk[s]) continue;
        const std::string key = stage_key(P, s);
        auto it = cache.find(key);
        if (it != cache.end()) {
            const int sh = it->second % 4, pp = it->second / 4;
            if (sh < GEMM_NSHAPES && P.pipe_valid(s, pp, sh)) {
                P.set_shape(dev, (int)s, sh);
                P.pipe[s] = (char)pp;
                continue;
            }
        }
        // every (tile shape, pipeline) pair the stage allows; BF16 stages
        // have one pipeline
        int best = P.shape[s] + 4 * P.pipe[s];
        float best_ms = -1.0f;
        for (int sh = 0; sh < GEMM_NSHAPES; ++sh)
            for (int pp = 0; pp < (P.dtype == QED_BF16 ? 1 : GEMM_NPIPES); ++pp) {
                if (!P.pipe_valid(s, pp, sh)) continue;
                if (pp == GEMM_PIPE_SKINNY && sh != 0) continue;   // the tile shape does not apply
                P.set_shape(dev, (int)s, sh);
                P.pipe[s] = (char)pp;
                hipEvent_t a, b;
                dev->check(hipEventCreate(&a), "event");
                dev->check(hipEventCreate(&b), "event");
                P.run_stage(dev, (int)s, ws, x, y);   // warm-up
                dev->check(hipEventRecord(a, dev->stream), "event");
                for (int r = 0; r < 3; ++r) P.run_stage(dev, (int)s, ws, x, y);
                dev->check(hipEventRecord(b, dev->stream), "event");
                dev->sync();
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, a, b);
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
                if (best_ms < 0 || ms < best_ms) {
                    best_ms = ms;
                    best = sh + 4 * pp;
                }
            }
        P.set_shape(dev, (int)s, best % 4);
        P.pipe[s] = (char)(best / 4);
        cache[key] = best;
        changed = true;
    }
    if (changed) save();
}

// ---------------------------------------------------------------------
// batch object
// ---------------------------------------------------------------------
void HeffBatch::matvec(const double* x, double* y, hipStream_t s) {
    Dev* dev = &ctx->dev;
    hipStream_t keep = dev->stream;
    dev->stream = s;
    if (plan.dtype == QED_FP64) {
        plan.run(dev, ws->p, (void*)x, (void*)y);
    } else {
        to_compute(plan.dtype, x, xc->p, off.back(), s);
        plan.run(dev, ws->p, xc->p, yc->p);
        from_compute(plan.dtype, yc->p, y, off.back(), s);
    }
    dev->stream = keep;
}

void HeffBatch::matvec32(const float* x, double* y, hipStream_t s) {
    Dev* dev = &ctx->dev;
    hipStream_t keep = dev->stream;
    dev->stream = s;
    plan.run(dev, ws->p, (void*)x, yc->p);
    from_compute(plan.dtype, yc->p, y, off.back(), s);
    dev->stream = keep;
}

HeffBatch::~HeffBatch() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (stream) {
        (void)hipStreamSynchronize(stream);
        (void)hipStreamDestroy(stream);
    }
}

}  // namespace qed
