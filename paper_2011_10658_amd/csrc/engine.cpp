// Host side of the device engine: memory, plans, Lanczos, the TTN sweep.
//
// Every contraction of the node update is planned here as a list of
// block-level GEMM jobs and executed by the grouped batch-reduce GEMM
// kernel in stages:
//   H_eff matvec  (Methods, "Tensor Networks" steps (i)-(ii)):
//     stage 0: T1 = x  x_p C_k   for every term with C_k != 1, every block
//     stage 1: T2 = T1 x_r B_k   (batched over the l index)
//     stage 2: y_b = sum_k c_k A_k T2_k  (or c_k T2_k when A_k = 1): one job
//              per output block sums every term and input block that lands
//              on it, so y is written once, with no atomics.
//   renormalisation of the environment across a leg (step (iii) moves the
//   isometry centre): T = n x_f1 A x_f2 B, then O[out, in] = sum over the
//   two other legs of n * T, again one job per output block.
#include "engine.h"

#include <algorithm>
#include <type_traits>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstring>
#include <tuple>

namespace qed {

// ---------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------
void Dev::check(hipError_t e, const char* what) {
    if (e != hipSuccess)
        fail(QED_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// size class of a request: multiples of 256 B up to 4 KiB, above that
// eight classes per power of two (at most 12.5% unused)
static size_t size_class(size_t bytes) {
    if (bytes <= 4096) return std::max<size_t>(256, (bytes + 255) / 256 * 256);
    int k = 63 - __builtin_clzll((unsigned long long)bytes);
    const size_t step = (size_t)1 << (k - 3);
    return (bytes + step - 1) / step * step;
}

// blocks above this total go straight back to the pool
static constexpr size_t CACHE_LIMIT = (size_t)8 << 30;

static bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

void* Dev::alloc(size_t bytes) {
    if (device < 0) fail(QED_ERR_BAD_STATE, "host-only context has no device memory");
    used = true;
    void* p = nullptr;
    if (ualloc) {
        p = ualloc((uint64_t)bytes, (void*)stream, user);
        if (!p) fail(QED_ERR_OOM, "allocator hook returned NULL");
        return p;
    }
    if (capturing(stream)) {
        // a graph owns what is allocated during its capture
        check(hipMallocAsync(&p, bytes, stream), "hipMallocAsync");
        return p;
    }
    const size_t cls = size_class(bytes);
    auto range = cache.equal_range(cls);
    for (auto it = range.first; it != range.second; ++it)
        if (it->second.stream == stream) {
            p = it->second.p;
            cache.erase(it);
            cached_bytes -= cls;
            live[p] = cls;
            return p;
        }
    hipError_t e = hipMallocAsync(&p, cls, stream);
    if (e == hipErrorOutOfMemory && !cache.empty()) {
        (void)hipGetLastError();
        sync();
        trim();
        sync();
        e = hipMallocAsync(&p, cls, stream);
    }
    if (e == hipErrorOutOfMemory) fail(QED_ERR_OOM, "out of device memory");
    check(e, "hipMallocAsync");
    live[p] = cls;
    return p;
}

void Dev::release(void* p) {
    if (!p) return;
    if (ufree) {
        ufree(p, (void*)stream, user);
        return;
    }
    auto it = live.find(p);
    if (it == live.end()) {   // allocated during a capture
        (void)hipFreeAsync(p, stream);
        return;
    }
    const size_t cls = it->second;
    live.erase(it);
    if (capturing(stream) || cached_bytes + cls > CACHE_LIMIT) {
        (void)hipFreeAsync(p, stream);
        return;
    }
    cache.emplace(cls, Cached{p, stream});
    cached_bytes += cls;
}

void Dev::trim() {
    for (auto& kv : cache) (void)hipFreeAsync(kv.second.p, kv.second.stream);
    cache.clear();
    cached_bytes = 0;
}

void Dev::restream(hipStream_t s) {
    for (auto& kv : cache) kv.second.stream = s;
}

Dev::~Dev() {
    // the streams may be gone by now: synchronous frees
    for (auto& kv : cache) (void)hipFree(kv.second.p);
    if (ring) {
        (void)hipDeviceSynchronize();
        (void)hipHostFree(ring);
    }
}

void Dev::sync() {
    check(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (stream == ring_stream) ring_pos = 0;   // every staged copy has completed
}

static constexpr size_t RING_BYTES = (size_t)64 << 20;

bool Dev::stage(void* dst, const void* src, size_t bytes) {
    if (bytes > RING_BYTES / 4 || ring_failed || capturing(stream)) return false;
    if (!ring) {
        if (hipHostMalloc((void**)&ring, RING_BYTES, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            ring = nullptr;
            ring_failed = true;
            return false;
        }
        ring_stream = stream;
        ring_pos = 0;
    }
    if (stream != ring_stream) {   // copies staged on another stream: let them finish
        if (ring_pos) check(hipStreamSynchronize(ring_stream), "hipStreamSynchronize");
        ring_stream = stream;
        ring_pos = 0;
    }
    size_t at = (ring_pos + 255) & ~(size_t)255;
    if (at + bytes > RING_BYTES) {
        sync();
        at = 0;
    }
    std::memcpy(ring + at, src, bytes);
    check(hipMemcpyAsync(dst, ring + at, bytes, hipMemcpyHostToDevice, stream), "upload");
    ring_pos = at + bytes;
    return true;
}

void Dev::upload(void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    if (stage(dst, src, bytes)) return;
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream), "upload");
    sync();  // the host buffer may be temporary
}

void Dev::download(void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream), "download");
    sync();
}

const void* LegOpD::data(int dtype) {
    if (dtype == QED_FP64) return f64();
    BufP& d = dtype == QED_BF16 ? d16 : d32;
    if (!d && lay.size) {
        d = std::make_shared<DBuf>(dev, lay.size * dtype_size(dtype));
        to_compute(dtype, f64(), d->p, lay.size, dev->stream);
    }
    return d ? d->p : nullptr;
}

void to_compute(int dtype, const double* a, void* b, int64_t n, hipStream_t s) {
    if (dtype == QED_BF16) launch_f64_to_bf16(a, b, n, s);
    else if (dtype == QED_FP32) launch_f64_to_f32(a, (float*)b, n, s);
    else fail(QED_ERR_INVALID_ARG, "to_compute: FP64 needs no conversion");
}

void from_compute(int dtype, const void* a, double* b, int64_t n, hipStream_t s) {
    if (dtype == QED_BF16) launch_bf16_to_f64(a, b, n, 1.0, s);
    else if (dtype == QED_FP32) launch_f32_to_f64((const float*)a, b, n, s);
    else fail(QED_ERR_INVALID_ARG, "from_compute: FP64 needs no conversion");
}

void prepare_f32_copies(Dev* dev, const std::vector<LegOpD*>& ops) {
    std::vector<ConvSeg> segs;
    for (LegOpD* o : ops) {
        if (!o || o->d32 || !o->lay.size || !o->d64) continue;
        o->d32 = std::make_shared<DBuf>(dev, o->lay.size * sizeof(float));
        segs.push_back(ConvSeg{o->f64(), o->d32->p, o->lay.size});
    }
    if (segs.empty()) return;
    DBuf list(dev, segs.size() * sizeof(ConvSeg));
    dev->upload(list.p, segs.data(), segs.size() * sizeof(ConvSeg));
    launch_f64_to_f32_segs(list.as<ConvSeg>(), (int)segs.size(), dev->stream);
    dev->check(hipGetLastError(), "conversion launch");
}

OpP make_op(Dev* dev, const Leg& leg, int delta, bool zero) {
    auto o = std::make_shared<LegOpD>();
    o->dev = dev;
    o->leg = leg;
    o->lay = make_op_layout(leg, delta);
    if (o->lay.size) {
        o->d64 = std::make_shared<DBuf>(dev, o->lay.size * sizeof(double));
        if (zero) launch_fill(o->d64->as<double>(), o->lay.size, 0.0, dev->stream);
    }
    return o;
}

// ---------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------
namespace {

GRef gabs(const void* p) { return GRef{p, 0, TAG_ABS, 0}; }
GRef gtag(int tag, int64_t off) { return GRef{nullptr, off, tag, 0}; }

// a dense block: pointer, sector indices and extents per leg
struct BV {
    GRef p;
    int s[3];
    int n[3];
};

struct Builder {
    Plan& P;
    int esize;
    explicit Builder(Plan& p) : P(p), esize(dtype_size(p.dtype)) {}

    GRef ws(int64_t n) {
        GRef r = gtag(TAG_WS, P.ws_elems);
        P.ws_elems += (n + 63) & ~(int64_t)63;
        return r;
    }
    void stage(int s) {
        while ((int)P.jobs.size() <= s) {
            P.jobs.emplace_back();
            P.prods.emplace_back();
            P.stage_flops.push_back(0.0);
        }
        while ((int)P.fjobs.size() <= s) {
            P.fjobs.emplace_back();
            P.fprods.emplace_back();
            P.fstage_flops.push_back(0.0);
        }
    }
    void add_flops(int s, double f) {
        stage(s);
        P.stage_flops[s] += f;
        P.flops += f;
    }
    void job1(int s, GRef C, int M, int N, int ldc, int batch, int64_t bsC, const GProd& p) {
        stage(s);
        GJob j{};
        j.C = C;
        j.bsC = bsC;
        if (p.nsb) {   // split output columns like the input (mode on r)
            j.nsc = p.nsb;
            j.noc = bsC;
            j.bsC = 0;
        }
        j.M = M;
        j.N = N;
        j.ldc = ldc;
        j.batch = batch;
        j.p0 = (int)P.prods[s].size();
        P.prods[s].push_back(p);
        j.p1 = j.p0 + 1;
        j.acc = 0;
        P.jobs[s].push_back(j);
    }
    // the product that applies `op` (block opblk, n_out x n_in) on leg e
    // of block `in`; returns the job shape through M, N, ldc, batch, bsC
    static GProd mode_prod(const BV& in, int e, GRef opblk, int nout, double alpha, int& M, int& N,
                           int& ldc, int& batch, int64_t& bsC) {
        GProd p{};
        p.alpha = alpha;
        p.nred = 1;
        const int n0 = in.n[0], n1 = in.n[1], n2 = in.n[2];
        if (e == 2) {
            p.A = in.p; p.lda = n2; p.tA = 0;
            p.B = opblk; p.ldb = n2; p.tB = 1;
            p.K = n2;
            M = n0 * n1; N = nout; ldc = nout; batch = 1; bsC = 0;
        } else if (e == 1) {
            // n0 matrices (n1 x n2) side by side: one GEMM over N = n0 n2
            p.A = opblk; p.lda = n1; p.tA = 0;
            p.B = in.p; p.ldb = n2; p.tB = 0;
            p.nsb = n2; p.nob = (int64_t)n1 * n2;
            p.K = n1;
            M = nout; N = n0 * n2; ldc = n2; batch = 1; bsC = (int64_t)nout * n2;
        } else {
            p.A = opblk; p.lda = n0; p.tA = 0;
            p.B = in.p; p.ldb = n1 * n2; p.tB = 0;
            p.K = n0;
            M = nout; N = n1 * n2; ldc = n1 * n2; batch = 1; bsC = 0;
        }
        return p;
    }
    // fresh-workspace mode product; returns false if the output sector
    // does not exist
    bool mode(int s, const BV& in, int e, LegOpD& op, const Leg& leg, BV& out, bool count = true) {
        const int so = op.lay.out_of_in[in.s[e]];
        if (so < 0) return false;
        const int nout = leg.n[so];
        GRef opblk = gabs((const char*)op.data(P.dtype) + op.lay.off[in.s[e]] * esize);
        int M, N, ldc, batch;
        int64_t bsC;
        out = in;
        out.s[e] = so;
        out.n[e] = nout;
        const int64_t sz = (int64_t)out.n[0] * out.n[1] * out.n[2];
        out.p = ws(sz);
        GProd p = mode_prod(in, e, opblk, nout, 1.0, M, N, ldc, batch, bsC);
        job1(s, out.p, M, N, ldc, batch, bsC, p);
        if (count) add_flops(s, 2.0 * in.n[0] * in.n[1] * in.n[2] * nout);
        return true;
    }
};

int64_t key3(int a, int b, int c) { return ((int64_t)a * 4096 + b) * 4096 + c; }

}  // namespace

// Tile order of a launch.  Workgroup i runs on XCD i mod 8; tiles that
// read the same operand panel are kept on one XCD, one after another, so
// the panel is fetched from HBM once and then served by that XCD's L2.
// Usually the shared panel is B: the tiles of one output column panel
// (same job, batch entry and column tile; all row tiles).  Where many jobs
// multiply the same A operand (the first mode product of an H_eff
// application: every term's factor on the last leg applied to the same
// input block), the shared panel is A instead: the tiles of one row tile
// across all those jobs and their column tiles.  Panels go to the
// least-loaded XCD; slot 8 k + x holds the k-th tile of XCD x, and XCDs
// with fewer tiles are padded with empty tiles (job -1), which return at
// once.
constexpr int NXCD = 8;

static std::vector<GTile> make_tiles(const std::vector<GJob>& jobs, const std::vector<GProd>& prods,
                                     int sh) {
    const int TM = gemm_tm(sh), TN = gemm_tn(sh);
    std::vector<std::vector<GTile>> per(NXCD);
    auto least = [&]() {
        int x = 0;
        for (int y = 1; y < NXCD; ++y)
            if (per[y].size() < per[x].size()) x = y;
        return x;
    };
    // jobs grouped by their A operand (all products of a job must agree)
    std::map<std::tuple<const void*, int64_t, int, int, int64_t>, std::vector<int>> by_a;
    bool a_ok = true;
    for (size_t j = 0; j < jobs.size() && a_ok; ++j) {
        const GJob& J = jobs[j];
        if (J.p1 <= J.p0 || J.batch != 1) {
            a_ok = false;
            break;
        }
        const GProd& f = prods[J.p0];
        for (int q = J.p0; q < J.p1; ++q) {
            const GProd& P = prods[q];
            if (P.ident || P.A.abs != f.A.abs || P.A.off != f.A.off || P.A.tag != f.A.tag ||
                P.lda != f.lda || P.tA != f.tA || P.rsA != f.rsA)
                a_ok = false;
        }
        by_a[std::make_tuple(f.A.abs, f.A.off, f.A.tag, f.lda, f.rsA)].push_back((int)j);
    }
    if (a_ok && !jobs.empty() && by_a.size() * 2 <= jobs.size()) {
        for (const auto& g : by_a) {
            int tmax = 0;
            for (int j : g.second) tmax = std::max(tmax, (jobs[j].M + TM - 1) / TM);
            for (int a = 0; a < tmax; ++a) {
                const int x = least();
                for (int j : g.second) {
                    if (a >= (jobs[j].M + TM - 1) / TM) continue;
                    const int tn = (jobs[j].N + TN - 1) / TN;
                    for (int c = 0; c < tn; ++c) per[x].push_back(GTile{j, 0, a, c});
                }
            }
        }
    } else {
        for (size_t j = 0; j < jobs.size(); ++j) {
            const GJob& J = jobs[j];
            const int tm = (J.M + TM - 1) / TM, tn = (J.N + TN - 1) / TN;
            for (int b = 0; b < J.batch; ++b)
                for (int c = 0; c < tn; ++c) {
                    const int x = least();
                    for (int a = 0; a < tm; ++a) per[x].push_back(GTile{(int)j, b, a, c});
                }
        }
    }
    size_t slots = 0;
    for (const auto& v : per) slots = std::max(slots, v.size());
    std::vector<GTile> tiles(slots * NXCD, GTile{-1, 0, 0, 0});
    for (int x = 0; x < NXCD; ++x)
        for (size_t k = 0; k < per[x].size(); ++k) tiles[k * NXCD + x] = per[x][k];
    return tiles;
}

// Strip tiles of a skinny stage: jobs grouped by their first product's A
// panel; strip a of every job of a group goes to one XCD, so the group's
// panel strip is fetched once into that XCD's L2.
static std::vector<GTile> make_skinny_tiles(const std::vector<GJob>& jobs, const std::vector<GProd>& prods,
                                            int RS) {
    std::vector<std::vector<GTile>> per(NXCD);
    std::map<std::tuple<const void*, int64_t, int>, std::vector<int>> by_a;
    for (size_t j = 0; j < jobs.size(); ++j) {
        const GProd& f = prods[jobs[j].p0];
        by_a[std::make_tuple(f.A.abs, f.A.off, f.A.tag)].push_back((int)j);
    }
    for (const auto& g : by_a) {
        int tmax = 0;
        for (int j : g.second) tmax = std::max(tmax, (jobs[j].M + RS - 1) / RS);
        for (int a = 0; a < tmax; ++a) {
            int x = 0;
            for (int y = 1; y < NXCD; ++y)
                if (per[y].size() < per[x].size()) x = y;
            for (int j : g.second)
                if (a < (jobs[j].M + RS - 1) / RS) per[x].push_back(GTile{j, 0, a, 0});
        }
    }
    size_t slots = 0;
    for (const auto& v : per) slots = std::max(slots, v.size());
    std::vector<GTile> tiles(slots * NXCD, GTile{-1, 0, 0, 0});
    for (int x = 0; x < NXCD; ++x)
        for (size_t k = 0; k < per[x].size(); ++k) tiles[k * NXCD + x] = per[x][k];
    return tiles;
}

// Tiles of fused jobs: per job, its group tiles in order, each with all
// of its row tiles one after another on the least-loaded XCD (the row
// tiles of a group tile read the same input columns).
static std::vector<GTile> make_fused_tiles(const std::vector<FJob>& jobs) {
    std::vector<std::vector<GTile>> per(NXCD);
    for (size_t j = 0; j < jobs.size(); ++j) {
        const FJob& J = jobs[j];
        const int tm = (J.M + FUSED_TM - 1) / FUSED_TM, tn = (J.G + J.ng - 1) / J.ng;
        for (int c = 0; c < tn; ++c) {
            int x = 0;
            for (int y = 1; y < NXCD; ++y)
                if (per[y].size() < per[x].size()) x = y;
            for (int a = 0; a < tm; ++a) per[x].push_back(GTile{(int)j, 0, a, c});
        }
    }
    size_t slots = 0;
    for (const auto& v : per) slots = std::max(slots, v.size());
    std::vector<GTile> tiles(slots * NXCD, GTile{-1, 0, 0, 0});
    for (int x = 0; x < NXCD; ++x)
        for (size_t k = 0; k < per[x].size(); ++k) tiles[k * NXCD + x] = per[x][k];
    return tiles;
}

static std::vector<GTile> make_sum_tiles(const std::vector<GJob>& jobs) {
    std::vector<GTile> tiles;
    for (size_t j = 0; j < jobs.size(); ++j) {
        const int64_t n = (int64_t)jobs[j].M * jobs[j].N;
        for (int b = 0; b < jobs[j].batch; ++b)
            for (int64_t c = 0; c * SUM_TILE < n; ++c) tiles.push_back(GTile{(int)j, b, (int)c, 0});
    }
    return tiles;
}

// QEDTTN_GEMM_PIPELINE=flat, =loop, =dma or =skinny forces one GEMM
// pipeline on every stage of the plans built afterwards (dma or skinny
// where a stage allows it, loop elsewhere); =nodma chooses as by default
// without the dma pipeline; anything else (or unset) chooses per stage:
// flat for short mean reductions, else dma where an FP32 stage allows it,
// else loop.  The
// skinny pipeline is not chosen by default: on the d = 267 bottom nodes
// its stage (180 MB of per-term intermediates written per product) runs
// at the flat pipeline's rate or below; the autotuner may still pick it.
static int forced_pipeline() {
    const char* v = std::getenv("QEDTTN_GEMM_PIPELINE");
    if (!v) return -1;
    if (!std::strcmp(v, "nodma")) return -2;
    if (!std::strcmp(v, "skinny")) return GEMM_PIPE_SKINNY;
    if (!std::strcmp(v, "flat")) return GEMM_PIPE_FLAT;
    if (!std::strcmp(v, "loop")) return GEMM_PIPE_LOOP;
    if (!std::strcmp(v, "dma")) return GEMM_PIPE_DMA;
    return -1;
}

// The LDS-DMA pipeline reads FP32 or FP64 operands with tA = tB = 0 through
// 32-bit byte offsets: every offset a tile forms (rows and reduction chunks
// padded to the tile) must stay below 2^31 bytes.
static bool dma_operands_ok(int esize, const std::vector<GJob>& jobs, const std::vector<GProd>& prods) {
    const int64_t LIM = ((int64_t)1 << 31) / esize;
    bool any = false;
    for (const GJob& J : jobs) {
        // the output block, stored through a buffer resource as well
        const int64_t M = std::max(J.M, 1), N = std::max(J.N, 1);
        if ((M - 1) * J.ldc + (J.nsc ? (N / J.nsc + 1) * J.noc + J.nsc : N - 1) >= LIM - 2) return false;
        for (int p = J.p0; p < J.p1; ++p) {
            const GProd& P = prods[p];
            if (P.ident) continue;
            if (P.tA || P.tB) return false;
            any = true;
            const int64_t nlast = (int64_t)J.N + 128;
            const int64_t co = P.nsb ? (nlast / P.nsb) * P.nob + P.nsb : nlast;
            if ((int64_t)(J.M + 128) * P.lda + P.K + 16 >= LIM) return false;
            if ((int64_t)(P.K + 16) * P.ldb + co >= LIM) return false;
        }
    }
    return any;
}

// The flat pipeline reads operands and writes its output through buffer
// resources with 32-bit byte offsets from each block's start: every element
// a tile reads or writes must lie within 2^31 bytes of it.
static bool flat_operands_ok(int esize, const std::vector<GJob>& jobs, const std::vector<GProd>& prods) {
    const int64_t LIM = ((int64_t)1 << 31) / esize - 2;
    for (const GJob& J : jobs) {
        // the output block (its tiles are stored the same way)
        const int64_t M = std::max(J.M, 1), N = std::max(J.N, 1);
        const int64_t omax = (M - 1) * J.ldc + (J.nsc ? (N / J.nsc + 1) * J.noc + J.nsc : N - 1);
        if (omax >= LIM) return false;
        for (int p = J.p0; p < J.p1; ++p) {
            const GProd& P = prods[p];
            if (P.ident) continue;
            const int64_t M = std::max(J.M, 1), N = std::max(J.N, 1), K = std::max(P.K, 1);
            const int64_t amax = P.tA ? (K - 1) * P.lda + (M - 1) : (M - 1) * P.lda + (K - 1);
            const int64_t cmax = P.nsb ? (N / P.nsb + 1) * P.nob + P.nsb : N - 1;
            const int64_t bmax = P.tB ? (N - 1) * P.ldb + (K - 1) : (K - 1) * P.ldb + cmax;
            if (amax >= LIM || bmax >= LIM) return false;
        }
    }
    return true;
}

// The skinny kernel takes stages whose every product is A B^T on a
// contiguous panel (lda = K, ldb = K, K <= SK_KMAX, one reduction term)
// into contiguous overwritten outputs of at most SK_NMAX columns (FP32 and
// FP64).
static bool skinny_operands_ok(int dtype, const std::vector<GJob>& jobs, const std::vector<GProd>& prods) {
    if (dtype != QED_FP32 && dtype != QED_FP64) return false;
    if (jobs.empty()) return false;
    for (const GJob& J : jobs) {
        if (J.batch != 1 || J.nsc || J.acc || J.ldc != J.N || J.N > SK_NMAX || J.N < 1 || J.p1 <= J.p0)
            return false;
        for (int p = J.p0; p < J.p1; ++p) {
            const GProd& P = prods[p];
            if (P.ident || P.tA || !P.tB || P.nred != 1 || P.lda != P.K || P.ldb != P.K || P.K > SK_KMAX ||
                P.K < 1 || P.nsb)
                return false;
        }
    }
    return true;
}

bool Plan::pipe_valid(size_t s, int pp, int sh) const {
    if (pp == GEMM_PIPE_SKINNY) return skinny_ok[s] != 0;
    if (pp == GEMM_PIPE_FLAT) return flat_ok[s] != 0;
    if (pp != GEMM_PIPE_DMA) return pp == GEMM_PIPE_LOOP;
    return (dtype == QED_FP32 || dtype == QED_FP64) && dma_ok[s] && brgemm_dma_shape(sh);
}

// QEDTTN_HEFF_FUSED=1 plans the terms with a bond-leg factor of every FP32
// and FP64 H_eff as fused stages where they apply; otherwise (the default)
// every H_eff runs as three mode-product stages.  On the d = 267 nodes the
// fused stages move about 3.5 times fewer bytes but run slower (each term's
// short reduction waits on fresh operand loads), so they are not the
// default.
static bool fused_enabled() {
    const char* v = std::getenv("QEDTTN_HEFF_FUSED");
    return v && !std::strcmp(v, "1");
}

void Plan::upload(Dev* dev) {
    hold.clear();
    dj.clear();
    dp.clear();
    dt.clear();
    std::vector<std::vector<GTile>> tiles;
    ntiles.clear();
    shape.clear();
    sumk.clear();
    pipe.clear();
    dma_ok.clear();
    flat_ok.clear();
    skinny_ok.clear();
    std::vector<std::vector<GTile>> stiles;
    for (size_t s = 0; s < jobs.size(); ++s) {
        bool only_ident = !jobs[s].empty();
        double ksum = 0.0, kn = 0.0;
        for (const GProd& p : prods[s])
            if (!p.ident) {
                only_ident = false;
                ksum += (double)p.K * p.nred;
                kn += 1.0;
            }
        sumk.push_back(only_ident ? 1 : 0);
        dma_ok.push_back((dtype == QED_FP32 || dtype == QED_FP64) && !only_ident &&
                                 dma_operands_ok(dtype_size(dtype), jobs[s], prods[s])
                             ? 1
                             : 0);
        flat_ok.push_back(flat_operands_ok(dtype_size(dtype), jobs[s], prods[s]) ? 1 : 0);
        skinny_ok.push_back(!only_ident && skinny_operands_ok(dtype, jobs[s], prods[s]) ? 1 : 0);
        stiles.push_back(skinny_ok.back() ? make_skinny_tiles(jobs[s], prods[s], skinny_rows(dtype))
                                          : std::vector<GTile>());
        // the tile shape that pads the stage's jobs least
        int best = GEMM_SHAPE_SQUARE;
        double best_area = -1.0;
        for (int sh = 0; sh < GEMM_NSHAPES; ++sh) {
            const int TM = gemm_tm(sh), TN = gemm_tn(sh);
            double area = 0.0;
            for (const GJob& J : jobs[s])
                area += (double)J.batch * ((J.M + TM - 1) / TM) * TM * ((J.N + TN - 1) / TN) * TN;
            if (best_area < 0 || area < best_area * 0.999) {
                best_area = area;
                best = sh;
            }
        }
        tiles.push_back(only_ident ? make_sum_tiles(jobs[s]) : make_tiles(jobs[s], prods[s], best));
        ntiles.push_back((int)tiles.back().size());
        shape.push_back(best);
        // short reductions per product: pipeline across products; long
        // ones through the LDS ring where the stage allows it (the
        // environment may force one pipeline, to compare them on one plan)
        const int forced = forced_pipeline();
        // (the FP64 ring is no faster than the register-staged loop on a
        // 267 x 267 x 64 node: two 4-byte loads per element, half the
        // occupancy; it stays a forced or tuned choice)
        int pp = kn > 0.0 && ksum / kn < 64.0 ? GEMM_PIPE_FLAT
                                              : (dtype == QED_FP32 ? GEMM_PIPE_DMA : GEMM_PIPE_LOOP);
        if (forced >= 0) pp = forced;
        if (forced == -2 && pp == GEMM_PIPE_DMA) pp = kn > 0.0 && ksum / kn < 64.0 ? GEMM_PIPE_FLAT : GEMM_PIPE_LOOP;
        if (!pipe_valid(s, pp, best)) pp = GEMM_PIPE_LOOP;
        pipe.push_back((char)pp);
    }
    if (std::getenv("QEDTTN_TRACE")) {
        static const char* pn[] = {"loop", "flat", "dma", "skinny"};
        for (size_t s = 0; s < jobs.size(); ++s) {
            size_t maxp = 0, single = 0;
            double out = 0.0, ain = 0.0, kk = 0.0, nn = 0.0;
            for (const GJob& J : jobs[s]) {
                const size_t np = (size_t)(J.p1 - J.p0);
                maxp = std::max(maxp, np);
                single += np == 1;
                out += (double)J.M * J.N * J.batch;
                nn += J.N;
                for (int p = J.p0; p < J.p1; ++p) {
                    ain += (double)J.M * prods[s][p].K * prods[s][p].nred * J.batch;
                    kk += prods[s][p].K;
                }
            }
            std::fprintf(stderr,
                         "[qedttn] plan stage %zu: %zu jobs (%zu of one product, at most %zu), %zu products, "
                         "output %.3e, A read %.3e elements, mean N %.1f, mean K %.1f, pipeline %s\n",
                         s, jobs[s].size(), single, maxp, prods[s].size(), out, ain,
                         jobs[s].empty() ? 0.0 : nn / jobs[s].size(), prods[s].empty() ? 0.0 : kk / prods[s].size(),
                         sumk[s] ? "sum" : pn[pipe[s] % 4]);
        }
    }
    // fused jobs of each stage
    const size_t S = jobs.size();
    fjobs.resize(S);
    fprods.resize(S);
    fstage_flops.resize(S, 0.0);
    std::vector<std::vector<GTile>> ftiles(S);
    dfj.clear();
    dfp.clear();
    dft.clear();
    dts.clear();
    nts.clear();
    nftiles.clear();
    fcs_rows.assign(S, 0);
    fcs_cols.assign(S, 0);
    for (size_t s = 0; s < S; ++s) {
        ftiles[s] = make_fused_tiles(fjobs[s]);
        nftiles.push_back((int)ftiles[s].size());
        for (const FJob& J : fjobs[s])
            for (int p = J.p0; p < J.p1; ++p)
                if (fprods[s][p].hasC) {
                    fcs_rows[s] = std::max(fcs_rows[s], fprods[s][p].np_in);
                    fcs_cols[s] = std::max(fcs_cols[s], (J.np + 15) & ~15);
                }
    }
    // one device buffer and one copy for the whole plan; arrays at 256-byte
    // aligned offsets
    std::vector<size_t> oj(S), op(S), ot(S), ofj(S), ofp(S), oft(S), ost(S);
    size_t total = 0;
    auto place = [&](size_t bytes) {
        const size_t at = total;
        total += (bytes + 255) / 256 * 256;
        return at;
    };
    for (size_t s = 0; s < S; ++s) {
        oj[s] = place(jobs[s].size() * sizeof(GJob));
        op[s] = place(prods[s].size() * sizeof(GProd));
        ot[s] = place(tiles[s].size() * sizeof(GTile));
        ofj[s] = place(fjobs[s].size() * sizeof(FJob));
        ofp[s] = place(fprods[s].size() * sizeof(FProd));
        oft[s] = place(ftiles[s].size() * sizeof(GTile));
        ost[s] = place(stiles[s].size() * sizeof(GTile));
    }
    std::vector<unsigned char> host(total);
    auto put = [&](size_t at, const void* src, size_t bytes) {
        if (bytes) std::memcpy(&host[at], src, bytes);
    };
    for (size_t s = 0; s < S; ++s) {
        put(oj[s], jobs[s].data(), jobs[s].size() * sizeof(GJob));
        put(op[s], prods[s].data(), prods[s].size() * sizeof(GProd));
        put(ot[s], tiles[s].data(), tiles[s].size() * sizeof(GTile));
        put(ofj[s], fjobs[s].data(), fjobs[s].size() * sizeof(FJob));
        put(ofp[s], fprods[s].data(), fprods[s].size() * sizeof(FProd));
        put(oft[s], ftiles[s].data(), ftiles[s].size() * sizeof(GTile));
        put(ost[s], stiles[s].data(), stiles[s].size() * sizeof(GTile));
    }
    auto buf = std::make_shared<DBuf>(dev, total);
    dev->upload(buf->p, host.data(), total);   // staged (asynchronous) or synchronous
    const unsigned char* base = buf->as<unsigned char>();
    for (size_t s = 0; s < S; ++s) {
        dj.push_back((const GJob*)(base + oj[s]));
        dp.push_back((const GProd*)(base + op[s]));
        dt.push_back((const GTile*)(base + ot[s]));
        dfj.push_back((const FJob*)(base + ofj[s]));
        dfp.push_back((const FProd*)(base + ofp[s]));
        dft.push_back((const GTile*)(base + oft[s]));
        dts.push_back((const GTile*)(base + ost[s]));
        nts.push_back((int)stiles[s].size());
    }
    hold.push_back(buf);
}

void Plan::set_shape(Dev* dev, int s, int sh) {
    if (shape[s] == sh || sumk[s]) return;
    std::vector<GTile> tiles = make_tiles(jobs[s], prods[s], sh);
    auto bt = std::make_shared<DBuf>(dev, tiles.size() * sizeof(GTile));
    dev->upload(bt->p, tiles.data(), tiles.size() * sizeof(GTile));
    hold.push_back(bt);
    dt[s] = bt->as<GTile>();
    ntiles[s] = (int)tiles.size();
    shape[s] = sh;
}

void Plan::run_stage(Dev* dev, int s, void* ws, void* x, void* y) {
    Bases b;
    b.b[TAG_ABS] = nullptr;
    b.b[TAG_WS] = ws;
    b.b[TAG_X] = x;
    b.b[TAG_Y] = y;
    if (ntiles[s]) launch_stage(s, b, dev->stream);
    launch_fused(s, b, dev->stream);
}

void Plan::launch_fused(size_t s, const Bases& b, hipStream_t st) const {
    if (s >= nftiles.size() || !nftiles[s]) return;
    if (dtype == QED_FP64)
        launch_heff_fused<double>(dfj[s], dfp[s], dft[s], nftiles[s], b, fcs_rows[s], fcs_cols[s], st);
    else
        launch_heff_fused<float>(dfj[s], dfp[s], dft[s], nftiles[s], b, fcs_rows[s], fcs_cols[s], st);
}

void Plan::launch_stage(size_t s, const Bases& b, hipStream_t st) const {
    const GJob* J = dj[s];
    const GProd* Pp = dp[s];
    const GTile* T = dt[s];
    if (sumk[s]) {
        launch_sum_stage(dtype, J, Pp, T, ntiles[s], b, st);
        return;
    }
    const bool fl = pipe[s] == GEMM_PIPE_FLAT && flat_ok[s];
    if (pipe[s] == GEMM_PIPE_SKINNY && skinny_ok[s]) {
        if (dtype == QED_FP64) launch_skinny<double>(J, Pp, dts[s], nts[s], b, st);
        else launch_skinny<float>(J, Pp, dts[s], nts[s], b, st);
        return;
    }
    if (dtype == QED_FP64) {
        if (pipe[s] == GEMM_PIPE_DMA && pipe_valid(s, GEMM_PIPE_DMA, shape[s]))
            launch_brgemm_dma64(J, Pp, T, ntiles[s], b, shape[s], st);
        else
            launch_brgemm<double>(J, Pp, T, ntiles[s], b, shape[s], fl, flat_ok[s] != 0, st);
    } else if (dtype == QED_BF16) launch_brgemm_bf16(J, Pp, T, ntiles[s], b, shape[s], st);
    else if (pipe[s] == GEMM_PIPE_DMA && pipe_valid(s, GEMM_PIPE_DMA, shape[s]))
        launch_brgemm_dma(J, Pp, T, ntiles[s], b, shape[s], st);
    else launch_brgemm<float>(J, Pp, T, ntiles[s], b, shape[s], fl, flat_ok[s] != 0, st);
}

void Prof::record_begin(hipStream_t s, hipEvent_t& a) {
    // harvested events are recorded again instead of being recreated
    if (!pool.empty()) {
        a = pool.back();
        pool.pop_back();
    } else {
        (void)hipEventCreate(&a);
    }
    (void)hipEventRecord(a, s);
}

void Prof::harvest() {
    for (size_t i = 0; i < ev.size(); ++i) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, ev[i].first, ev[i].second) == hipSuccess) ms += t;
        flops += ev_flops[i];
        if (i < ev_key.size() && ev_key[i] % 16 == FUSED_KEY) {
            f_ms += t;
            f_flops += ev_flops[i];
        }
        auto& k = by_key[i < ev_key.size() ? ev_key[i] : -1];
        k[0] += 1.0;
        k[1] += t;
        k[2] += ev_flops[i];
        pool.push_back(ev[i].first);
        pool.push_back(ev[i].second);
    }
    ev.clear();
    ev_flops.clear();
    ev_key.clear();
}

void Prof::report() const {
    static const char* shapes[] = {"64x64", "128x32", "32x128"};
    static const char* pipes[] = {"loop", "flat", "dma", "skinny"};
    for (const auto& kv : by_key) {
        if (kv.first == RUN_KEY) continue;   // whole-run brackets: no per-stage split
        const int st = kv.first / 16, k = kv.first % 16;
        const int sh = k % 4, pp = k / 4;
        const auto& v = kv.second;
        std::fprintf(stderr,
                     "[qedttn] gemm stage %d tile %s %s: %.0f launches, %.3f ms, %.3e flops, %.2f TFLOP/s\n", st,
                     k == FUSED_KEY ? "fused" : (sh < 3 ? shapes[sh] : "?"), k == FUSED_KEY ? "" : pipes[pp % 4],
                     v[0], v[1], v[2], v[1] > 0 ? v[2] / v[1] / 1e9 : 0.0);
    }
}

void Prof::reset() {
    harvest();
    if (std::getenv("QEDTTN_TRACE") && !by_key.empty()) report();
    by_key.clear();
    launches = 0;
    ms = flops = 0.0;
    f_launches = 0;
    f_ms = f_flops = 0.0;
}

Prof::~Prof() {
    for (auto& e : ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

// Profiling: every GEMM and fused launch of the plan counts.  Timing
// events around each launch add their own processing to every interval,
// so by default one event pair brackets the run's GEMM launches, which are
// issued back to back (a summation stage between two GEMM stages would
// fall inside; the matvec plans end with theirs); on the 2x2x2 free-flux
// chi = 64 sweep the bracketed time per launch is within 3% of a rocprofv3
// kernel trace's.  With
// QEDTTN_TRACE set, or for plans with fused stages (whose share is reported
// apart), every launch gets its own pair, for the per-stage breakdown.
void Plan::run(Dev* dev, void* ws, void* x, void* y) {
    Bases b;
    b.b[TAG_ABS] = nullptr;
    b.b[TAG_WS] = ws;
    b.b[TAG_X] = x;
    b.b[TAG_Y] = y;
    const bool on = prof && prof->on;
    static const bool trace = std::getenv("QEDTTN_TRACE") != nullptr;
    bool any_fused = false;
    int last = -1;   // the last stage with a timed launch
    for (size_t s = 0; s < dj.size(); ++s) {
        const bool f = s < nftiles.size() && nftiles[s];
        any_fused = any_fused || f;
        if ((ntiles[s] && !sumk[s]) || f) last = (int)s;
    }
    const bool per_launch = on && (trace || any_fused);
    const bool bracket = on && !per_launch && last >= 0;
    hipEvent_t b0 = nullptr;
    long long nb = 0;
    double fb = 0.0;
    if (bracket) prof->record_begin(dev->stream, b0);
    for (size_t s = 0; s < dj.size(); ++s) {
        if (ntiles[s]) {
            // summation stages run another kernel: only GEMM launches are timed
            const bool timed = per_launch && !sumk[s];
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timed) prof->record_begin(dev->stream, e0);
            launch_stage(s, b, dev->stream);
            if (timed) {
                prof->record_begin(dev->stream, e1);
                prof->ev.push_back({e0, e1});
                prof->ev_flops.push_back(s < stage_flops.size() ? stage_flops[s] : 0.0);
                prof->ev_key.push_back((int)s * 16 + shape[s] + 4 * pipe[s]);
                prof->launches += 1;
            }
            if (bracket && !sumk[s]) {
                nb += 1;
                fb += s < stage_flops.size() ? stage_flops[s] : 0.0;
            }
        }
        if (s < nftiles.size() && nftiles[s]) {
            const bool timed = per_launch;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timed) prof->record_begin(dev->stream, e0);
            launch_fused(s, b, dev->stream);
            if (timed) {
                prof->record_begin(dev->stream, e1);
                prof->ev.push_back({e0, e1});
                prof->ev_flops.push_back(s < fstage_flops.size() ? fstage_flops[s] : 0.0);
                prof->ev_key.push_back((int)s * 16 + Prof::FUSED_KEY);
                prof->launches += 1;
                prof->f_launches += 1;
            }
        }
        if (bracket && (int)s == last) {
            hipEvent_t b1 = nullptr;
            prof->record_begin(dev->stream, b1);
            prof->ev.push_back({b0, b1});
            prof->ev_flops.push_back(fb);
            prof->ev_key.push_back(Prof::RUN_KEY);
            prof->launches += nb;
        }
    }
    dev->check(hipGetLastError(), "brgemm launch");
}

// Output shape of a block's mode product on leg e as a GEMM job, from the
// output extents n: rows and columns of the row-major block (l, r, p) seen
// as (l r) x p, l x (r p), or r x (l p) split per l (e = 2, 0, 1).
static void mode_out_shape(int e, const int n[3], GJob& j) {
    if (e == 2) {
        j.M = n[0] * n[1];
        j.N = n[2];
        j.ldc = n[2];
    } else if (e == 0) {
        j.M = n[0];
        j.N = n[1] * n[2];
        j.ldc = n[1] * n[2];
    } else {
        j.M = n[1];
        j.N = n[0] * n[2];
        j.ldc = n[2];
        j.nsc = n[2];
        j.noc = (int64_t)n[1] * n[2];
    }
}

// Leg order of the staged plan.  By default the bond-leg factor is applied
// first and the terms are summed on l.  QEDTTN_HEFF_ORDER=lrp applies the
// factor on l first and sums the terms on the bond leg (the long products
// then write the per-term intermediates, the short ones reduce): on a
// 267 x 267 x 64 node in FP32 its matvec takes 545 against 505 us, the
// bond-leg reduction over about 30 products of K = 13..37 running at a
// third of the rate of the long stages.
static bool bond_last() {
    const char* v = std::getenv("QEDTTN_HEFF_ORDER");
    return v && !std::strcmp(v, "lrp");
}

static void term_block_flops(const int n[3], const int no[3], bool hA, bool hB, bool hC,
                             double& fA, double& fB, double& fC);

void append_matvec_staged(Plan& P, const Leg legs[3], const BlockTable& tab,
                          const std::vector<HTerm>& terms, int64_t xoff) {
    Builder B(P);
    B.stage(2);
    // legs in the order their factors are applied: the first two write one
    // intermediate per term and block (stages 0, 1); the last sums every
    // term landing on an output block (stage 2)
    const bool bl = bond_last();
    const int ord[3] = {bl ? 0 : 2, 1, bl ? 2 : 0};
    std::map<int64_t, int> bidx;
    for (int b = 0; b < tab.nblk(); ++b) bidx[key3(tab.s[0][b], tab.s[1][b], tab.s[2][b])] = b;
    std::vector<std::vector<GProd>> groups(tab.nblk());
    // terms without a factor on the last leg end in stage 0 (a factor on the
    // first leg only) or in stage 1 (last factor on r): they are summed
    // there, per output block, into one partial that stage 2 adds once
    std::vector<std::vector<GProd>> acc0(tab.nblk()), acc1(tab.nblk());
    for (const HTerm& t : terms) {
        if (t.coef == 0.0) continue;
        for (int b = 0; b < tab.nblk(); ++b) {
            BV cur;
            cur.p = gtag(TAG_X, xoff + tab.off[b]);
            for (int e = 0; e < 3; ++e) {
                cur.s[e] = tab.s[e][b];
                cur.n[e] = legs[e].n[cur.s[e]];
            }
            // output sectors must all exist
            int os[3], no[3];
            bool ok = true;
            for (int e = 0; e < 3; ++e) {
                os[e] = t.op[e] ? t.op[e]->lay.out_of_in[cur.s[e]] : cur.s[e];
                if (os[e] < 0) ok = false;
                else no[e] = legs[e].n[os[e]];
            }
            if (!ok) continue;
            auto it = bidx.find(key3(os[0], os[1], os[2]));
            if (it == bidx.end()) continue;
            const int ob = it->second;
            // algorithmic flops by the definition's order, booked to the
            // stage that applies each factor
            double fl[3];
            term_block_flops(cur.n, no, (bool)t.op[0], (bool)t.op[1], (bool)t.op[2], fl[0], fl[1], fl[2]);
            auto opblk = [&](int e) {
                return gabs((const char*)t.op[e]->data(P.dtype) + t.op[e]->lay.off[cur.s[e]] * B.esize);
            };
            const int f = ord[0], l = ord[2];
            int M, N, ldc, batch;
            int64_t bsC;
            if (t.op[f] && !t.op[1] && !t.op[l]) {
                acc0[ob].push_back(Builder::mode_prod(cur, f, opblk(f), no[f], t.coef, M, N, ldc, batch, bsC));
                B.add_flops(0, fl[f]);
                continue;
            }
            if (t.op[f]) {
                BV nxt;
                B.mode(0, cur, f, *t.op[f], legs[f], nxt, false);
                B.add_flops(0, fl[f]);
                cur = nxt;
            }
            if (t.op[1] && !t.op[l]) {
                acc1[ob].push_back(Builder::mode_prod(cur, 1, opblk(1), no[1], t.coef, M, N, ldc, batch, bsC));
                B.add_flops(1, fl[1]);
                continue;
            }
            if (t.op[1]) {
                BV nxt;
                B.mode(1, cur, 1, *t.op[1], legs[1], nxt, false);
                B.add_flops(1, fl[1]);
                cur = nxt;
            }
            GProd p{};
            if (t.op[l]) {
                p = Builder::mode_prod(cur, l, opblk(l), no[l], t.coef, M, N, ldc, batch, bsC);
                B.add_flops(2, fl[l]);
            } else {
                // no factor at all: c x, read in the output job's shape
                GJob sh{};
                mode_out_shape(l, cur.n, sh);
                p.ident = 1;
                p.B = cur.p;
                p.ldb = sh.ldc;
                p.alpha = t.coef;
                p.nred = 1;
            }
            groups[ob].push_back(p);
        }
    }
    // the partial-sum jobs go first in their stages (their tiles run longest)
    std::vector<GJob> first0, first1;
    for (int b = 0; b < tab.nblk(); ++b) {
        const int n[3] = {legs[0].n[tab.s[0][b]], legs[1].n[tab.s[1][b]], legs[2].n[tab.s[2][b]]};
        const int64_t sz = (int64_t)n[0] * n[1] * n[2];
        GJob out{};
        mode_out_shape(ord[2], n, out);
        for (int st = 0; st < 2; ++st) {
            auto& list = st == 0 ? acc0[b] : acc1[b];
            if (list.empty()) continue;
            B.stage(st);
            GRef part = B.ws(sz);
            GJob j{};
            mode_out_shape(st == 0 ? ord[0] : 1, n, j);
            j.C = part;
            j.batch = 1;
            j.p0 = (int)P.prods[st].size();
            for (auto& p : list) P.prods[st].push_back(p);
            j.p1 = (int)P.prods[st].size();
            (st == 0 ? first0 : first1).push_back(j);
            GProd add{};
            add.ident = 1;
            add.B = part;
            add.ldb = out.ldc;
            add.alpha = 1.0;
            add.nred = 1;
            groups[b].push_back(add);
        }
    }
    if (!first0.empty()) P.jobs[0].insert(P.jobs[0].begin(), first0.begin(), first0.end());
    if (!first1.empty()) P.jobs[1].insert(P.jobs[1].begin(), first1.begin(), first1.end());
    for (int b = 0; b < tab.nblk(); ++b) {
        const int n[3] = {legs[0].n[tab.s[0][b]], legs[1].n[tab.s[1][b]], legs[2].n[tab.s[2][b]]};
        GJob j{};
        mode_out_shape(ord[2], n, j);
        j.C = gtag(TAG_Y, xoff + tab.off[b]);
        j.batch = 1;
        j.p0 = (int)P.prods[2].size();
        for (auto& p : groups[b]) P.prods[2].push_back(p);
        j.p1 = (int)P.prods[2].size();
        j.acc = 0;
        P.jobs[2].push_back(j);
    }
    // algorithmic bytes: x, y and the operator blocks in the GEMM dtype
    const double es = B.esize;
    P.bytes += 2.0 * tab.size() * es;
    for (const HTerm& t : terms)
        for (int e = 0; e < 3; ++e)
            if (t.op[e] && t.coef != 0.0) P.bytes += t.op[e]->lay.size * es;
}

// Algorithmic flops of one term on one block, by the definition's order:
// the factor on p first, then r, then l, each a dense product on the
// extents the previous one produced (n: input extents, no: output).
static void term_block_flops(const int n[3], const int no[3], bool hA, bool hB, bool hC,
                             double& fA, double& fB, double& fC) {
    const double n0 = n[0], n1 = n[1], n2 = n[2];
    fC = hC ? 2.0 * n0 * n1 * n2 * no[2] : 0.0;
    const double c2 = hC ? no[2] : n2;
    fB = hB ? 2.0 * n0 * n1 * no[1] * c2 : 0.0;
    const double b2 = hB ? no[1] : n1;
    fA = hA ? 2.0 * n0 * no[0] * b2 * c2 : 0.0;
}

// The same product as a block-GEMM product (no bond factor): F X on the
// row leg, or alpha X for an identity F.  X of a dense L job is read as
// rows (ldx) by contiguous columns; X of a dense R job as rows (ldx) by
// groups of np_in (stride gox) split like the output.
static GProd as_gprod(const FProd& f, bool split) {
    GProd g{};
    g.alpha = f.alpha;
    g.nred = 1;
    if (f.identF) {
        g.ident = 1;
        g.B = f.X;
        g.ldb = (int)f.ldx;
    } else {
        g.A = f.F;
        g.lda = f.lda;
        g.tA = 0;
        g.B = f.X;
        g.ldb = (int)f.ldx;
        g.tB = 0;
        g.K = f.K;
    }
    if (split) {
        g.nsb = f.np_in;
        g.nob = f.gox;
    }
    return g;
}

bool append_matvec_fused(Plan& P, const Leg legs[3], const BlockTable& tab,
                         const std::vector<HTerm>& terms, int64_t xoff) {
    if (P.dtype != QED_FP32 && P.dtype != QED_FP64) return false;
    const int WCc = P.dtype == QED_FP32 ? FUSED_COLS_F32 : FUSED_COLS_F64;
    // every bond sector must fit one 16-padded group of a tile
    for (int v : legs[2].n)
        if (((v + 15) & ~15) > WCc) return false;
    Builder B(P);
    B.stage(1);
    const int es = B.esize;
    const int nb = tab.nblk();
    std::map<int64_t, int> bidx;
    for (int b = 0; b < nb; ++b) bidx[key3(tab.s[0][b], tab.s[1][b], tab.s[2][b])] = b;
    // per output block: products of the R job (factor on r, none on l; their
    // sum P_R is added in the L job) and of the L job (everything else)
    std::vector<std::vector<FProd>> Rp(nb), Lp(nb);
    std::vector<char> Rc(nb, 0), Lc(nb, 0);
    std::vector<double> rfl(nb, 0.0), lfl(nb, 0.0);
    auto opblk = [&](const OpP& op, int s_in) {
        return gabs((const char*)op->data(P.dtype) + op->lay.off[s_in] * es);
    };
    for (const HTerm& t : terms) {
        if (t.coef == 0.0) continue;
        for (int b = 0; b < nb; ++b) {
            int s[3], n[3], os[3], no[3];
            bool ok = true;
            for (int e = 0; e < 3; ++e) {
                s[e] = tab.s[e][b];
                n[e] = legs[e].n[s[e]];
                os[e] = t.op[e] ? t.op[e]->lay.out_of_in[s[e]] : s[e];
                if (os[e] < 0) ok = false;
                else no[e] = legs[e].n[os[e]];
            }
            if (!ok) continue;
            auto it = bidx.find(key3(os[0], os[1], os[2]));
            if (it == bidx.end()) continue;
            const int ob = it->second;
            const bool hA = (bool)t.op[0], hB = (bool)t.op[1], hC = (bool)t.op[2];
            double fA, fB, fC;
            term_block_flops(n, no, hA, hB, hC, fA, fB, fC);
            const GRef xb = gtag(TAG_X, xoff + tab.off[b]);
            FProd f{};
            f.alpha = t.coef;
            f.hasC = hC ? 1 : 0;
            if (hC) f.Cb = opblk(t.op[2], s[2]);
            f.np_in = n[2];
            if (hB && !hA) {
                // rows r', reduction over r, groups l: P_R(l, r', p') of the block
                f.F = opblk(t.op[1], s[1]);
                f.lda = n[1];
                f.K = n[1];
                f.X = xb;
                f.ldx = n[2];
                f.gox = (int64_t)n[1] * n[2];
                Rp[ob].push_back(f);
                Rc[ob] |= hC ? 1 : 0;
                rfl[ob] += fB + fC;
                continue;
            }
            GRef xin = xb;
            int nr = n[1];
            if (hB) {
                // l and r factors: B x_r x into a workspace block first
                BV cur, nxt;
                cur.p = xb;
                for (int e = 0; e < 3; ++e) {
                    cur.s[e] = s[e];
                    cur.n[e] = n[e];
                }
                B.mode(0, cur, 1, *t.op[1], legs[1], nxt, false);
                B.add_flops(0, fB);
                xin = nxt.p;
                nr = nxt.n[1];
            }
            // rows l', reduction over l, groups r, bond entries p
            if (hA) {
                f.F = opblk(t.op[0], s[0]);
                f.lda = n[0];
            } else {
                f.identF = 1;
            }
            f.K = n[0];
            f.X = xin;
            f.ldx = (int64_t)nr * n[2];
            f.gox = n[2];
            Lp[ob].push_back(f);
            Lc[ob] |= hC ? 1 : 0;
            lfl[ob] += fA + fC;
        }
    }
    auto choose_ng = [&](int np, const std::vector<FProd>& ps, int G) {
        const int p16 = (np + 15) & ~15;
        int maxin = 1;
        for (const FProd& f : ps) maxin = std::max(maxin, f.np_in);
        int ng = std::min(WCc / p16, WCc / maxin);
        return std::max(1, std::min(ng, G));
    };
    auto add_fjob = [&](int st, FJob J, const std::vector<FProd>& ps) {
        J.p0 = (int)P.fprods[st].size();
        for (const FProd& f : ps) P.fprods[st].push_back(f);
        J.p1 = (int)P.fprods[st].size();
        P.fjobs[st].push_back(J);
    };
    for (int ob = 0; ob < nb; ++ob) {
        const int n0 = legs[0].n[tab.s[0][ob]], n1 = legs[1].n[tab.s[1][ob]],
                  n2 = legs[2].n[tab.s[2][ob]];
        if (!Rp[ob].empty()) {
            const GRef pr = B.ws((int64_t)n0 * n1 * n2);
            if (Rc[ob]) {
                FJob J{};
                J.Y = pr;
                J.ldy = n2;
                J.goy = (int64_t)n1 * n2;
                J.M = n1;
                J.G = n0;
                J.np = n2;
                J.ng = choose_ng(n2, Rp[ob], n0);
                add_fjob(0, J, Rp[ob]);
                P.fstage_flops[0] += rfl[ob];
                P.flops += rfl[ob];
            } else {
                GJob J{};
                J.C = pr;
                J.M = n1;
                J.N = n0 * n2;
                J.ldc = n2;
                J.nsc = n2;
                J.noc = (int64_t)n1 * n2;
                J.batch = 1;
                J.p0 = (int)P.prods[0].size();
                for (const FProd& f : Rp[ob]) P.prods[0].push_back(as_gprod(f, true));
                J.p1 = (int)P.prods[0].size();
                P.jobs[0].push_back(J);
                B.add_flops(0, rfl[ob]);
            }
            FProd add{};
            add.identF = 1;
            add.alpha = 1.0;
            add.X = pr;
            add.K = n0;
            add.ldx = (int64_t)n1 * n2;
            add.gox = n2;
            add.np_in = n2;
            Lp[ob].push_back(add);
        }
        const GRef yb = gtag(TAG_Y, xoff + tab.off[ob]);
        if (Lc[ob]) {
            FJob J{};
            J.Y = yb;
            J.ldy = (int64_t)n1 * n2;
            J.goy = n2;
            J.M = n0;
            J.G = n1;
            J.np = n2;
            J.ng = choose_ng(n2, Lp[ob], n1);
            add_fjob(1, J, Lp[ob]);
            P.fstage_flops[1] += lfl[ob];
            P.flops += lfl[ob];
        } else {
            GJob J{};
            J.C = yb;
            J.M = n0;
            J.N = n1 * n2;
            J.ldc = n1 * n2;
            J.batch = 1;
            J.p0 = (int)P.prods[1].size();
            for (const FProd& f : Lp[ob]) P.prods[1].push_back(as_gprod(f, false));
            J.p1 = (int)P.prods[1].size();
            P.jobs[1].push_back(J);
            B.add_flops(1, lfl[ob]);
        }
    }
    // algorithmic bytes: x, y and the operator blocks in the GEMM dtype
    P.bytes += 2.0 * tab.size() * es;
    for (const HTerm& t : terms)
        for (int e = 0; e < 3; ++e)
            if (t.op[e] && t.coef != 0.0) P.bytes += t.op[e]->lay.size * es;
    return true;
}

void append_matvec(Plan& P, const Leg legs[3], const BlockTable& tab,
                   const std::vector<HTerm>& terms, int64_t xoff) {
    if (fused_enabled() && append_matvec_fused(P, legs, tab, terms, xoff)) return;
    append_matvec_staged(P, legs, tab, terms, xoff);
}

// When the fused jobs of the last stage s have fewer than target tiles,
// split every job's products into up to 8 contiguous groups of about equal
// work, each written to a workspace block by a partial job (stage s), and
// add the partial blocks in a new stage s + 1, in a fixed order.
static bool split_fused_for_occupancy(Plan& P, int64_t target) {
    const int s = (int)P.jobs.size() - 1;
    if (s < 0 || (int)P.fjobs.size() <= s || P.fjobs[s].empty()) return false;
    auto tiles_of = [](const FJob& J) {
        return (int64_t)((J.M + FUSED_TM - 1) / FUSED_TM) * ((J.G + J.ng - 1) / J.ng);
    };
    int64_t T = 0;
    for (const FJob& J : P.fjobs[s]) T += tiles_of(J);
    if (T == 0 || T >= target) return false;
    const int S = (int)std::min<int64_t>(8, (target + T - 1) / T);
    if (S < 2) return false;
    Builder B(P);
    B.stage(s + 1);
    std::vector<FJob> old = P.fjobs[s];
    std::vector<FProd> oldp = P.fprods[s];
    P.fjobs[s].clear();
    P.fprods[s].clear();
    auto work = [](const FProd& f) { return (int64_t)(f.identF ? 1 : f.K) + (f.hasC ? f.np_in : 0); };
    for (const FJob& J : old) {
        const int nprod = J.p1 - J.p0;
        const int parts = std::min(S, nprod);
        if (parts < 2) {
            FJob j = J;
            j.p0 = (int)P.fprods[s].size();
            for (int p = J.p0; p < J.p1; ++p) P.fprods[s].push_back(oldp[p]);
            j.p1 = (int)P.fprods[s].size();
            P.fjobs[s].push_back(j);
            continue;
        }
        int64_t W = 0;
        for (int p = J.p0; p < J.p1; ++p) W += work(oldp[p]);
        // the sum job reads Y's block densely: rows of G * np entries
        GJob sum{};
        sum.C = J.Y;
        sum.M = J.M;
        sum.N = J.G * J.np;
        sum.ldc = (int)J.ldy;
        sum.batch = 1;
        sum.acc = J.acc;
        sum.p0 = (int)P.prods[s + 1].size();
        int q = J.p0;
        int64_t done = 0;
        for (int g = 0; g < parts && q < J.p1; ++g) {
            const int64_t goal = W * (g + 1) / parts;
            const GRef part = B.ws((int64_t)J.M * J.G * J.np);
            FJob pj = J;
            pj.Y = part;
            pj.ldy = (int64_t)J.G * J.np;
            pj.goy = J.np;
            pj.acc = 0;
            pj.p0 = (int)P.fprods[s].size();
            do {
                P.fprods[s].push_back(oldp[q]);
                done += work(oldp[q]);
                ++q;
            } while (q < J.p1 && (done < goal || g == parts - 1));
            pj.p1 = (int)P.fprods[s].size();
            P.fjobs[s].push_back(pj);
            GProd add{};
            add.ident = 1;
            add.B = part;
            add.ldb = J.G * J.np;
            add.alpha = 1.0;
            add.nred = 1;
            P.prods[s + 1].push_back(add);
        }
        sum.p1 = (int)P.prods[s + 1].size();
        P.jobs[s + 1].push_back(sum);
    }
    return true;
}

Plan plan_matvec(const Leg legs[3], const BlockTable& tab, const std::vector<HTerm>& terms,
                 int dtype) {
    Plan P;
    P.dtype = dtype;
    append_matvec(P, legs, tab, terms, 0);
    // a single node's last stage has one job per output block, each summing
    // every term: too few tiles to fill the chip, so the term sums are split
    // into partial jobs and added in a final stage
    if (!split_fused_for_occupancy(P, 3072)) split_for_occupancy(P, (int)P.jobs.size() - 1, 2048);
    return P;
}

void append_contract(Plan& P, const Leg legs[3], const BlockTable& tab, GRef in_base,
                     GRef partner_base, int which, const std::vector<RTerm>& terms,
                     const std::vector<ContractOut>& outs, bool split, int base) {
    Builder B(P);
    // mode stages s0, s0+1; contraction s0+2 (new stages, or shared ones)
    const int s0 = base >= 0 ? base : (int)P.jobs.size();
    B.stage(s0 + 2);
    const int es = B.esize;
    int f1 = which == 0 ? 1 : 0;
    int f2 = which == 2 ? 1 : 2;
    std::map<int64_t, int> bidx;
    for (int b = 0; b < tab.nblk(); ++b) bidx[key3(tab.s[0][b], tab.s[1][b], tab.s[2][b])] = b;
    std::map<std::pair<int, int>, std::vector<GProd>> groups;
    auto shift = [&](GRef r, int64_t elems) {
        if (r.tag == TAG_ABS) r.abs = (const char*)r.abs + elems * es;
        else r.off += elems;
        return r;
    };
    for (const RTerm& t : terms) {
        if (t.coef == 0.0) continue;
        for (int b = 0; b < tab.nblk(); ++b) {
            BV cur;
            cur.p = shift(in_base, tab.off[b]);
            for (int e = 0; e < 3; ++e) {
                cur.s[e] = tab.s[e][b];
                cur.n[e] = legs[e].n[cur.s[e]];
            }
            if (t.a) {
                BV nx;
                if (!B.mode(s0, cur, f1, *t.a, legs[f1], nx)) continue;
                cur = nx;
            }
            if (t.b) {
                BV nx;
                if (!B.mode(s0 + 1, cur, f2, *t.b, legs[f2], nx)) continue;
                cur = nx;
            }
            // partner block: same sectors on f1, f2, flux 0
            int ps[3] = {cur.s[0], cur.s[1], cur.s[2]};
            if (which == 2) ps[2] = legs[2].find(legs[0].q[ps[0]] + legs[1].q[ps[1]]);
            else if (which == 0) ps[0] = legs[0].find(legs[2].q[ps[2]] - legs[1].q[ps[1]]);
            else ps[1] = legs[1].find(legs[2].q[ps[2]] - legs[0].q[ps[0]]);
            if (ps[which] < 0) continue;
            auto it = bidx.find(key3(ps[0], ps[1], ps[2]));
            if (it == bidx.end()) continue;
            const int pb = it->second;
            const ContractOut& out = outs[t.out];
            const int sin = cur.s[which], sout = ps[which];
            if (out.lay.out_of_in[sin] != sout)
                fail(QED_ERR_BAD_STATE, "contraction output: charge shift mismatch");
            GRef nb = shift(partner_base, tab.off[pb]);
            const int no = legs[which].n[sout], ni = cur.n[which];
            GProd p{};
            p.alpha = t.coef;
            p.nred = 1;
            if (which == 2) {
                const int K = cur.n[0] * cur.n[1];
                p.A = nb; p.tA = 1; p.lda = no;
                p.B = cur.p; p.tB = 0; p.ldb = ni;
                p.K = K;
                B.add_flops(s0 + 2, 2.0 * K * no * ni);
            } else if (which == 0) {
                const int K = cur.n[1] * cur.n[2];
                p.A = nb; p.tA = 0; p.lda = K;
                p.B = cur.p; p.tB = 1; p.ldb = K;
                p.K = K;
                B.add_flops(s0 + 2, 2.0 * K * no * ni);
            } else {
                const int na = cur.n[0], nc = cur.n[2];
                p.A = nb; p.tA = 0; p.lda = nc; p.rsA = (int64_t)no * nc;
                p.B = cur.p; p.tB = 1; p.ldb = nc; p.rsB = (int64_t)ni * nc;
                p.K = nc;
                p.nred = na;
                B.add_flops(s0 + 2, 2.0 * na * nc * no * ni);
            }
            groups[{t.out, sin}].push_back(p);
        }
    }
    for (int o = 0; o < (int)outs.size(); ++o) {
        const ContractOut& out = outs[o];
        for (int s = 0; s < out.leg.nsec(); ++s) {
            const int so = out.lay.out_of_in[s];
            if (so < 0) continue;
            GJob j{};
            j.C = shift(out.base, out.lay.off[s]);
            j.M = out.leg.n[so];
            j.N = out.leg.n[s];
            j.ldc = j.N;
            j.batch = 1;
            j.p0 = (int)P.prods[s0 + 2].size();
            auto it = groups.find({o, s});
            if (it != groups.end())
                for (auto& p : it->second) P.prods[s0 + 2].push_back(p);
            j.p1 = (int)P.prods[s0 + 2].size();
            P.jobs[s0 + 2].push_back(j);
        }
    }
    if (split) split_long_reductions(P, s0 + 2);
}

Plan plan_renorm(const TensorD& n, int which, const std::vector<RTerm>& terms,
                 const std::vector<OpP>& outs) {
    Plan P;
    P.dtype = QED_FP64;
    std::vector<ContractOut> co;
    // an output with no block (its charge shift maps no sector of the leg
    // onto another) has no storage and receives no job
    for (const OpP& o : outs) co.push_back(ContractOut{o->leg, o->lay, gabs(o->d64 ? o->d64->p : nullptr)});
    append_contract(P, n.legs, n.tab, gabs(n.ptr()), gabs(n.ptr()), which, terms, co, true);
    return P;
}

Plan plan_mode(const TensorD& in, int e, const OpP& op, double* out) {
    Plan P;
    P.dtype = QED_FP64;
    Builder B(P);
    B.stage(0);
    for (int b = 0; b < in.tab.nblk(); ++b) {
        BV cur;
        cur.p = gabs(in.ptr() + in.tab.off[b]);
        for (int k = 0; k < 3; ++k) {
            cur.s[k] = in.tab.s[k][b];
            cur.n[k] = in.legs[k].n[cur.s[k]];
        }
        const int so = op->lay.out_of_in[cur.s[e]];
        if (so != cur.s[e]) fail(QED_ERR_BAD_STATE, "mode product expects a sector-preserving op");
        GRef opblk = gabs(op->f64() + op->lay.off[cur.s[e]]);
        int M, N, ldc, batch;
        int64_t bsC;
        GProd p = Builder::mode_prod(cur, e, opblk, cur.n[e], 1.0, M, N, ldc, batch, bsC);
        B.job1(0, gabs(out + in.tab.off[b]), M, N, ldc, batch, bsC, p);
        P.flops += 2.0 * cur.n[0] * cur.n[1] * cur.n[2] * cur.n[e];
    }
    return P;
}

namespace {

GRef gshift(GRef r, int64_t elems, int esize) {
    if (r.tag == TAG_ABS) r.abs = (const char*)r.abs + elems * esize;
    else r.off += elems;
    return r;
}

}  // namespace

void split_long_reductions(Plan& P, int s) {
    const int64_t KCHUNK = 1024;
    const int MIN_TILES = 16;
    const int esize = dtype_size(P.dtype);
    if ((int)P.jobs.size() <= s) return;
    while ((int)P.jobs.size() <= s + 1) {
        P.jobs.emplace_back();
        P.prods.emplace_back();
        P.stage_flops.push_back(0.0);
    }
    std::vector<GJob> old = P.jobs[s];
    std::vector<GProd> oldp = P.prods[s];
    P.jobs[s].clear();
    P.prods[s].clear();
    for (const GJob& J : old) {
        const int64_t tiles = (int64_t)((J.M + 63) / 64) * ((J.N + 63) / 64) * J.batch;
        int64_t W = 0;
        for (int p = J.p0; p < J.p1; ++p)
            if (!oldp[p].ident) W += (int64_t)oldp[p].K * oldp[p].nred;
        if (J.batch != 1 || tiles >= MIN_TILES || W <= 2 * KCHUNK) {
            GJob j = J;
            j.p0 = (int)P.prods[s].size();
            for (int p = J.p0; p < J.p1; ++p) P.prods[s].push_back(oldp[p]);
            j.p1 = (int)P.prods[s].size();
            P.jobs[s].push_back(j);
            continue;
        }
        std::vector<std::vector<GProd>> chunks(1);
        std::vector<GProd> direct;
        int64_t cur = 0;
        auto push = [&](const GProd& q, int64_t w) {
            if (cur > 0 && cur + w > KCHUNK) {
                chunks.emplace_back();
                cur = 0;
            }
            chunks.back().push_back(q);
            cur += w;
        };
        for (int p = J.p0; p < J.p1; ++p) {
            const GProd& q = oldp[p];
            if (q.ident) {
                direct.push_back(q);
                continue;
            }
            if (q.nred > 1) {
                const int rc = (int)std::max<int64_t>(1, KCHUNK / std::max(1, q.K));
                for (int r0 = 0; r0 < q.nred; r0 += rc) {
                    GProd sub = q;
                    sub.A = gshift(q.A, (int64_t)r0 * q.rsA, esize);
                    sub.B = gshift(q.B, (int64_t)r0 * q.rsB, esize);
                    sub.nred = std::min(rc, q.nred - r0);
                    push(sub, (int64_t)sub.K * sub.nred);
                }
            } else {
                for (int k0 = 0; k0 < q.K; k0 += (int)KCHUNK) {
                    GProd sub = q;
                    const int kl = (int)std::min<int64_t>(KCHUNK, q.K - k0);
                    sub.A = gshift(q.A, q.tA ? (int64_t)k0 * q.lda : k0, esize);
                    sub.B = gshift(q.B, q.tB ? (int64_t)k0 : (int64_t)k0 * q.ldb, esize);
                    sub.K = kl;
                    push(sub, kl);
                }
            }
        }
        GJob sum{};
        sum.C = J.C;
        sum.M = J.M;
        sum.N = J.N;
        sum.ldc = J.ldc;
        sum.batch = 1;
        sum.acc = J.acc;
        sum.p0 = (int)P.prods[s + 1].size();
        for (auto& ch : chunks) {
            if (ch.empty()) continue;
            GRef part = GRef{nullptr, P.ws_elems, TAG_WS, 0};
            P.ws_elems += ((int64_t)J.M * J.N + 63) & ~(int64_t)63;
            GJob pj{};
            pj.C = part;
            pj.M = J.M;
            pj.N = J.N;
            pj.ldc = J.N;
            pj.batch = 1;
            pj.p0 = (int)P.prods[s].size();
            for (auto& q : ch) P.prods[s].push_back(q);
            pj.p1 = (int)P.prods[s].size();
            P.jobs[s].push_back(pj);
            GProd add{};
            add.ident = 1;
            add.B = part;
            add.ldb = J.N;
            add.alpha = 1.0;
            add.nred = 1;
            P.prods[s + 1].push_back(add);
        }
        for (auto& q : direct) P.prods[s + 1].push_back(q);
        sum.p1 = (int)P.prods[s + 1].size();
        P.jobs[s + 1].push_back(sum);
    }
}

void split_for_occupancy(Plan& P, int s, int64_t target_tiles) {
    if ((int)P.jobs.size() != s + 1) return;   // only the last stage of a plan
    auto tiles_of = [](const GJob& J) {
        return (int64_t)((J.M + 63) / 64) * ((J.N + 63) / 64) * J.batch;
    };
    int64_t T = 0;
    for (const GJob& J : P.jobs[s]) T += tiles_of(J);
    if (T == 0 || T >= target_tiles) return;
    const int S = (int)std::min<int64_t>(8, (target_tiles + T - 1) / T);
    if (S < 2) return;
    P.jobs.emplace_back();
    P.prods.emplace_back();
    P.stage_flops.push_back(0.0);
    std::vector<GJob> old = P.jobs[s];
    std::vector<GProd> oldp = P.prods[s];
    P.jobs[s].clear();
    P.prods[s].clear();
    for (const GJob& J : old) {
        std::vector<GProd> work, direct;
        int64_t W = 0;
        for (int p = J.p0; p < J.p1; ++p) {
            if (oldp[p].ident) {
                direct.push_back(oldp[p]);
            } else {
                work.push_back(oldp[p]);
                W += (int64_t)oldp[p].K * oldp[p].nred;
            }
        }
        const int parts = (int)std::min<size_t>((size_t)S, work.size());
        if (J.batch != 1 || parts < 2) {
            GJob j = J;
            j.p0 = (int)P.prods[s].size();
            for (int p = J.p0; p < J.p1; ++p) P.prods[s].push_back(oldp[p]);
            j.p1 = (int)P.prods[s].size();
            P.jobs[s].push_back(j);
            continue;
        }
        // contiguous groups of products with about W / parts work each
        GJob sum{};
        sum.C = J.C;
        sum.M = J.M;
        sum.N = J.N;
        sum.ldc = J.ldc;
        sum.batch = 1;
        sum.acc = J.acc;
        sum.nsc = J.nsc;
        sum.noc = J.noc;
        sum.p0 = (int)P.prods[s + 1].size();
        size_t q = 0;
        int64_t done = 0;
        for (int g = 0; g < parts && q < work.size(); ++g) {
            const int64_t goal = W * (g + 1) / parts;
            GRef part = GRef{nullptr, P.ws_elems, TAG_WS, 0};
            P.ws_elems += ((int64_t)J.M * J.N + 63) & ~(int64_t)63;
            GJob pj{};
            pj.C = part;
            pj.M = J.M;
            pj.N = J.N;
            pj.ldc = J.N;
            pj.batch = 1;
            pj.p0 = (int)P.prods[s].size();
            do {
                P.prods[s].push_back(work[q]);
                done += (int64_t)work[q].K * work[q].nred;
                ++q;
            } while (q < work.size() && (done < goal || g == parts - 1));
            pj.p1 = (int)P.prods[s].size();
            P.jobs[s].push_back(pj);
            GProd add{};
            add.ident = 1;
            add.B = part;
            add.ldb = J.N;
            add.alpha = 1.0;
            add.nred = 1;
            P.prods[s + 1].push_back(add);
        }
        for (auto& d : direct) P.prods[s + 1].push_back(d);
        sum.p1 = (int)P.prods[s + 1].size();
        P.jobs[s + 1].push_back(sum);
    }
}

// Shifted CholeskyQR3 of every task's column-major matrix (Methods,
// "Tensor Networks", step (iii): the isometrisation of a node is a QR per
// sector; the method is that of Fukaya, Kannan, Nakatsukasa, Yamamoto and
// Yanagisawa, SIAM J. Sci. Comput. 42 (2020)).  Pass p: G = A^T A (block
// GEMM, split-K over the long rows), G + s_p I = R_p^T R_p and R_p^-1 (one
// workgroup per sector), A := A R_p^-1 (block GEMM).  The first pass is
// shifted by s_0 = 11 (m n + n (n + 1)) u |A|_F^2, which keeps it positive
// definite for condition numbers up to ~1/u (the downward moves of a sweep
// meet Schmidt spectra that decay to zero); it leaves a condition number of
// at most ~1e8, and two plain passes then give columns orthonormal to
// rounding.  R = R_2 R_1 R_0 has a positive diagonal, so for full-rank
// sectors Q and R equal those of the Householder route.  Returns false,
// with the matrices unchanged, when a sector is wider than CHOL_MAX_COLS or
// a pivot still fails (the caller then takes the Householder route).
bool cholqr_multi(Dev* dev, const std::vector<QRTask>& tasks) {
    if (tasks.empty()) return true;
    int maxn = 0;
    int64_t tot = 0, gtot = 0;
    for (const QRTask& t : tasks) {
        if (t.n > CHOL_MAX_COLS || t.m < t.n) return false;
        maxn = std::max(maxn, t.n);
        tot += t.m * t.n;
        gtot += (int64_t)t.n * t.n;
    }
    const int nt = (int)tasks.size();
    DBuf w1(dev, tot * sizeof(double)), w2(dev, tot * sizeof(double));
    DBuf gram(dev, gtot * sizeof(double));
    DBuf rinv(dev, gtot * sizeof(double));
    DBuf ra(dev, gtot * sizeof(double)), rb(dev, gtot * sizeof(double));
    DBuf status(dev, 3 * nt * sizeof(int));
    std::vector<int64_t> goff(nt), woff(nt);
    {
        int64_t g = 0, w = 0;
        for (int i = 0; i < nt; ++i) {
            goff[i] = g;
            woff[i] = w;
            g += (int64_t)tasks[i].n * tasks[i].n;
            w += tasks[i].m * tasks[i].n;
        }
    }
    auto absref = [](const void* p) { return GRef{p, 0, TAG_ABS, 0}; };
    using In = std::function<const double*(int)>;
    using Out = std::function<double*(int)>;
    // G_i = A_i^T A_i for the matrices at a(i)
    auto gram_pass = [&](const In& a) {
        Plan P;
        P.dtype = QED_FP64;
        P.jobs.emplace_back();
        P.prods.emplace_back();
        P.stage_flops.push_back(0.0);
        for (int i = 0; i < nt; ++i) {
            const QRTask& t = tasks[i];
            GProd q{};
            q.A = absref(a(i));
            q.lda = (int)t.m;
            q.tA = 0;
            q.B = absref(a(i));
            q.ldb = (int)t.m;
            q.tB = 1;
            q.K = (int)t.m;
            q.alpha = 1.0;
            q.nred = 1;
            GJob j{};
            j.C = absref(gram.as<double>() + goff[i]);
            j.M = t.n;
            j.N = t.n;
            j.ldc = t.n;
            j.batch = 1;
            j.p0 = (int)P.prods[0].size();
            P.prods[0].push_back(q);
            j.p1 = j.p0 + 1;
            P.jobs[0].push_back(j);
        }
        split_long_reductions(P, 0);
        P.upload(dev);
        DBuf ws(dev, std::max<int64_t>(1, P.ws_elems) * sizeof(double));
        P.run(dev, ws.p, nullptr, nullptr);
    };
    // out_i = in_i R_i^-1 (column-major m x n, as (R^-T)(A^T) row-major)
    auto apply_pass = [&](const In& in, const Out& out) {
        Plan P;
        P.dtype = QED_FP64;
        P.jobs.emplace_back();
        P.prods.emplace_back();
        P.stage_flops.push_back(0.0);
        for (int i = 0; i < nt; ++i) {
            const QRTask& t = tasks[i];
            GProd q{};
            q.A = absref(rinv.as<double>() + goff[i]);
            q.lda = t.n;
            q.tA = 1;
            q.B = absref(in(i));
            q.ldb = (int)t.m;
            q.tB = 0;
            q.K = t.n;
            q.alpha = 1.0;
            q.nred = 1;
            GJob j{};
            j.C = absref(out(i));
            j.M = t.n;
            j.N = (int)t.m;
            j.ldc = (int)t.m;
            j.batch = 1;
            j.p0 = (int)P.prods[0].size();
            P.prods[0].push_back(q);
            j.p1 = j.p0 + 1;
            P.jobs[0].push_back(j);
        }
        P.upload(dev);
        P.run(dev, nullptr, nullptr, nullptr);
    };
    // Cholesky of pass p; the running R goes ra (pass 0) -> rb (pass 1) ->
    // the caller's R (pass 2)
    auto chol_pass = [&](int pass) {
        std::vector<CholMat> cm(nt);
        for (int i = 0; i < nt; ++i) {
            const QRTask& t = tasks[i];
            CholMat& c = cm[i];
            c.g = gram.as<double>() + goff[i];
            c.rinv = rinv.as<double>() + goff[i];
            c.n = t.n;
            c.status = status.as<int>() + pass * nt + i;
            c.shift = pass == 0 ? 11.0 * ((double)t.m * t.n + (double)t.n * (t.n + 1)) * 0x1p-53 : 0.0;
            c.rprev = pass == 0 ? nullptr : (pass == 1 ? ra : rb).as<double>() + goff[i];
            if (pass < 2) {
                c.rout = (pass == 0 ? ra : rb).as<double>() + goff[i];
                c.rrs = t.n;
                c.rcs = 1;
            } else {
                c.rout = t.R;
                c.rrs = t.rrs;
                c.rcs = t.rcs;
            }
        }
        DBuf d(dev, nt * sizeof(CholMat));
        dev->upload(d.p, cm.data(), nt * sizeof(CholMat));
        launch_chol_inv(d.as<CholMat>(), nt, maxn, dev->stream);
        dev->check(hipGetLastError(), "cholesky launch");
    };
    const In a0 = [&](int i) { return (const double*)tasks[i].M; };
    const In in1 = [&](int i) { return (const double*)(w1.as<double>() + woff[i]); };
    const In in2 = [&](int i) { return (const double*)(w2.as<double>() + woff[i]); };
    gram_pass(a0);
    chol_pass(0);
    apply_pass(a0, [&](int i) { return w1.as<double>() + woff[i]; });
    gram_pass(in1);
    chol_pass(1);
    apply_pass(in1, [&](int i) { return w2.as<double>() + woff[i]; });
    gram_pass(in2);
    chol_pass(2);
    // the caller's matrices are written only once every pivot test passed
    std::vector<int> st(3 * nt);
    dev->download(st.data(), status.p, 3 * nt * sizeof(int));
    for (int v : st)
        if (v) return false;
    apply_pass(in2, [&](int i) { return tasks[i].M; });
    return true;
}

// Rows per chunk of the LDS-resident QR: its time per column step grows
// with the rows, so tall sectors are cut into chunks of at most 256 rows
// (QEDTTN_QR_CHUNK sets another target; never fewer than 3n rows).
static int64_t qr_lds_chunk(int n) {
    static const int64_t target = [] {
        const char* v = std::getenv("QEDTTN_QR_CHUNK");
        const long t = v ? std::atol(v) : 0;
        return (int64_t)(t > 0 ? t : 256);
    }();
    return std::max<int64_t>(target, 3 * (int64_t)n);
}

void tsqr_multi(Dev* dev, const std::vector<QRTask>& tasks) {
    if (tasks.empty()) return;
    // level 1: every direct matrix and every row chunk of every tall one.
    // Matrices of at most QRL_MAXC columns take the LDS-resident kernel;
    // wider ones up to QR_COLS columns the blocked kernel (up to QR_ROWS
    // rows), wider still the unblocked one
    std::vector<QRMat> lds, blocked, wide;
    int64_t rows_b = 0, rows_w = 0;
    int cols_b = 0, cols_w = 0;
    size_t lds_bytes = 0;   // the largest single matrix's need, not max rows x max cols
    std::vector<BufP> keep;
    struct Tall {
        QRTask t;
        std::vector<int64_t> cut;   // first row of every chunk, then m
        BufP S, T;
    };
    std::vector<Tall> tall;
    auto add = [&](const QRMat& q) {
        if (qr_lds_fits(q.rows, q.cols)) {
            lds.push_back(q);
            lds_bytes = std::max(lds_bytes, qr_lds_bytes(q.rows, q.cols));
            return;
        }
        const bool bl = q.rows <= QR_ROWS && q.cols <= QR_COLS;
        (bl ? blocked : wide).push_back(q);
        if (bl) {
            rows_b = std::max<int64_t>(rows_b, q.rows);
            cols_b = std::max(cols_b, q.cols);
        } else {
            rows_w = std::max<int64_t>(rows_w, q.rows);
            cols_w = std::max(cols_w, q.cols);
        }
    };
    for (const QRTask& t : tasks) {
        if (t.m < t.n) fail(QED_ERR_BAD_STATE, "QR of a wide matrix");
        if (t.n > 8192) fail(QED_ERR_UNSUPPORTED, "QR of a sector wider than 8192 columns");
        if (t.n == 0) continue;
        const bool in_lds = t.n <= QRL_MAXC;
        const bool bl = t.n <= QR_COLS;
        const int64_t direct_max = in_lds ? std::min<int64_t>(qr_lds_chunk(t.n), QRL_CAP / t.n - 1)
                                          : (bl ? QR_ROWS : std::max<int64_t>(4096, 16 * (int64_t)t.n));
        if (t.m <= direct_max) {
            auto q = std::make_shared<DBuf>(dev, (size_t)t.m * t.n * sizeof(double));
            keep.push_back(q);
            add(QRMat{t.M, q->as<double>(), t.R, t.m, t.rrs, t.rcs, (int)t.m, t.n});
            continue;
        }
        Tall T;
        T.t = t;
        if (in_lds) {
            // P near-equal chunks of at most direct_max rows (each at least
            // direct_max / 2 >= n rows)
            const int64_t P = (t.m + direct_max - 1) / direct_max;
            for (int64_t i = 0; i <= P; ++i) T.cut.push_back(t.m * i / P);
        } else {
            // chunks of b rows, the last one takes the remainder (< 2b,
            // which is at most QR_ROWS on the blocked path)
            const int64_t b = bl ? std::max<int64_t>(512, 4 * (int64_t)t.n) : std::max<int64_t>(2048, 4 * (int64_t)t.n);
            const int64_t P = t.m / b;
            for (int64_t i = 0; i < P; ++i) T.cut.push_back(i * b);
            T.cut.push_back(t.m);
        }
        const int P = (int)T.cut.size() - 1;
        const int64_t ls = (int64_t)P * t.n;   // rows of the stacked R factors
        T.S = std::make_shared<DBuf>(dev, (size_t)ls * t.n * sizeof(double));
        T.T = std::make_shared<DBuf>(dev, (size_t)t.m * t.n * sizeof(double));
        for (int i = 0; i < P; ++i) {
            const int64_t r0 = T.cut[i];
            add(QRMat{t.M + r0, T.T->as<double>() + r0, T.S->as<double>() + (int64_t)i * t.n, t.m, 1, ls,
                      (int)(T.cut[i + 1] - r0), t.n});
        }
        tall.push_back(T);
    }
    if (!lds.empty()) {
        DBuf dq(dev, lds.size() * sizeof(QRMat));
        dev->upload(dq.p, lds.data(), lds.size() * sizeof(QRMat));
        launch_qr_lds(dq.as<QRMat>(), (int)lds.size(), lds_bytes, dev->stream);
        dev->check(hipGetLastError(), "qr launch");
    }
    for (int kind = 0; kind < 2; ++kind) {
        const auto& list = kind == 0 ? blocked : wide;
        if (list.empty()) continue;
        DBuf dq(dev, list.size() * sizeof(QRMat));
        dev->upload(dq.p, list.data(), list.size() * sizeof(QRMat));
        launch_qr(dq.as<QRMat>(), (int)list.size(), kind == 0 ? rows_b : rows_w,
                  kind == 0 ? cols_b : cols_w, dev->stream);
        dev->check(hipGetLastError(), "qr launch");
    }
    if (tall.empty()) return;
    // the stacked R factors of every tall matrix, one level further up
    std::vector<QRTask> up;
    for (const Tall& T : tall)
        up.push_back(QRTask{T.S->as<double>(), (int64_t)(T.cut.size() - 1) * T.t.n, T.t.n, T.t.R, T.t.rrs,
                            T.t.rcs});
    tsqr_multi(dev, up);
    // Q = blockdiag(Q1_i) * Q2: chunk i of Q is Q1_i Q2[i n .. (i+1) n), all
    // matrices in one GEMM launch
    Plan pl;
    pl.dtype = QED_FP64;
    pl.jobs.emplace_back();
    pl.prods.emplace_back();
    pl.stage_flops.push_back(0.0);
    for (const Tall& T : tall) {
        const int n = T.t.n;
        const int P = (int)T.cut.size() - 1;
        const int64_t m = T.t.m, ls = (int64_t)P * n;
        for (int i = 0; i < P; ++i) {
            const int64_t r0 = T.cut[i];
            const int rows = (int)(T.cut[i + 1] - r0);
            GProd pr{};
            pr.A = GRef{T.S->as<double>() + (int64_t)i * n, 0, TAG_ABS, 0};
            pr.lda = (int)ls;
            pr.B = GRef{T.t.M + r0, 0, TAG_ABS, 0};
            pr.ldb = (int)m;
            pr.K = n;
            pr.alpha = 1.0;
            pr.nred = 1;
            GJob j{};
            j.C = GRef{T.T->as<double>() + r0, 0, TAG_ABS, 0};
            j.M = n;
            j.N = rows;
            j.ldc = (int)m;
            j.batch = 1;
            j.p0 = (int)pl.prods[0].size();
            pl.prods[0].push_back(pr);
            j.p1 = j.p0 + 1;
            pl.jobs[0].push_back(j);
        }
    }
    pl.upload(dev);
    pl.run(dev, nullptr, nullptr, nullptr);
    for (const Tall& T : tall)
        dev->check(hipMemcpyAsync(T.t.M, T.T->p, (size_t)T.t.m * T.t.n * sizeof(double),
                                  hipMemcpyDeviceToDevice, dev->stream), "tsqr copy");
}

void tsqr(Dev* dev, double* M, int64_t m, int n, double* R, int64_t rrs, int64_t rcs) {
    tsqr_multi(dev, {QRTask{M, m, n, R, rrs, rcs}});
}

// ---------------------------------------------------------------------
// Lanczos (Methods, step (ii)), FP64 on the device
// ---------------------------------------------------------------------
void LanczosWS::ensure(Dev* dev, int mm, int64_t nn, bool b32) {
    if (!w || m < mm || n < nn) {
        m = std::max(mm, m);
        n = std::max(nn, n);
        const int G = dot_grid(n);
        w = std::make_shared<DBuf>(dev, n * sizeof(double));
        alpha = std::make_shared<DBuf>(dev, 72 * sizeof(double));
        beta = std::make_shared<DBuf>(dev, 72 * sizeof(double));
        coef = std::make_shared<DBuf>(dev, 144 * sizeof(double));   // two passes of coefficients
        partial = std::make_shared<DBuf>(dev, (size_t)72 * G * sizeof(double));
        sv = std::make_shared<DBuf>(dev, 72 * sizeof(double));
        work = std::make_shared<DBuf>(dev, 256 * sizeof(double));
        st = std::make_shared<DBuf>(dev, sizeof(LState));
        pv = std::make_shared<DBuf>(dev, 512 * sizeof(double));
        pi = std::make_shared<DBuf>(dev, 512 * sizeof(int64_t));
        scal = std::make_shared<DBuf>(dev, 8 * sizeof(double));
        V.reset();
        V32.reset();
    }
    // the basis in the type the run asks for (the other one is not needed)
    if (b32 && !V32) V32 = std::make_shared<DBuf>(dev, (size_t)(m + 1) * n * sizeof(float));
    if (!b32 && !V) V = std::make_shared<DBuf>(dev, (size_t)(m + 1) * n * sizeof(double));
}

LanczosResult lanczos(Dev* dev, LanczosWS& W, const LanczosApply& apply, double* x, int64_t n, int m,
                      int cycles, double tol, float* vc, double exit_tol, bool basis32) {
    if (n <= 0) fail(QED_ERR_INVALID_ARG, "empty eigenproblem");
    m = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(m, 64), n));
    // an FP32 basis needs every pass to fit the fused kernels' 32 rows and no
    // exact first product (the correction's exit copies an FP64 basis row)
    const bool b32 = basis32 && m + 1 <= 32 && exit_tol <= 0.0;
    W.ensure(dev, m, n, b32);
    hipStream_t s = dev->stream;
    double* w = W.w->as<double>();
    double* al = W.alpha->as<double>();
    double* be = W.beta->as<double>();
    double* co = W.coef->as<double>();
    double* co2 = co + 72;
    double* part = W.partial->as<double>();
    double* sc = W.scal->as<double>();
    LState* st = W.st->as<LState>();
    LanczosResult R;
    const int64_t ld = n;
    auto run = [&](auto* V) {
        using TV = typename std::remove_pointer<decltype(V)>::type;
        constexpr bool F64 = std::is_same<TV, double>::value;
        for (int cyc = 0; cyc < std::max(1, cycles); ++cyc) {
            launch_dots(x, n, 1, x, n, part, sc + 0, 1, nullptr, 0, s);
            launch_lz_start<TV>(V, x, sc + 0, n, st, m, s);
            for (int j = 0; j < m; ++j) {
                TV* vj = V + (int64_t)j * ld;
                bool fused_alpha;
                if constexpr (F64) fused_alpha = apply(vj, vc && j > 0 ? vc : nullptr, w, part);
                else fused_alpha = apply(nullptr, vj, w, part);
                if (fused_alpha) {
                    launch_dot_final(part, n, 1, al + j, 0, st, 1, s);
                } else {
                    if constexpr (F64) launch_dots(vj, ld, 1, w, n, part, al + j, 0, st, 1, s);
                    else fail(QED_ERR_BAD_STATE, "an FP32 Lanczos basis needs the fused alpha dot");
                }
                ++R.matvecs;
                // three-term recurrence, classical Gram-Schmidt against V, a
                // second pass where the first removed more than half of |w|^2
                // (decided on the device), norm: fused so that each pass reads
                // the basis once
                if (launch_lz_fused<TV>(0, w, V, ld, 0, j, al, be, nullptr, nullptr, n, part, co, st, s)) {
                    launch_lz_fused<TV>(1, w, V, ld, j + 1, j, al, be, co, co, n, part, co2, st, s);
                    launch_lz_norm_beta<TV>(w, V, ld, j + 1, j, al, be, co2, co, n, part, sc + 1, st, 1e-14, s);
                } else {
                    if constexpr (F64) {
                        launch_lz_three_term(w, V, ld, j, al, be, n, st, s);
                        for (int pass = 0; pass < 2; ++pass) {
                            launch_dots(V, ld, j + 1, w, n, part, co, 0, st, 1, s);
                            launch_lz_subtract(w, V, ld, j + 1, co, n, st, s);
                        }
                        launch_dots(w, n, 1, w, n, part, sc + 1, 0, st, 1, s);
                        launch_lz_beta(sc + 1, al, be, j, st, 1e-14, s);
                    } else {
                        fail(QED_ERR_BAD_STATE, "an FP32 Lanczos basis is limited to 31 steps");
                    }
                }
                if (j == 0 && exit_tol > 0.0) {
                    if constexpr (F64) {
                        // the exact residual of the current vector decides
                        double ab[2];
                        dev->download(&ab[0], al, sizeof(double));
                        dev->download(&ab[1], be, sizeof(double));
                        if (!std::isfinite(ab[0]) || !std::isfinite(ab[1]))
                            fail(QED_ERR_NONFINITE, "Lanczos produced a non-finite value");
                        if (ab[1] <= exit_tol * std::max(std::fabs(ab[0]), 1e-300)) {
                            dev->check(hipMemcpyAsync(x, V, n * sizeof(double), hipMemcpyDeviceToDevice, s),
                                       "copy");
                            R.theta = ab[0];
                            R.resid = ab[1];
                            R.cycles = cyc + 1;
                            R.exact = true;
                            return true;
                        }
                    }
                }
                launch_lz_next<TV>(V, ld, j, w, be, n, st, s, F64 ? vc : nullptr);
            }
            launch_tridiag(al, be, W.sv->as<double>(), st, W.work->as<double>(), s);
            launch_ritz<TV>(x, V, ld, W.sv->as<double>(), n, st, s);
            launch_dots(x, n, 1, x, n, part, sc + 2, 1, nullptr, 0, s);
            launch_normalise_sign(x, n, sc + 2, W.pv->as<double>(), W.pi->as<int64_t>(), sc + 3, s);
            dev->check(hipGetLastError(), "lanczos launch");
            LState hs;
            dev->download(&hs, st, sizeof(LState));
            R.theta = hs.theta;
            R.resid = hs.resid;
            R.cycles = cyc + 1;
            if (!std::isfinite(hs.theta) || !std::isfinite(hs.norm) || hs.norm == 0.0)
                fail(QED_ERR_NONFINITE, "Lanczos produced a non-finite value (zero or invalid start vector?)");
            if (exit_tol <= 0.0 && hs.resid <= tol * std::max(std::fabs(hs.theta), 1e-300)) break;
        }
        return false;
    };
    if (b32) run(W.V32->as<float>());
    else run(W.V->as<double>());
    return R;
}

// ---------------------------------------------------------------------
// node-level H_eff
// ---------------------------------------------------------------------
void Heff::matvec(const double* x, double* y) {
    Dev* dev = &ctx->dev;
    plan.prof = &ctx->prof;
    void* w = ws.get(dev, std::max<int64_t>(1, plan.ws_elems) * dtype_size(plan.dtype));
    run_matvec(x, y, w);
}

void Heff::matvec_ws(const double* x, double* y, void* w) {
    plan.prof = nullptr;   // no timing events: nothing is created
    run_matvec(x, y, w);
}

void Heff::run_matvec(const double* x, double* y, void* w) {
    Dev* dev = &ctx->dev;
    ctx->mv_flops += plan.flops;
    ctx->mv_count += 1;
    const int64_t n = tab.size();
    if (plan.dtype == QED_FP64) {
        plan.run(dev, w, (void*)x, (void*)y);
    } else {
        to_compute(plan.dtype, x, xc->p, n, dev->stream);
        plan.run(dev, w, xc->p, yc->p);
        from_compute(plan.dtype, yc->p, y, n, dev->stream);
    }
}

}  // namespace qed
