// extern "C" boundary of libqedttn (declarations and contracts in
// include/qedttn.h).  Every entry point turns internal errors into status
// codes and a context-owned message.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "engine.h"

using namespace qed;

struct qed_ctx {
    Ctx c;
};

struct qed_heff {
    Heff h;
    qed_ctx* owner = nullptr;
};

struct qed_heff_batch {
    HeffBatch b;
    qed_ctx* owner = nullptr;
};

namespace {

template <typename F>
int guard(qed_ctx* ctx, F&& f) {
    if (!ctx) return QED_ERR_INVALID_ARG;
    try {
        ctx->c.err.clear();
        return f();
    } catch (const Error& e) {
        ctx->c.err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        ctx->c.err = "host out of memory";
        return QED_ERR_OOM;
    } catch (const std::exception& e) {
        ctx->c.err = e.what();
        return QED_ERR_INVALID_ARG;
    }
}

Ctx& C(qed_ctx* c) { return c->c; }

void need_device(Ctx& c) {
    if (c.host_only) fail(QED_ERR_BAD_STATE, "host-only context: no GPU work possible");
}

void need_built(Ctx& c) {
    if (!c.built || !c.eng) fail(QED_ERR_BAD_STATE, "call qed_build_hamiltonian first");
}

Leg make_leg(const int* ch, const int* n, int s) {
    if (s <= 0 || !ch || !n) fail(QED_ERR_INVALID_ARG, "a leg needs at least one sector");
    Leg L;
    for (int i = 0; i < s; ++i) {
        if (n[i] <= 0) fail(QED_ERR_INVALID_ARG, "sector sizes must be positive");
        if (i && ch[i] <= ch[i - 1]) fail(QED_ERR_INVALID_ARG, "charges must be strictly ascending");
        L.q.push_back(ch[i]);
        L.n.push_back(n[i]);
    }
    return L;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

// ---- scratch of the allocation-free matvec -----------------------------
// Device memory with static storage: every GPU the library runs on holds
// its own copy (at its own address) from module load until the process
// ends.  Host code never passes `scratch` itself to a kernel (on the host
// the name is a stand-in, not a device address): the address of each
// device's copy is looked up once per device, with that device current,
// when a context is created on it.
namespace {

constexpr size_t SCRATCH_BYTES = QED_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex scratch_mu;
std::vector<void*> scratch_ptr;     // per device: address of its copy, or null
std::vector<int> scratch_rc;        // per device: 0 = not looked up, 1 = ok, < 0 = failed

// with `device` current
void scratch_lookup(int device) {
    std::lock_guard<std::mutex> g(scratch_mu);
    if ((int)scratch_ptr.size() <= device) {
        scratch_ptr.resize(device + 1, nullptr);
        scratch_rc.resize(device + 1, 0);
    }
    if (scratch_rc[device] == 1) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && p) {
        scratch_ptr[device] = p;
        scratch_rc[device] = 1;
    } else {
        (void)hipGetLastError();
        scratch_rc[device] = -1;
    }
}

void* scratch_for(int device) {
    std::lock_guard<std::mutex> g(scratch_mu);
    if (device < 0 || device >= (int)scratch_ptr.size() || scratch_rc[device] != 1) return nullptr;
    return scratch_ptr[device];
}

}  // namespace

// ---- checkpoint / resume -------------------------------------------------
namespace {

constexpr char CKPT_MAGIC[8] = {'Q', 'E', 'D', 'T', 'T', 'N', 'S', '\0'};
constexpr uint32_t CKPT_VERSION = 1;

struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(const void* p, size_t n) {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    }
};

struct Writer {
    std::FILE* f;
    Fnv sum;
    void put(const void* p, size_t n) {
        if (std::fwrite(p, 1, n, f) != n) fail(QED_ERR_IO, "checkpoint write failed");
        sum.add(p, n);
    }
    template <typename T> void val(T v) { put(&v, sizeof(T)); }
};

struct Reader {
    std::FILE* f;
    Fnv sum;
    int64_t left = 0;   // bytes not read yet
    void get(void* p, size_t n) {
        if ((int64_t)n > left || std::fread(p, 1, n, f) != n) fail(QED_ERR_IO, "checkpoint truncated");
        left -= (int64_t)n;
        sum.add(p, n);
    }
    template <typename T> T val() {
        T v;
        get(&v, sizeof(T));
        return v;
    }
};

struct FileCloser {
    std::FILE* f;
    ~FileCloser() {
        if (f) std::fclose(f);
    }
};

}  // namespace

extern "C" {

int qed_create(qed_ctx** out, int hip_device) {
    if (!out) return QED_ERR_INVALID_ARG;
    *out = nullptr;
    qed_ctx* ctx = new (std::nothrow) qed_ctx();
    if (!ctx) return QED_ERR_OOM;
    if (hip_device >= 0) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || hip_device >= count) {
            delete ctx;
            return QED_ERR_HIP;
        }
        if (hipSetDevice(hip_device) != hipSuccess) {
            delete ctx;
            return QED_ERR_HIP;
        }
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, hip_device) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        ctx->c.dev.device = hip_device;
        ctx->c.host_only = false;
        scratch_lookup(hip_device);
    }
    *out = ctx;
    return QED_OK;
}

int qed_destroy(qed_ctx* ctx) {
    if (!ctx) return QED_ERR_INVALID_ARG;
    try {
        if (!ctx->c.host_only) {
            (void)hipSetDevice(ctx->c.dev.device);
            (void)hipStreamSynchronize(ctx->c.dev.stream);
        }
        ctx->c.eng.reset();
        if (!ctx->c.host_only) {
            (void)hipStreamSynchronize(ctx->c.dev.stream);
            ctx->c.dev.trim();
            (void)hipStreamSynchronize(ctx->c.dev.stream);
        }
    } catch (...) {
    }
    delete ctx;
    return QED_OK;
}

const char* qed_last_error(const qed_ctx* ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

int qed_set_allocator(qed_ctx* ctx, void* (*alloc)(uint64_t, void*, void*),
                      void (*free_fn)(void*, void*, void*), void* user) {
    return guard(ctx, [&] {
        if ((alloc == nullptr) != (free_fn == nullptr))
            fail(QED_ERR_INVALID_ARG, "alloc and free must both be set or both be NULL");
        if (C(ctx).dev.used) fail(QED_ERR_BAD_STATE, "the allocator must be set before any allocation");
        C(ctx).dev.ualloc = alloc;
        C(ctx).dev.ufree = free_fn;
        C(ctx).dev.user = user;
        return QED_OK;
    });
}

int qed_set_stream(qed_ctx* ctx, void* stream) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        C(ctx).dev.sync();
        C(ctx).dev.stream = (hipStream_t)stream;
        C(ctx).dev.restream((hipStream_t)stream);
        return QED_OK;
    });
}

int qed_set_lattice(qed_ctx* ctx, int Lx, int Ly, int Lz, int bc) {
    return guard(ctx, [&] {
        if (bc != QED_BC_OPEN_ZERO_FLUX && bc != QED_BC_OPEN_FREE_FLUX && bc != QED_BC_PERIODIC)
            fail(QED_ERR_INVALID_ARG, "unknown boundary condition");
        if (!pow2(Lx) || !pow2(Ly) || !pow2(Lz))
            fail(QED_ERR_INVALID_ARG, "lattice extents must be powers of two");
        if ((int64_t)Lx * Ly * Lz < 2 || (int64_t)Lx * Ly * Lz > 4096)
            fail(QED_ERR_INVALID_ARG, "the lattice needs 2 .. 4096 sites");
        Params& P = C(ctx).prm;
        P.Lx = Lx;
        P.Ly = Ly;
        P.Lz = Lz;
        P.bc = bc;
        P.have_lattice = true;
        P.mu.clear();   // one potential per site: reset with the lattice
        C(ctx).built = false;
        return QED_OK;
    });
}

int qed_set_chemical_potential(qed_ctx* ctx, const double* mu) {
    return guard(ctx, [&] {
        Params& P = C(ctx).prm;
        if (!P.have_lattice) fail(QED_ERR_BAD_STATE, "call qed_set_lattice first");
        const int n = P.Lx * P.Ly * P.Lz;
        std::vector<double> v;
        if (mu) {
            v.assign(mu, mu + n);
            for (double x : v)
                if (!std::isfinite(x)) fail(QED_ERR_INVALID_ARG, "chemical potentials must be finite");
        }
        P.mu = v;
        C(ctx).built = false;
        return QED_OK;
    });
}

int qed_set_couplings(qed_ctx* ctx, double t, double m, double g2_e, double g2_m) {
    return guard(ctx, [&] {
        if (!std::isfinite(t) || !std::isfinite(m) || !std::isfinite(g2_e) || !std::isfinite(g2_m))
            fail(QED_ERR_INVALID_ARG, "couplings must be finite");
        Params& P = C(ctx).prm;
        P.t = t;
        P.m = m;
        P.g2e = g2_e;
        P.g2m = g2_m;
        P.have_couplings = true;
        C(ctx).built = false;
        return QED_OK;
    });
}

int qed_physical_line(double g2, double t, double* g2_e, double* g2_m) {
    if (!g2_e || !g2_m || !(g2 > 0.0) || !std::isfinite(t)) return QED_ERR_INVALID_ARG;
    *g2_e = g2 * t;
    *g2_m = 8.0 * t / g2;
    return QED_OK;
}

int qed_set_penalty(qed_ctx* ctx, double nu_max, int n_linear, int n_quadratic, int adaptive) {
    return guard(ctx, [&] {
        if (!(nu_max >= 0.0) || n_linear < 0 || n_quadratic < 0)
            fail(QED_ERR_INVALID_ARG, "invalid penalty schedule");
        Params& P = C(ctx).prm;
        P.nu_max = nu_max;
        P.n_lin = n_linear;
        P.n_quad = n_quadratic;
        P.pen_adaptive = adaptive ? 1 : 0;
        return QED_OK;
    });
}

int qed_set_charge_sector(qed_ctx* ctx, int Q) {
    return guard(ctx, [&] {
        C(ctx).prm.Q = Q;
        C(ctx).built = false;
        return QED_OK;
    });
}

int qed_set_bond_dim(qed_ctx* ctx, int chi) {
    return guard(ctx, [&] {
        if (chi < 1 || chi > 65536) fail(QED_ERR_INVALID_ARG, "chi out of range");
        C(ctx).prm.chi = chi;
        C(ctx).built = false;
        return QED_OK;
    });
}

int qed_set_lanczos(qed_ctx* ctx, int steps, int max_cycles, double tol) {
    return guard(ctx, [&] {
        if (steps < 1 || steps > 64 || max_cycles < 1 || !(tol >= 0.0))
            fail(QED_ERR_INVALID_ARG, "Lanczos: 1 <= steps <= 64, cycles >= 1, tol >= 0");
        Params& P = C(ctx).prm;
        P.lz_steps = steps;
        P.lz_cycles = max_cycles;
        P.lz_tol = tol;
        return QED_OK;
    });
}

int qed_set_expansion(qed_ctx* ctx, int on, double alpha, int delta, int chi_max, uint64_t seed) {
    return guard(ctx, [&] {
        if (!std::isfinite(alpha) || alpha < 0.0 || delta < 0 || chi_max < 0)
            fail(QED_ERR_INVALID_ARG, "expansion: alpha >= 0, delta >= 0, chi_max >= 0");
        Params& P = C(ctx).prm;
        P.exp_on = on != 0;
        P.exp_alpha = alpha;
        P.exp_delta = delta;
        P.exp_chimax = chi_max;
        P.exp_seed = seed;
        return QED_OK;
    });
}

int qed_set_lanczos_schedule(qed_ctx* ctx, double tol0, double factor) {
    return guard(ctx, [&] {
        if (!(tol0 >= 0.0) || !(factor > 0.0 && factor < 1.0))
            fail(QED_ERR_INVALID_ARG, "Lanczos schedule: tol0 >= 0 and 0 < factor < 1");
        Params& P = C(ctx).prm;
        P.lz_tol0 = tol0;
        P.lz_factor = factor;
        return QED_OK;
    });
}

int qed_set_precision(qed_ctx* ctx, int gemm_dtype, int refine) {
    return guard(ctx, [&] {
        if (gemm_dtype != QED_FP64 && gemm_dtype != QED_FP32 && gemm_dtype != QED_BF16)
            fail(QED_ERR_INVALID_ARG, "unknown GEMM dtype");
        if (refine < 0) fail(QED_ERR_INVALID_ARG, "refine must be >= 0");
        C(ctx).prm.dtype = gemm_dtype;
        C(ctx).prm.refine = std::min(refine, 2);
        return QED_OK;
    });
}

int qed_build_hamiltonian(qed_ctx* ctx) {
    return guard(ctx, [&] {
        Ctx& c = C(ctx);
        if (!c.prm.have_lattice || !c.prm.have_couplings)
            fail(QED_ERR_BAD_STATE, "set the lattice and the couplings first");
        if (!c.host_only) (void)hipSetDevice(c.dev.device);
        auto e = std::make_unique<Engine>();
        e->build(&c);
        if (c.eng && !c.host_only) c.dev.sync();
        c.eng = std::move(e);
        c.built = true;
        return QED_OK;
    });
}

int qed_get_local_dims(qed_ctx* ctx, int* dims) {
    return guard(ctx, [&] {
        need_built(C(ctx));
        if (!dims) fail(QED_ERR_INVALID_ARG, "dims is NULL");
        const auto& m = C(ctx).eng->model;
        for (int s = 0; s < m.lat.N; ++s) dims[s] = m.sites[s].d();
        return QED_OK;
    });
}

int qed_get_tree(qed_ctx* ctx, int* n_nodes, int* n_sites) {
    return guard(ctx, [&] {
        need_built(C(ctx));
        if (n_nodes) *n_nodes = (int)C(ctx).eng->tree.nodes.size();
        if (n_sites) *n_sites = C(ctx).eng->tree.N;
        return QED_OK;
    });
}

int qed_get_node_links(qed_ctx* ctx, int node, int links[3]) {
    return guard(ctx, [&] {
        need_built(C(ctx));
        const Tree& t = C(ctx).eng->tree;
        if (node < 0 || node >= (int)t.nodes.size() || !links) fail(QED_ERR_INVALID_ARG, "bad node");
        links[0] = t.nodes[node].l;
        links[1] = t.nodes[node].r;
        links[2] = t.nodes[node].p;
        return QED_OK;
    });
}

int qed_get_leg_sectors(qed_ctx* ctx, int link, int* charges, int* sizes, int cap, int* nsec) {
    return guard(ctx, [&] {
        need_built(C(ctx));
        const Engine& e = *C(ctx).eng;
        if (link < 0 || link >= e.tree.nlinks()) fail(QED_ERR_INVALID_ARG, "bad link");
        const Leg& L = e.legs[link];
        if (nsec) *nsec = L.nsec();
        for (int i = 0; i < L.nsec() && i < cap; ++i) {
            if (charges) charges[i] = L.q[i];
            if (sizes) sizes[i] = L.n[i];
        }
        return QED_OK;
    });
}

int qed_init_state(qed_ctx* ctx, uint64_t seed) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        need_built(C(ctx));
        C(ctx).eng->init_nodes(seed);
        return QED_OK;
    });
}

int qed_node_size(qed_ctx* ctx, int node, int64_t* n_entries) {
    return guard(ctx, [&] {
        need_built(C(ctx));
        const Engine& e = *C(ctx).eng;
        if (node < 0 || node >= (int)e.tree.nodes.size() || !n_entries) fail(QED_ERR_INVALID_ARG, "bad node");
        const auto& nd = e.tree.nodes[node];
        *n_entries = make_table(e.legs[nd.l], e.legs[nd.r], e.legs[nd.p], 0).size();
        return QED_OK;
    });
}

int qed_set_node(qed_ctx* ctx, int node, const double* host, int64_t n) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        need_built(C(ctx));
        Engine& e = *C(ctx).eng;
        if (node < 0 || node >= (int)e.tree.nodes.size() || !host) fail(QED_ERR_INVALID_ARG, "bad node");
        if (e.nodes.empty()) e.init_nodes(0);
        TensorD& T = e.nodes[node];
        if (n != T.tab.size()) fail(QED_ERR_INVALID_ARG, "wrong number of entries");
        C(ctx).dev.upload(T.d->p, host, n * sizeof(double));
        e.invalidate();
        return QED_OK;
    });
}

int qed_get_node(qed_ctx* ctx, int node, double* host, int64_t n) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        need_built(C(ctx));
        Engine& e = *C(ctx).eng;
        if (node < 0 || node >= (int)e.nodes.size() || !host) fail(QED_ERR_INVALID_ARG, "bad node");
        TensorD& T = e.nodes[node];
        if (n != T.tab.size()) fail(QED_ERR_INVALID_ARG, "wrong number of entries");
        C(ctx).dev.download(host, T.d->p, n * sizeof(double));
        return QED_OK;
    });
}


int qed_save_state(qed_ctx* ctx, const char* path) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        need_built(C(ctx));
        if (!path || !*path) fail(QED_ERR_INVALID_ARG, "empty path");
        Engine& e = *C(ctx).eng;
        if (e.nodes.empty()) fail(QED_ERR_BAD_STATE, "no state to save");
        const Params& P = C(ctx).prm;
        const std::string tmp = std::string(path) + ".tmp";
        {
            FileCloser fc{std::fopen(tmp.c_str(), "wb")};
            if (!fc.f) fail(QED_ERR_IO, "cannot open checkpoint file for writing");
            Writer w{fc.f, {}};
            w.put(CKPT_MAGIC, sizeof(CKPT_MAGIC));
            w.val<uint32_t>(CKPT_VERSION);
            for (int v : {P.Lx, P.Ly, P.Lz, P.bc, P.Q, P.chi}) w.val<int32_t>(v);
            for (double v : {P.t, P.m, P.g2e, P.g2m}) w.val<double>(v);
            w.val<int32_t>(e.sweeps_done);
            w.val<int32_t>(e.centre == e.tree.root ? 1 : 0);
            w.val<int32_t>(e.have_energy ? 1 : 0);
            w.val<double>(e.energy);
            w.val<int32_t>((int)e.legs.size());
            for (const Leg& L : e.legs) {
                w.val<int32_t>(L.nsec());
                for (int s = 0; s < L.nsec(); ++s) {
                    w.val<int32_t>(L.q[s]);
                    w.val<int32_t>(L.n[s]);
                }
            }
            w.val<int32_t>((int)e.nodes.size());
            std::vector<double> h;
            for (const TensorD& T : e.nodes) {
                h.resize(T.tab.size());
                C(ctx).dev.download(h.data(), T.ptr(), h.size() * sizeof(double));
                w.val<int64_t>((int64_t)h.size());
                w.put(h.data(), h.size() * sizeof(double));
            }
            const uint64_t s = w.sum.h;
            if (std::fwrite(&s, 1, sizeof(s), fc.f) != sizeof(s)) fail(QED_ERR_IO, "checkpoint write failed");
            if (std::fflush(fc.f) != 0) fail(QED_ERR_IO, "checkpoint flush failed");
        }
        if (std::rename(tmp.c_str(), path) != 0) fail(QED_ERR_IO, "cannot move the checkpoint into place");
        return QED_OK;
    });
}

int qed_load_state(qed_ctx* ctx, const char* path) {
    return guard(ctx, [&] {
        if (!path || !*path) fail(QED_ERR_INVALID_ARG, "empty path");
        FileCloser fc{std::fopen(path, "rb")};
        if (!fc.f) fail(QED_ERR_IO, "cannot open checkpoint file");
        Reader r{fc.f, {}, 0};
        if (std::fseek(fc.f, 0, SEEK_END) != 0) fail(QED_ERR_IO, "cannot size the checkpoint file");
        r.left = (int64_t)std::ftell(fc.f);
        if (r.left < 0 || std::fseek(fc.f, 0, SEEK_SET) != 0) fail(QED_ERR_IO, "cannot size the checkpoint file");
        char magic[8];
        r.get(magic, sizeof(magic));
        if (std::memcmp(magic, CKPT_MAGIC, sizeof(magic)) != 0) fail(QED_ERR_IO, "not a checkpoint file");
        if (r.val<uint32_t>() != CKPT_VERSION) fail(QED_ERR_IO, "unsupported checkpoint version");
        int32_t hdr[6];
        for (int& v : hdr) v = r.val<int32_t>();
        double cpl[4];
        for (double& v : cpl) v = r.val<double>();
        const int32_t sweeps = r.val<int32_t>();
        const int32_t iso = r.val<int32_t>();
        const int32_t have_e = r.val<int32_t>();
        const double energy = r.val<double>();
        const int32_t nlegs = r.val<int32_t>();
        if (nlegs < 1 || nlegs > (1 << 20)) fail(QED_ERR_IO, "corrupt checkpoint (legs)");
        std::vector<Leg> legs(nlegs);
        for (Leg& L : legs) {
            const int32_t ns = r.val<int32_t>();
            if (ns < 1 || ns > 4096) fail(QED_ERR_IO, "corrupt checkpoint (sectors)");
            for (int s = 0; s < ns; ++s) {
                L.q.push_back(r.val<int32_t>());
                L.n.push_back(r.val<int32_t>());
            }
        }
        const int32_t nn = r.val<int32_t>();
        if (nn < 1 || nn > (1 << 20)) fail(QED_ERR_IO, "corrupt checkpoint (nodes)");
        std::vector<std::vector<double>> data(nn);
        for (auto& d : data) {
            const int64_t sz = r.val<int64_t>();
            if (sz < 0 || sz > r.left / (int64_t)sizeof(double)) fail(QED_ERR_IO, "corrupt checkpoint (node size)");
            d.resize(sz);
            r.get(d.data(), sz * sizeof(double));
        }
        uint64_t stored = 0;
        const uint64_t computed = r.sum.h;
        if (std::fread(&stored, 1, sizeof(stored), fc.f) != sizeof(stored) || stored != computed)
            fail(QED_ERR_IO, "checkpoint checksum mismatch");
        // the file is whole; now it has to fit the configured problem
        need_device(C(ctx));
        need_built(C(ctx));
        Engine& e = *C(ctx).eng;
        const Params& P = C(ctx).prm;
        const int cur[6] = {P.Lx, P.Ly, P.Lz, P.bc, P.Q, P.chi};
        for (int i = 0; i < 6; ++i)
            if (hdr[i] != cur[i])
                fail(QED_ERR_INVALID_ARG, "checkpoint is for another lattice, boundary, charge or bond dimension");
        if (nlegs != (int)e.legs.size() || nn != (int)e.tree.nodes.size())
            fail(QED_ERR_INVALID_ARG, "checkpoint tree does not match");
        // site legs and the root's charge leg are fixed by the model; the
        // internal legs may differ from the allocation rule (subspace
        // expansion changes them), but every sector must fit its rows
        bool same = true;
        for (int i = 0; i < nlegs; ++i) {
            const bool fixed = i < e.tree.N || i == e.tree.top;
            const bool eq = legs[i].q == e.alloc_legs[i].q && legs[i].n == e.alloc_legs[i].n;
            if (fixed && !eq) fail(QED_ERR_INVALID_ARG, "checkpoint leg sectors do not match");
            for (int s = 0; s < legs[i].nsec(); ++s)
                if (legs[i].n[s] < 1 || (s && legs[i].q[s] <= legs[i].q[s - 1]))
                    fail(QED_ERR_IO, "corrupt checkpoint (leg sectors)");
            if (!(legs[i].q == e.legs[i].q && legs[i].n == e.legs[i].n)) same = false;
        }
        if (e.nodes.empty()) e.init_nodes(0);
        if (!same) e.adopt_legs(legs);
        for (int i = 0; i < nn; ++i) {
            if ((int64_t)data[i].size() != e.nodes[i].tab.size())
                fail(QED_ERR_INVALID_ARG, "checkpoint node size does not match");
            C(ctx).dev.upload(e.nodes[i].ptr(), data[i].data(), data[i].size() * sizeof(double));
        }
        e.invalidate();
        e.isometric = iso != 0;
        e.sweeps_done = sweeps;
        e.sweep_energies.assign(sweeps, NAN);
        e.have_energy = have_e != 0;
        e.energy = energy;
        return QED_OK;
    });
}

int qed_debug_poison(qed_ctx* ctx, int node) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        need_built(C(ctx));
        Engine& e = *C(ctx).eng;
        if (e.nodes.empty()) fail(QED_ERR_BAD_STATE, "no state");
        if (node < 0 || node >= (int)e.nodes.size()) fail(QED_ERR_INVALID_ARG, "bad node");
        const double nan = std::numeric_limits<double>::quiet_NaN();
        C(ctx).dev.upload(e.nodes[node].ptr(), &nan, sizeof(double));
        e.invalidate();
        return QED_OK;
    });
}

int qed_sweep(qed_ctx* ctx, int n, qed_sweep_report* rep) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        need_built(C(ctx));
        if (n < 0) fail(QED_ERR_INVALID_ARG, "negative sweep count");
        Engine& e = *C(ctx).eng;
        if (e.nodes.empty()) fail(QED_ERR_BAD_STATE, "no state: call qed_init_state first");
        for (int i = 0; i < n; ++i) e.sweep(i, rep ? rep + i : nullptr);
        if (e.have_energy && !std::isfinite(e.energy)) fail(QED_ERR_NONFINITE, "non-finite energy");
        return QED_OK;
    });
}

int qed_get_energy(qed_ctx* ctx, double* E) {
    return guard(ctx, [&] {
        need_built(C(ctx));
        if (!E) fail(QED_ERR_INVALID_ARG, "E is NULL");
        if (!C(ctx).eng->have_energy) fail(QED_ERR_BAD_STATE, "no sweep has run");
        *E = C(ctx).eng->energy;
        return QED_OK;
    });
}

int qed_get_observables(qed_ctx* ctx, double* occ, double* efield, double* deltaL, double* rho,
                        double* Q) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        need_built(C(ctx));
        Engine& e = *C(ctx).eng;
        if (e.nodes.empty()) fail(QED_ERR_BAD_STATE, "no state");
        std::vector<double> s7;
        e.observables(s7);
        const Lattice& L = e.model.lat;
        double dL = 0.0, q = 0.0, r = 0.0;
        for (int x = 0; x < L.N; ++x) {
            const double phi = s7[x * 7];
            const int p = L.parity(x);
            if (occ) occ[x] = phi;
            q += phi - p;
            r += p + (1 - 2 * p) * phi;
            for (int mu = 0; mu < 3; ++mu) {
                const int y = L.neighbour(x, 3 + mu);
                if (efield) efield[x * 3 + mu] = y < 0 ? 0.0 : 1.0 - s7[x * 7 + 1 + 3 + mu];
                if (y >= 0) dL += std::fabs(s7[x * 7 + 1 + 3 + mu] + s7[y * 7 + 1 + mu] - 2.0);
            }
        }
        if (deltaL) *deltaL = dL;
        if (rho) *rho = r / L.N;
        if (Q) *Q = q;
        return QED_OK;
    });
}

namespace {

// Per-site Gauss-law charge <phi - p> and outgoing half-link fluxes
// <1 - k_h> (h = -x, -y, -z, +x, +y, +z) of the current state.
void site_fluxes(qed::Engine& e, std::vector<double>& charge, std::vector<double>& flux) {
    std::vector<double> s7;
    e.observables(s7);
    const qed::Lattice& L = e.model.lat;
    charge.assign(L.N, 0.0);
    flux.assign((size_t)L.N * 6, 0.0);
    for (int x = 0; x < L.N; ++x) {
        charge[x] = s7[x * 7] - L.parity(x);
        for (int h = 0; h < 6; ++h) flux[(size_t)x * 6 + h] = 1.0 - s7[x * 7 + 1 + h];
    }
}

int shell_count(const qed::Lattice& L) {
    int m = L.L[0];
    for (int a = 1; a < 3; ++a) m = std::min(m, L.L[a]);
    return 1 + (m - 1) / 2;
}

}  // namespace

int qed_get_site_fluxes(qed_ctx* ctx, double* charge, double* flux) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        need_built(C(ctx));
        Engine& e = *C(ctx).eng;
        if (e.nodes.empty()) fail(QED_ERR_BAD_STATE, "no state");
        std::vector<double> q, f;
        site_fluxes(e, q, f);
        if (charge) std::copy(q.begin(), q.end(), charge);
        if (flux) std::copy(f.begin(), f.end(), flux);
        return QED_OK;
    });
}

int qed_get_plane_profiles(qed_ctx* ctx, int axis, double* qc, double* ec) {
    return guard(ctx, [&] {
        if (axis < 0 || axis > 2) fail(QED_ERR_INVALID_ARG, "axis must be 0, 1 or 2");
        need_device(C(ctx));
        need_built(C(ctx));
        Engine& e = *C(ctx).eng;
        if (e.nodes.empty()) fail(QED_ERR_BAD_STATE, "no state");
        std::vector<double> q, f;
        site_fluxes(e, q, f);
        const Lattice& L = e.model.lat;
        const int La = L.L[axis];
        const double w = 2.0 * La / L.N;  // 2 / (sites per plane)
        std::vector<double> sq(La, 0.0), se(La + 1, 0.0);
        for (int x = 0; x < L.N; ++x) {
            int c[3];
            L.coords(x, c);
            const int d = c[axis];
            sq[d] += q[x];
            se[d + 1] += f[(size_t)x * 6 + 3 + axis];
            if (d == 0) se[0] -= f[(size_t)x * 6 + axis];
        }
        if (qc)
            for (int d = 0; d < La; ++d) qc[d] = w * sq[d];
        if (ec)
            for (int d = 0; d <= La; ++d) ec[d] = w * se[d];
        return QED_OK;
    });
}

int qed_get_surface_density(qed_ctx* ctx, double* sigma, int* nshell) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        need_built(C(ctx));
        Engine& e = *C(ctx).eng;
        if (e.nodes.empty()) fail(QED_ERR_BAD_STATE, "no state");
        const Lattice& L = e.model.lat;
        const int ns = shell_count(L);
        if (nshell) *nshell = ns;
        if (!sigma) return QED_OK;
        std::vector<double> q, f;
        site_fluxes(e, q, f);
        std::vector<double> tot(ns, 0.0);
        std::vector<int> cnt(ns, 0);
        for (int x = 0; x < L.N; ++x) {
            int c[3];
            L.coords(x, c);
            int l = INT32_MAX;
            for (int a = 0; a < 3; ++a) l = std::min(l, std::min(c[a], L.L[a] - 1 - c[a]));
            tot[l] += q[x];
            ++cnt[l];
        }
        for (int l = 0; l < ns; ++l) sigma[l] = tot[l] / cnt[l];
        return QED_OK;
    });
}

int qed_pin_charges(qed_ctx* ctx, int n, const int* sites, const int* charges, double lambda) {
    return guard(ctx, [&] {
        Params& P = C(ctx).prm;
        if (!P.have_lattice) fail(QED_ERR_BAD_STATE, "call qed_set_lattice first");
        if (n < 0 || (n > 0 && (!sites || !charges)))
            fail(QED_ERR_INVALID_ARG, "need n >= 0 sites and charges");
        if (!std::isfinite(lambda) || lambda <= 0.0)
            fail(QED_ERR_INVALID_ARG, "lambda must be finite and positive");
        const int N = P.Lx * P.Ly * P.Lz;
        std::vector<double> mu = P.mu.empty() ? std::vector<double>(N, 0.0) : P.mu;
        std::vector<char> seen(N, 0);
        for (int i = 0; i < n; ++i) {
            const int s = sites[i], q = charges[i];
            if (s < 0 || s >= N) fail(QED_ERR_INVALID_ARG, "site index out of range");
            if (seen[s]) fail(QED_ERR_INVALID_ARG, "site pinned twice");
            seen[s] = 1;
            const int p = (s % P.Lx + (s / P.Lx) % P.Ly + s / (P.Lx * P.Ly)) & 1;
            const int occ = q + p;
            if (occ != 0 && occ != 1)
                fail(QED_ERR_INVALID_ARG, "charge cannot sit on a site of this parity "
                                          "(+1 needs an even site, -1 an odd site)");
            mu[s] += occ == 1 ? -lambda : lambda;
        }
        P.mu = mu;
        C(ctx).built = false;
        return QED_OK;
    });
}

int qed_set_profiling(qed_ctx* ctx, int on) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        C(ctx).dev.sync();
        C(ctx).prof.reset();
        C(ctx).prof.on = on != 0;
        return QED_OK;
    });
}

int qed_get_stats(qed_ctx* ctx, qed_stats* out) {
    return guard(ctx, [&] {
        if (!out) fail(QED_ERR_INVALID_ARG, "out is NULL");
        if (!C(ctx).host_only) {
            C(ctx).dev.sync();
            C(ctx).prof.harvest();
        }
        out->matvec_flops = C(ctx).mv_flops;
        out->matvecs = C(ctx).mv_count;
        out->gemm_launches = C(ctx).prof.launches;
        out->gemm_ms = C(ctx).prof.ms;
        out->gemm_flops = C(ctx).prof.flops;
        out->fused_launches = C(ctx).prof.f_launches;
        out->fused_ms = C(ctx).prof.f_ms;
        out->fused_flops = C(ctx).prof.f_flops;
        return QED_OK;
    });
}

int qed_node_blocks(const int* ch_l, const int* n_l, int s_l, const int* ch_r, const int* n_r,
                    int s_r, const int* ch_p, const int* n_p, int s_p, int flux, int cap, int* nblk,
                    int* triples, int64_t* offs) {
    try {
        Leg l = make_leg(ch_l, n_l, s_l), r = make_leg(ch_r, n_r, s_r), p = make_leg(ch_p, n_p, s_p);
        BlockTable t = make_table(l, r, p, flux);
        if (!nblk) return QED_ERR_INVALID_ARG;
        *nblk = t.nblk();
        if ((triples || offs) && cap < t.nblk()) return QED_ERR_INVALID_ARG;
        for (int b = 0; b < t.nblk(); ++b) {
            if (triples) {
                triples[3 * b] = t.s[0][b];
                triples[3 * b + 1] = t.s[1][b];
                triples[3 * b + 2] = t.s[2][b];
            }
            if (offs) offs[b] = t.off[b];
        }
        if (offs) offs[t.nblk()] = t.size();
        return QED_OK;
    } catch (const Error& e) {
        return e.code;
    } catch (...) {
        return QED_ERR_INVALID_ARG;
    }
}

int qed_heff_create(qed_ctx* ctx, const int* ch_l, const int* n_l, int s_l, const int* ch_r,
                    const int* n_r, int s_r, const int* ch_p, const int* n_p, int s_p, int K,
                    const qed_term* terms, qed_heff** out) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        if (!out || K < 0 || (K > 0 && !terms)) fail(QED_ERR_INVALID_ARG, "bad arguments");
        *out = nullptr;
        auto h = std::make_unique<qed_heff>();
        Heff& H = h->h;
        h->owner = ctx;
        H.ctx = &C(ctx);
        H.legs[0] = make_leg(ch_l, n_l, s_l);
        H.legs[1] = make_leg(ch_r, n_r, s_r);
        H.legs[2] = make_leg(ch_p, n_p, s_p);
        H.tab = make_table(H.legs[0], H.legs[1], H.legs[2], 0);
        if (H.tab.nblk() == 0) fail(QED_ERR_INVALID_ARG, "the node has no allowed block");
        Dev* dev = &C(ctx).dev;
        for (int k = 0; k < K; ++k) {
            const qed_term& t = terms[k];
            if (!std::isfinite(t.coef)) fail(QED_ERR_INVALID_ARG, "non-finite coefficient");
            int sh[3];
            for (int e = 0; e < 3; ++e) sh[e] = t.op[e] ? t.shift[e] : 0;
            if (sh[0] + sh[1] != sh[2]) fail(QED_ERR_INVALID_ARG, "term shifts must obey shift_l + shift_r = shift_p");
            HTerm ht{t.coef, {nullptr, nullptr, nullptr}};
            for (int e = 0; e < 3; ++e) {
                if (!t.op[e]) continue;
                OpP o = make_op(dev, H.legs[e], sh[e], false);
                if (o->lay.size)
                    dev->check(hipMemcpyAsync(o->d64->p, t.op[e], o->lay.size * sizeof(double),
                                              hipMemcpyDeviceToDevice, dev->stream), "operator copy");
                ht.op[e] = o;
            }
            H.terms.push_back(ht);
        }
        const int dtype = C(ctx).prm.dtype;
        H.plan = plan_matvec(H.legs, H.tab, H.terms, dtype);
        H.plan.upload(dev);
        if (dtype != QED_FP64) {
            H.xc = std::make_shared<DBuf>(dev, H.tab.size() * dtype_size(dtype));
            H.yc = std::make_shared<DBuf>(dev, H.tab.size() * dtype_size(dtype));
        }
        if (C(ctx).tuner.on) {
            const size_t es = dtype_size(dtype);
            void* w = H.ws.get(dev, std::max<int64_t>(1, H.plan.ws_elems) * es);
            DBuf tx(dev, H.tab.size() * es), ty(dev, H.tab.size() * es);
            C(ctx).tuner.tune(dev, H.plan, w, tx.p, ty.p);
        }
        dev->sync();
        *out = h.release();
        return QED_OK;
    });
}

int qed_heff_destroy(qed_heff* h) {
    if (!h) return QED_ERR_INVALID_ARG;
    try {
        (void)hipStreamSynchronize(h->h.ctx->dev.stream);
    } catch (...) {
    }
    delete h;
    return QED_OK;
}

int qed_heff_size(qed_heff* h, int64_t* size) {
    if (!h || !size) return QED_ERR_INVALID_ARG;
    *size = h->h.tab.size();
    return QED_OK;
}

int qed_heff_matvec(qed_heff* h, const double* x, double* y) {
    if (!h) return QED_ERR_INVALID_ARG;
    qed_ctx* ctx = h->owner;
    return guard(ctx, [&] {
        if (!x || !y || x == y) fail(QED_ERR_INVALID_ARG, "x and y must be distinct device buffers");
        h->h.matvec(x, y);
        h->h.ctx->dev.check(hipGetLastError(), "matvec");
        return QED_OK;
    });
}

int qed_heff_matvec_noalloc(qed_heff* h, const double* x, double* y) {
    if (!h) return QED_ERR_INVALID_ARG;
    qed_ctx* ctx = h->owner;
    return guard(ctx, [&] {
        if (!x || !y || x == y) fail(QED_ERR_INVALID_ARG, "x and y must be distinct device buffers");
        Heff& H = h->h;
        const size_t need =
            (size_t)std::max<int64_t>(1, H.plan.ws_elems) * (size_t)dtype_size(H.plan.dtype);
        if (need > SCRATCH_BYTES)
            fail(QED_ERR_INVALID_ARG, "this H_eff needs " + std::to_string(need) +
                                          " bytes of workspace; the allocation-free matvec has " +
                                          std::to_string(SCRATCH_BYTES));
        void* w = scratch_for(H.ctx->dev.device);
        if (!w) fail(QED_ERR_HIP, "the scratch address of this device could not be looked up");
        H.matvec_ws(x, y, w);
        H.ctx->dev.check(hipGetLastError(), "matvec (allocation-free)");
        return QED_OK;
    });
}

int qed_heff_lanczos(qed_heff* h, double* x, int steps, double* eval, double* resid) {
    if (!h) return QED_ERR_INVALID_ARG;
    qed_ctx* ctx = h->owner;
    return guard(ctx, [&] {
        if (!x || !eval) fail(QED_ERR_INVALID_ARG, "x and eval are required");
        Heff& H = h->h;
        const Params& P = H.ctx->prm;
        const int m = steps > 0 ? steps : P.lz_steps;
        if (m > 64) fail(QED_ERR_INVALID_ARG, "at most 64 Lanczos steps");
        LanczosResult R = lanczos(&H.ctx->dev, H.lws,
                                  [&](const double* v, const float*, double* w, double*) {
                                      H.matvec(v, w);
                                      return false;
                                  },
                                  x,
                                  H.tab.size(), m, P.lz_cycles, P.lz_tol);
        *eval = R.theta;
        if (resid) *resid = R.resid;
        if (P.lz_tol > 0 && R.resid > P.lz_tol * std::fabs(R.theta)) return (int)QED_NOT_CONVERGED;
        return (int)QED_OK;
    });
}

int qed_heff_matvec_adjoint(qed_heff* h, const double* x, const double* ybar, double* xbar,
                            double* const* opbar, double* coefbar) {
    if (!h) return QED_ERR_INVALID_ARG;
    return guard(h->owner, [&] {
        if (!x || !ybar) fail(QED_ERR_INVALID_ARG, "x and ybar are required");
        if (xbar && (xbar == x || xbar == ybar)) fail(QED_ERR_INVALID_ARG, "xbar must not alias");
        h->h.adjoint(x, ybar, xbar, opbar, coefbar);
        return (int)QED_OK;
    });
}

int qed_heff_flops(qed_heff* h, double* flops, double* bytes) {
    if (!h) return QED_ERR_INVALID_ARG;
    if (flops) *flops = h->h.plan.flops;
    if (bytes) *bytes = h->h.plan.bytes;
    return QED_OK;
}

int qed_heff_adjoint_flops(qed_heff* h, double* xbar_flops, double* grad_flops) {
    if (!h) return QED_ERR_INVALID_ARG;
    return guard(h->owner, [&] {
        if (!h->h.adj.built) h->h.build_adjoint();
        if (xbar_flops) *xbar_flops = h->h.adj.xbar.flops;
        if (grad_flops) *grad_flops = h->h.adj.grads.flops;
        return (int)QED_OK;
    });
}

int qed_autotune(qed_ctx* ctx, const char* cache_path) {
    return guard(ctx, [&] {
        Tuner& t = C(ctx).tuner;
        if (cache_path && cache_path[0] == '\0') {
            t.on = false;
            return (int)QED_OK;
        }
        t.on = true;
        t.path = cache_path ? cache_path : "";
        t.load();
        return (int)QED_OK;
    });
}

int qed_heff_batch_create(qed_ctx* ctx, int nnodes, const qed_heff_desc* nodes,
                          qed_heff_batch** out) {
    return guard(ctx, [&] {
        need_device(C(ctx));
        if (!out || nnodes <= 0 || !nodes) fail(QED_ERR_INVALID_ARG, "bad arguments");
        *out = nullptr;
        auto hb = std::make_unique<qed_heff_batch>();
        hb->owner = ctx;
        HeffBatch& B = hb->b;
        B.ctx = &C(ctx);
        Dev* dev = &C(ctx).dev;
        const int dtype = C(ctx).prm.dtype;
        B.nn = nnodes;
        B.off.push_back(0);
        B.plan.dtype = dtype;
        for (int i = 0; i < nnodes; ++i) {
            const qed_heff_desc& d = nodes[i];
            std::array<Leg, 3> lg;
            for (int e = 0; e < 3; ++e) lg[e] = make_leg(d.ch[e], d.n[e], d.nsec[e]);
            BlockTable tab = make_table(lg[0], lg[1], lg[2], 0);
            if (tab.nblk() == 0) fail(QED_ERR_INVALID_ARG, "a node has no allowed block");
            if (d.K < 0 || (d.K > 0 && !d.terms)) fail(QED_ERR_INVALID_ARG, "bad terms");
            std::vector<HTerm> ts;
            for (int k = 0; k < d.K; ++k) {
                const qed_term& t = d.terms[k];
                if (!std::isfinite(t.coef)) fail(QED_ERR_INVALID_ARG, "non-finite coefficient");
                int sh[3];
                for (int e = 0; e < 3; ++e) sh[e] = t.op[e] ? t.shift[e] : 0;
                if (sh[0] + sh[1] != sh[2]) fail(QED_ERR_INVALID_ARG, "term shifts must obey shift_l + shift_r = shift_p");
                HTerm ht{t.coef, {nullptr, nullptr, nullptr}};
                for (int e = 0; e < 3; ++e) {
                    if (!t.op[e]) continue;
                    OpP o = make_op(dev, lg[e], sh[e], false);
                    if (o->lay.size)
                        dev->check(hipMemcpyAsync(o->d64->p, t.op[e], o->lay.size * sizeof(double),
                                                  hipMemcpyDeviceToDevice, dev->stream), "operator copy");
                    ht.op[e] = o;
                }
                ts.push_back(ht);
            }
            B.legs.push_back(lg);
            B.tabs.push_back(tab);
            B.terms.push_back(ts);
            append_matvec(B.plan, lg.data(), tab, ts, B.off.back());
            B.off.push_back(B.off.back() + tab.size());
        }
        const int64_t N = B.off.back();
        B.plan.upload(dev);
        B.ws = std::make_shared<DBuf>(dev, std::max<int64_t>(1, B.plan.ws_elems) * dtype_size(dtype));
        if (dtype != QED_FP64) {
            B.xc = std::make_shared<DBuf>(dev, N * dtype_size(dtype));
            B.yc = std::make_shared<DBuf>(dev, N * dtype_size(dtype));
        }
        dev->check(hipStreamCreateWithFlags(&B.stream, hipStreamNonBlocking), "stream");
        if (C(ctx).tuner.on) {
            DBuf tx(dev, N * dtype_size(dtype)), ty(dev, N * dtype_size(dtype));
            C(ctx).tuner.tune(dev, B.plan, B.ws->p, tx.p, ty.p);
        }
        dev->sync();
        *out = hb.release();
        return (int)QED_OK;
    });
}

int qed_heff_batch_destroy(qed_heff_batch* b) {
    if (!b) return QED_ERR_INVALID_ARG;
    try {
        (void)hipStreamSynchronize(b->b.ctx->dev.stream);
    } catch (...) {
    }
    delete b;
    return QED_OK;
}

int qed_heff_batch_size(qed_heff_batch* b, int64_t* total, int64_t* offs) {
    if (!b) return QED_ERR_INVALID_ARG;
    if (total) *total = b->b.off.back();
    if (offs)
        for (size_t i = 0; i < b->b.off.size(); ++i) offs[i] = b->b.off[i];
    return QED_OK;
}

int qed_heff_batch_matvec(qed_heff_batch* b, const double* x, double* y) {
    if (!b) return QED_ERR_INVALID_ARG;
    return guard(b->owner, [&] {
        if (!x || !y || x == y) fail(QED_ERR_INVALID_ARG, "x and y must be distinct device buffers");
        Dev& dev = b->b.ctx->dev;
        b->b.plan.prof = &b->b.ctx->prof;
        b->b.matvec(x, y, dev.stream);
        b->b.plan.prof = nullptr;
        dev.check(hipGetLastError(), "batch matvec");
        Ctx& c = *b->b.ctx;
        c.mv_flops += b->b.plan.flops;
        c.mv_count += 1;
        return (int)QED_OK;
    });
}

int qed_heff_batch_lanczos(qed_heff_batch* b, double* x, int steps, double* evals, double* resids,
                           int use_graph) {
    if (!b) return QED_ERR_INVALID_ARG;
    return guard(b->owner, [&] {
        if (!x || !evals) fail(QED_ERR_INVALID_ARG, "x and evals are required");
        HeffBatch& B = b->b;
        Ctx& c = *B.ctx;
        Dev& dev = c.dev;
        const Params& P = c.prm;
        const int m = steps > 0 ? steps : P.lz_steps;
        if (m < 1 || m > 64) fail(QED_ERR_INVALID_ARG, "1 .. 64 Lanczos steps");
        // an FP32 plan keeps the basis in FP32 (its matvec reads the basis
        // row itself), as the sweep path does; QEDTTN_LZ_BASIS=fp64 keeps it
        // in FP64
        const char* bv = std::getenv("QEDTTN_LZ_BASIS");
        const bool b32 = B.plan.dtype == QED_FP32 && m + 1 <= 32 && !(bv && !std::strcmp(bv, "fp64"));
        if (B.lz.m != m || B.lz.nseg != B.nn || B.lz.b32 != b32) {
            B.lz.setup(&dev, B.off, B.off.back(), m, b32);
            // a captured cycle refers to the old buffers
            if (B.gexec) (void)hipGraphExecDestroy(B.gexec);
            if (B.graph) (void)hipGraphDestroy(B.graph);
            B.gexec = nullptr;
            B.graph = nullptr;
        }
        // the batch runs on its own stream (graph capture needs one)
        dev.sync();
        auto apply = [&](const double* v, const float* v32, double* y) {
            if (v32) B.matvec32(v32, y, B.stream);
            else B.matvec(v, y, B.stream);
        };
        if (use_graph && (!B.gexec || B.gm != m || B.gx != x)) {
            if (B.gexec) (void)hipGraphExecDestroy(B.gexec);
            if (B.graph) (void)hipGraphDestroy(B.graph);
            B.gexec = nullptr;
            B.graph = nullptr;
            dev.check(hipStreamBeginCapture(B.stream, hipStreamCaptureModeThreadLocal), "capture");
            B.lz.cycle(apply, x, B.stream);
            dev.check(hipStreamEndCapture(B.stream, &B.graph), "capture");
            dev.check(hipGraphInstantiate(&B.gexec, B.graph, nullptr, nullptr, 0), "graph instantiate");
            B.gm = m;
            B.gx = x;
        }
        std::vector<LState> hs(B.nn);
        int rc = QED_OK;
        for (int cyc = 0; cyc < std::max(1, P.lz_cycles); ++cyc) {
            if (use_graph) dev.check(hipGraphLaunch(B.gexec, B.stream), "graph launch");
            else B.lz.cycle(apply, x, B.stream);
            dev.check(hipGetLastError(), "batch lanczos");
            dev.check(hipMemcpyAsync(hs.data(), B.lz.st->p, B.nn * sizeof(LState),
                                     hipMemcpyDeviceToHost, B.stream), "state copy");
            dev.check(hipStreamSynchronize(B.stream), "sync");
            c.mv_count += m;
            c.mv_flops += (double)m * B.plan.flops;
            bool all = true;
            for (int i = 0; i < B.nn; ++i) {
                if (!std::isfinite(hs[i].theta)) fail(QED_ERR_NONFINITE, "non-finite Ritz value");
                if (hs[i].resid > P.lz_tol * std::fabs(hs[i].theta)) all = false;
            }
            if (all) break;
            if (cyc + 1 == std::max(1, P.lz_cycles) && P.lz_tol > 0) rc = QED_NOT_CONVERGED;
        }
        for (int i = 0; i < B.nn; ++i) {
            evals[i] = hs[i].theta;
            if (resids) resids[i] = hs[i].resid;
        }
        return rc;
    });
}

int qed_heff_batch_flops(qed_heff_batch* b, double* flops, double* bytes) {
    if (!b) return QED_ERR_INVALID_ARG;
    if (flops) *flops = b->b.plan.flops;
    if (bytes) *bytes = b->b.plan.bytes;
    return QED_OK;
}

}  // extern "C"
