// Device-side engine of the TTN node update: memory, block-sparse leg
// operators, contraction plans, the Lanczos driver and the sweep.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "model.h"
#include "tree.h"

namespace qed {

// ---- kernel launchers (kernels.hip) ----------------------------------
// flat: products of a job as one pipelined sequence of K chunks (pays off
// for short reductions); otherwise one pipeline per product.  buf: operands
// and output through buffer resources (every block of the stage within
// 2^31-byte offsets; the flat pipeline always needs it)
template <typename T>
void launch_brgemm(const GJob*, const GProd*, const GTile*, int, const Bases&, int shape, bool flat,
                   bool buf, hipStream_t);
// fused H_eff stage: per output tile, every term's child-leg product and
// bond-leg epilogue (heff_fused.hip)
// (cs_rows x cs_cols: the largest bond-factor block of the launch, input
// sector by 16-padded output sector)
template <typename T>
void launch_heff_fused(const FJob*, const FProd*, const GTile*, int, const Bases&, int cs_rows,
                       int cs_cols, hipStream_t);
void launch_fill(double*, int64_t, double, hipStream_t);
void launch_f64_to_f32(const double*, float*, int64_t, hipStream_t);
void launch_f64_to_f32_segs(const ConvSeg* segs, int nseg, hipStream_t);
void launch_f32_to_f64(const float*, double*, int64_t, hipStream_t);
int dot_grid(int64_t n);
void launch_dots(const double* V, int64_t ldv, int nrows, const double* w, int64_t n,
                 double* partial, double* out, int mode, const LState* st, int skip,
                 hipStream_t stream);
// stages whose products are all identity products (sums of blocks): one
// workgroup per SUM_TILE consecutive output elements of a job
void launch_sum_stage(int dtype, const GJob*, const GProd*, const GTile*, int, const Bases&, hipStream_t);
// (TV: the basis element type, double or float)
template <typename TV>
bool launch_lz_fused(int mode, double* w, const TV* V, int64_t ldv, int nrows, int j,
                     const double* alpha, const double* beta, const double* c, const double* cf,
                     int64_t n, double* partial, double* out, const LState* st, hipStream_t s);
// mode 2 of launch_lz_fused with the beta step of launch_lz_beta fused into
// its final reduction
template <typename TV>
bool launch_lz_norm_beta(double* w, const TV* V, int64_t ldv, int nrows, int j, double* alpha,
                         double* beta, const double* c, const double* cf, int64_t n, double* partial,
                         double* ww, LState* st, double tol, hipStream_t s);
// w = (double) a with the partials of v . w (layout of launch_dots, one row)
template <typename TV>
void launch_f32_to_f64_dot(const float* a, double* w, const TV* v, int64_t n, double* partial,
                           const LState* st, hipStream_t s);
// the final pass of launch_dots alone
void launch_dot_final(const double* partial, int64_t n, int nrows, double* out, int mode,
                      const LState* st, int skip, hipStream_t s);
void launch_lz_three_term(double*, const double*, int64_t, int, const double*, const double*,
                          int64_t, const LState*, hipStream_t);
void launch_lz_subtract(double*, const double*, int64_t, int, const double*, int64_t,
                        const LState*, hipStream_t);
void launch_lz_beta(const double*, double*, double*, int, LState*, double, hipStream_t);
template <typename TV>
void launch_lz_next(TV*, int64_t, int, const double*, const double*, int64_t, const LState*, hipStream_t,
                    float* vc = nullptr);
template <typename TV>
void launch_lz_start(TV*, const double*, const double*, int64_t, LState*, int, hipStream_t);
void launch_tridiag(const double*, const double*, double*, LState*, double*, hipStream_t);
template <typename TV>
void launch_ritz(double*, const TV*, int64_t, const double*, int64_t, const LState*, hipStream_t);
void launch_normalise_sign(double*, int64_t, const double*, double*, int64_t*, double*,
                           hipStream_t);
void launch_pack(const PackBlk*, int, int64_t, double*, double*, int, hipStream_t);
// blocked kernel when every matrix has rows <= QR_ROWS and cols <= QR_COLS,
// else the unblocked one
void launch_qr(const QRMat*, int nmats, int64_t maxrows, int maxcols, hipStream_t);
void launch_qr_lds(const QRMat*, int nmats, size_t lds_bytes, hipStream_t);
void launch_site_expect(const double*, const int64_t*, const signed char*, int, double*,
                        hipStream_t);
void launch_jacobi_svd(const SvdMat*, int nmats, hipStream_t);
// Cholesky of every sector's Gram matrix, R^-1 and the running R
void launch_chol_inv(const CholMat*, int nmats, int maxn, hipStream_t);
void launch_axpy(double* y, const double* x, double f, int64_t n, hipStream_t);

// (TV: the basis element type, double or float; w, the coefficients and
// the Ritz vector are FP64 either way)
template <typename TV>
void seg_dots(const TV* V, int64_t ldv, int nrows, const double* w, const SegChunk* ch, int nch, const int* seg_c0,
              int nseg, double* partial, double* out, int ldo, int mode, const LState* st, int skip, hipStream_t s);
void seg_init(LState*, int, int, const double*, int, hipStream_t);
template <typename TV>
void seg_start(TV* dst, const double* src, const double* nrm, int ldn, const SegChunk* ch, int nch, hipStream_t s);
// one fused pass of a Lanczos step per segment (mode 0, 1, 2 as in
// launch_lz_fused), with its final sums into out[seg * ldo + r]; false
// (nothing launched) when the pass would need more than 32 rows
template <typename TV>
bool seg_fused(int mode, double* w, const TV* V, int64_t ldv, int nrows, int j, const double* al,
               const double* be, int lds, const double* c, const double* cf, const SegChunk* ch, int nch,
               const int* seg_c0, int nseg, double* partial, double* out, int ldo, const LState* st,
               hipStream_t s);
void seg_three_term(double*, const double*, int64_t, int, const double*, const double*, int,
                    const SegChunk*, int, const LState*, hipStream_t);
void seg_subtract(double*, const double*, int64_t, int, const double*, int, const SegChunk*, int,
                  const LState*, hipStream_t);
void seg_beta(const double*, int, double*, double*, int, int, LState*, int, double, hipStream_t);
template <typename TV>
void seg_next(TV* V, int64_t ldv, int j, const double* w, const double* be, int lds, const SegChunk* ch, int nch,
              const LState* st, hipStream_t s);
void seg_tridiag(const double*, const double*, int, double*, LState*, double*, int, hipStream_t);
template <typename TV>
void seg_ritz(double* u, const TV* V, int64_t ldv, const double* sv, int lds, const SegChunk* ch, int nch,
              const LState* st, hipStream_t s);
void seg_normalise_sign(double*, const SegChunk*, int, const int*, int, const double*, int,
                        double*, int64_t*, double*, hipStream_t);

// skinny stages (GEMM_PIPE_SKINNY): rows per workgroup strip, and launch
int skinny_rows(int dtype);
template <typename T>
void launch_skinny(const GJob*, const GProd*, const GTile*, int, const Bases&, hipStream_t);
// FP32 and FP64 block GEMMs whose operands travel straight into an LDS
// ring (GEMM_PIPE_DMA; SQUARE and WIDE tiles only)
bool brgemm_dma_shape(int shape);
void launch_brgemm_dma(const GJob*, const GProd*, const GTile*, int, const Bases&, int shape, hipStream_t);
void launch_brgemm_dma64(const GJob*, const GProd*, const GTile*, int, const Bases&, int shape, hipStream_t);
void launch_brgemm_bf16(const GJob*, const GProd*, const GTile*, int, const Bases&, int shape,
                        hipStream_t);
void launch_f64_to_bf16(const double*, void*, int64_t, hipStream_t);
void launch_bf16_to_f64(const void*, double*, int64_t, double, hipStream_t);
void launch_transpose_blocks(const double*, double*, const int64_t*, int, hipStream_t);
void launch_scale_to_f64(const void*, int, double*, int64_t, double, hipStream_t);
void launch_adj_scale(const AdjSeg*, int nseg, int64_t maxn, hipStream_t);
void launch_adj_dots(const AdjSeg*, int nseg, double* out, hipStream_t);

// ---- device memory ---------------------------------------------------
struct Dev {
    int device = -1;
    hipStream_t stream = nullptr;
    void* (*ualloc)(uint64_t, void*, void*) = nullptr;
    void (*ufree)(void*, void*, void*) = nullptr;
    void* user = nullptr;
    bool used = false;
    // Released blocks kept for reuse, keyed by size class.  A block is
    // handed out again only to an allocation on the stream that released
    // it, so stream order alone separates its old and new users (the same
    // rule as the stream-ordered pool, without an API call per buffer).
    struct Cached {
        void* p;
        hipStream_t stream;
    };
    std::multimap<size_t, Cached> cache;
    std::unordered_map<void*, size_t> live;   // cacheable blocks in use -> size class
    size_t cached_bytes = 0;

    void check(hipError_t e, const char* what);
    void* alloc(size_t bytes);
    void release(void* p);
    // Pinned upload ring: small host-to-device copies are staged here and
    // run asynchronously in stream order.  A region is written again only
    // after the staging stream has been synchronised (every Dev::sync of
    // that stream, or a wrap of the ring, which syncs).
    unsigned char* ring = nullptr;
    size_t ring_pos = 0;
    hipStream_t ring_stream = nullptr;
    bool ring_failed = false;
    bool stage(void* dst, const void* src, size_t bytes);   // false: not staged
    void trim();   // return every cached block to the pool (stream-ordered)
    void restream(hipStream_t s);   // after a sync: cached blocks move to stream s
    void sync();
    void upload(void* dst, const void* src, size_t bytes);
    void download(void* dst, const void* src, size_t bytes);
    ~Dev();
};

struct DBuf {
    Dev* dev = nullptr;
    void* p = nullptr;
    size_t bytes = 0;
    DBuf(Dev* d, size_t b) : dev(d), bytes(b) { p = b ? d->alloc(b) : nullptr; }
    ~DBuf() {
        if (p) dev->release(p);
    }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    template <typename T> T* as() const { return (T*)p; }
};
using BufP = std::shared_ptr<DBuf>;

// Grow-only scratch area.
struct Arena {
    BufP buf;
    void* get(Dev* d, size_t bytes) {
        if (!buf || buf->bytes < bytes) {
            buf.reset();
            buf = std::make_shared<DBuf>(d, bytes + bytes / 4 + 4096);
        }
        return buf->p;
    }
};

// Block-sparse operator on one leg (FP64 master data, lazy FP32 copy).
struct LegOpD {
    Leg leg;
    OpLayout lay;
    BufP d64, d32, d16;   // FP64 master copy; lazy FP32 and BF16 copies
    Dev* dev = nullptr;
    const double* f64() const { return d64 ? d64->as<double>() : nullptr; }
    const void* data(int dtype);
};
using OpP = std::shared_ptr<LegOpD>;

OpP make_op(Dev* dev, const Leg& leg, int delta, bool zero = true);
// The FP32 copies that ops still lack, made in one launch (instead of one
// lazy conversion per op when a plan first asks for it).
void prepare_f32_copies(Dev* dev, const std::vector<LegOpD*>& ops);

// Element size of a GEMM operand type and conversions between FP64
// vectors and the operand type (FP32: round to nearest; BF16: FP32 first,
// then round to nearest even).
inline int dtype_size(int dtype) { return dtype == QED_FP64 ? 8 : dtype == QED_BF16 ? 2 : 4; }
void to_compute(int dtype, const double* a, void* b, int64_t n, hipStream_t s);
void from_compute(int dtype, const void* a, double* b, int64_t n, hipStream_t s);

// Node tensor (canonical block layout, FP64).
struct TensorD {
    Leg legs[3];
    BlockTable tab;
    BufP d;
    double* ptr() const { return d ? d->as<double>() : nullptr; }
};

// ---- profiling of the H_eff GEMM launches ------------------------------
struct Prof {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<hipEvent_t> pool;        // harvested events, reused
    std::vector<double> ev_flops;
    std::vector<int> ev_key;             // stage index * 16 + tile shape + 4 pipeline (FUSED_KEY: fused)
    long long launches = 0;
    double ms = 0.0, flops = 0.0;
    long long f_launches = 0;            // the fused kernel's share of the above
    double f_ms = 0.0, f_flops = 0.0;
    static constexpr int FUSED_KEY = 15;
    static constexpr int RUN_KEY = -2;    // one bracket around a plan run's GEMM launches
    std::map<int, std::array<double, 3>> by_key;   // launches, ms, flops per stage and shape
    void record_begin(hipStream_t s, hipEvent_t& a);
    void harvest();     // fold finished event pairs into ms (stream synced)
    void reset();
    void report() const;   // per stage and shape, to stderr
    ~Prof();
};

// ---- contraction plans -----------------------------------------------
struct Plan {
    int dtype = QED_FP64;   // QED_FP64, QED_FP32 or QED_BF16 (GEMM operand type)
    std::vector<double> stage_flops;
    Prof* prof = nullptr;   // set for H_eff applications when profiling
    std::vector<std::vector<GJob>> jobs;
    std::vector<std::vector<GProd>> prods;
    int64_t ws_elems = 0;
    double flops = 0.0;
    double bytes = 0.0;
    // device copies: every stage's jobs, products and tiles in one buffer
    // (one copy per plan), plus re-tiled stages
    std::vector<BufP> hold;
    std::vector<const GJob*> dj;
    std::vector<const GProd*> dp;
    std::vector<const GTile*> dt;
    std::vector<int> ntiles;
    std::vector<int> shape;   // workgroup tile shape per stage
    std::vector<char> sumk;   // stage of identity products only: elementwise sum kernel
    // GEMM pipeline per stage (GEMM_PIPE_*): the flat product pipeline for
    // short reductions, the LDS-DMA ring for long FP32 reductions whose
    // operands it can read (dma_ok), the register-staged loop otherwise
    std::vector<char> pipe;
    std::vector<char> dma_ok;
    std::vector<char> flat_ok;                   // operands within the flat pipeline's 2^31-byte offsets
    std::vector<char> skinny_ok;                 // stage the skinny kernel can run
    std::vector<const GTile*> dts;               // its strip tiles
    std::vector<int> nts;
    // fused H_eff jobs (k_heff_fused) of each stage, launched after the
    // stage's GEMM jobs; stages without them have empty lists (the lists
    // may be shorter than `jobs`)
    std::vector<std::vector<FJob>> fjobs;
    std::vector<std::vector<FProd>> fprods;
    std::vector<double> fstage_flops;
    std::vector<const FJob*> dfj;
    std::vector<const FProd*> dfp;
    std::vector<const GTile*> dft;
    std::vector<int> nftiles;
    std::vector<int> fcs_rows, fcs_cols;   // largest bond block per stage
    void upload(Dev* dev);
    void run(Dev* dev, void* ws, void* x, void* y);
    void run_stage(Dev* dev, int s, void* ws, void* x, void* y);
    void launch_stage(size_t s, const Bases& b, hipStream_t st) const;
    void launch_fused(size_t s, const Bases& b, hipStream_t st) const;
    void set_shape(Dev* dev, int s, int sh);   // re-tile one stage
    bool pipe_valid(size_t s, int pipe, int sh) const;
};

struct HTerm {
    double coef;
    OpP op[3];   // null = identity
};

// y = sum_k coef_k A_k (x) B_k (x) C_k  x on the canonical layout.
Plan plan_matvec(const Leg legs[3], const BlockTable& tab, const std::vector<HTerm>& terms,
                 int dtype);
// Append the jobs of one node's H_eff to P, with x and y at element offset
// xoff of the bound vectors (batched plans concatenate nodes).  By default
// every node runs as mode products in three GEMM stages
// (append_matvec_staged); with QEDTTN_HEFF_FUSED=1, FP32 and FP64 plans of
// nodes whose bond sectors fit a fused tile run the terms with a bond-leg
// factor in fused stages (append_matvec_fused).
void append_matvec(Plan& P, const Leg legs[3], const BlockTable& tab,
                   const std::vector<HTerm>& terms, int64_t xoff);
void append_matvec_staged(Plan& P, const Leg legs[3], const BlockTable& tab,
                          const std::vector<HTerm>& terms, int64_t xoff);
bool append_matvec_fused(Plan& P, const Leg legs[3], const BlockTable& tab,
                         const std::vector<HTerm>& terms, int64_t xoff);

// Renormalised operators n^T (A (x) B) n on leg `which` of node tensor n.
struct RTerm {
    double coef;
    OpP a, b;    // on the two other legs in (l, r, p) order; null = identity
    int out;     // index into outs
};
Plan plan_renorm(const TensorD& n, int which, const std::vector<RTerm>& terms,
                 const std::vector<OpP>& outs);

// Output of a two-tensor contraction: an operator layout on one leg and
// the location of its blocks (compute dtype of the plan).
struct ContractOut {
    Leg leg;
    OpLayout lay;
    GRef base;
};
// Append out[t.out] += coef * sum over the two legs other than `which` of
// partner (x) (in x_f1 a x_f2 b), both canonical tensors with the given
// legs and table (renormalisation when partner = in = a node isometry;
// operator gradients when partner = ybar and in = x).  Uses three stages
// (two mode stages, one contraction stage, optionally split-K): new ones
// appended to the plan, or, with base >= 0, stages base .. base + 2 shared
// with other independent contractions.
void append_contract(Plan& P, const Leg legs[3], const BlockTable& tab, GRef in_base,
                     GRef partner_base, int which, const std::vector<RTerm>& terms,
                     const std::vector<ContractOut>& outs, bool split, int base = -1);

// out_tensor = op applied on leg e of in_tensor (sector preserving op)
Plan plan_mode(const TensorD& in, int e, const OpP& op, double* out);

// Split the jobs of stage s that have few output tiles and a long
// reduction into K-chunk partial products (stage s) summed in stage s+1.
void split_long_reductions(Plan& P, int s);

// When the last stage s of a plan has fewer than target_tiles 64x64 output
// tiles, split every job's product list into up to 8 contiguous groups of
// about equal work (partial jobs into workspace, stage s) and sum the
// partials in a new stage s+1, in a fixed order.
void split_for_occupancy(Plan& P, int s, int64_t target_tiles);

// In-place QR of contiguous column-major m x n matrices M (m >= n):
// M := Q (orthonormal columns), R(r, c) written at R[r*rrs + c*rcs],
// diag(R) >= 0.  Tall matrices use a tree of Householder QRs over row
// chunks (TSQR) with a block GEMM assembling Q.  All matrices of one call
// advance level by level together: one QR launch per tree level (per
// kernel kind), one GEMM launch assembling every Q.
struct QRTask {
    double* M;
    int64_t m;
    int n;
    double* R;
    int64_t rrs, rcs;
};
void tsqr_multi(Dev* dev, const std::vector<QRTask>& tasks);
// CholeskyQR2 of the same tasks: false (matrices untouched) when a sector
// is too wide or rank deficient, to be done by tsqr_multi instead
bool cholqr_multi(Dev* dev, const std::vector<QRTask>& tasks);
void tsqr(Dev* dev, double* M, int64_t m, int n, double* R, int64_t rrs, int64_t rcs);

// ---- Lanczos -----------------------------------------------------------
struct LanczosWS {
    int m = 0;
    int64_t n = 0;
    BufP V, V32, w, alpha, beta, coef, partial, sv, work, st, pv, pi, scal;
    // buffers for m steps on vectors of n; the basis in FP64 (V) or, with
    // b32, in FP32 (V32)
    void ensure(Dev* dev, int m, int64_t n, bool b32 = false);
};

struct LanczosResult {
    double theta = 0.0, resid = 0.0;
    int cycles = 0;
    long long matvecs = 0;
    bool exact = false;   // theta, resid: from the first step of a cycle (see exit_tol)
};

// Lowest eigenpair; x (device FP64, length n) is the start vector and
// receives the normalised Ritz vector.
// apply(v, v32, y, part) computes y = H v: v is the FP64 basis vector, and
// v32, where set, holds v rounded to FP32 already (written by the step that
// formed v); with an FP32 basis v is null and v32 is the basis vector
// itself.  apply may also leave the partials of v . y in part (the layout
// of launch_dots, one row) and then returns true.  With vc set, each new
// FP64 basis vector is also written to vc in FP32.  basis32 keeps the basis
// in FP32 (m <= 31, no exit_tol; apply must then return true): the passes
// over it read half the bytes, the matvec reads its input straight from
// it, and w, the coefficients and the Ritz vector stay FP64.
// exit_tol > 0 (for an apply whose first product of a cycle is exact):
// after the first step of every cycle, alpha_0 = <x, H x> and beta_0 =
// |H x - alpha_0 x| are those of the current vector itself; the run ends
// there once beta_0 <= exit_tol |alpha_0| (x is left normalised, theta =
// alpha_0, resid = beta_0, exact = true), and the estimate from the
// tridiagonal at the end of a cycle does not end it.
using LanczosApply = std::function<bool(const double*, const float*, double*, double*)>;
LanczosResult lanczos(Dev* dev, LanczosWS& ws, const LanczosApply& apply, double* x, int64_t n, int m,
                      int cycles, double tol, float* vc = nullptr, double exit_tol = 0.0, bool basis32 = false);

// ---- node-level effective Hamiltonian (C ABI object) ------------------
struct Ctx;

// Adjoint of H_eff x (hand-written reverse mode):
//   xbar       = sum_k c_k (A_k^T (x) B_k^T (x) C_k^T) ybar
//   Abar_k     = c_k sum_{r,p} ybar (x) (x x_r B_k x_p C_k)      (and B, C alike)
//   cbar_k     = <ybar, A_k (x) B_k (x) C_k x> = <G_k, A_k>_F with G_k the
//                unscaled gradient of the first non-identity factor.
// Intermediates are recomputed (nothing from the forward pass is kept).
struct Adjoint {
    bool built = false;
    Plan xbar;                                  // matvec with transposed factors
    Plan grads;                                 // two-tensor contractions
    std::vector<std::vector<OpP>> opT;          // transposed factors
    std::vector<std::array<int64_t, 3>> goff;   // per term and leg: offset in G, or -1
    int64_t gsize = 0;
    BufP G, G64, ybc;
    Arena ws;
    // coefficient cotangents: one dot segment per term, built once
    std::vector<AdjSeg> dots;
    BufP ddots, cbar;
    Arena dscale;                               // per-call scaling segments
};

struct Heff {
    Ctx* ctx = nullptr;
    Leg legs[3];
    BlockTable tab;
    std::vector<HTerm> terms;
    Plan plan;
    Arena ws;
    BufP xc, yc;   // compute-type staging for reduced precision
    LanczosWS lws;
    Adjoint adj;
    void matvec(const double* x, double* y);
    // the same application with the stage workspace at w (at least
    // plan.ws_elems elements of the plan's type); allocates nothing
    void matvec_ws(const double* x, double* y, void* w);
    void run_matvec(const double* x, double* y, void* w);
    void build_adjoint();
    void adjoint(const double* x, const double* ybar, double* xbar, double* const* opbar,
                 double* coefbar);
};

// ---- the TTN sweep engine ---------------------------------------------
struct EnvD {
    OpP H[2];
    std::map<int, OpP> open;
    bool valid = false;
};

struct Params {
    int Lx = 0, Ly = 0, Lz = 0, bc = QED_BC_OPEN_ZERO_FLUX;
    double t = 1, m = 1, g2e = 1, g2m = 1;
    std::vector<double> mu;   // local chemical potentials, one per site (empty: none)
    double nu_max = 10.0;
    int n_lin = 0, n_quad = 0;
    int pen_adaptive = 0;   // adaptive switch from linear to quadratic growth
    int Q = 0, chi = 16;
    int lz_steps = 30, lz_cycles = 1;
    double lz_tol = 0.0;
    double lz_tol0 = 0.0, lz_factor = 0.1;   // per-sweep tolerance schedule (off: tol0 = 0)
    int dtype = QED_FP64, refine = 1;
    // subspace expansion (off unless set): mixing alpha, columns added per
    // sector delta, bond-dimension cap chi_max, seed of the random maps
    bool exp_on = false;
    double exp_alpha = 0.0;
    int exp_delta = 0, exp_chimax = 0;
    uint64_t exp_seed = 0;
    bool have_lattice = false, have_couplings = false;
};

struct Engine {
    Ctx* ctx = nullptr;
    Model model;
    Tree tree;
    std::vector<Leg> legs;
    std::vector<Leg> alloc_legs;   // legs of the allocation rule (restored by init)
    std::vector<TensorD> nodes;
    std::vector<EnvD> up, dn;
    std::vector<std::vector<OpP>> siteops;   // per site, per op id
    std::vector<std::vector<char>> inside;   // per link: site membership
    std::vector<std::vector<int>> tsites;    // per term: its sites
    int centre = -1;
    int sweeps_done = 0;
    std::vector<double> sweep_energies;   // energy of every sweep of this run
    bool isometric = false;   // every non-root node is an isometry toward the root
    double energy = 0.0;
    bool have_energy = false;
    Arena ws, ws64;   // plan workspaces (ws64: the FP64 plan of a reduced-precision update)
    LanczosWS lws;
    long long matvecs = 0;
    double flops = 0.0;
    int last_updated = -1;     // node updated since the centre last moved, or -1
    long long n_expand = 0;    // expansion moves so far (stream of the random maps)
    double cur_nu = 0.0;       // penalty of the current sweep

    void build(Ctx* c);
    void init_nodes(uint64_t seed);
    bool ready() const { return !nodes.empty(); }
    void invalidate() {
        centre = -1;
        isometric = false;
    }
    void prepare();
    void sweep(int s, qed_sweep_report* rep);
    void observables(std::vector<double>& site7);

    double nu_for(int s) const;
    OpP qr_toward(int n, int which);
    void absorb(int n, int e, const OpP& R);
    void move(int a, int b);
    // SVD move with optional subspace expansion (expansion mode)
    void move_svd(int a, int b, bool grow);
    void adopt_legs(const std::vector<Leg>& nl);
    void move_to(int target);
    void build_env(int n, int which, EnvD& out);
    EnvD& env_for(int n, int which);
    double update(int n, double nu, bool refine_here = true);
};

// ---- segmented Lanczos: independent recurrences on segments of one
// concatenated vector (batched node updates) ------------------------------
struct SegLanczos {
    static constexpr int LDS = 72;   // per-segment scalar stride
    static constexpr int LDN = 8;    // per-segment norm slots
    int nseg = 0, nch = 0, m = 0;
    int64_t N = 0;
    bool b32 = false;                // the basis V is stored in FP32
    BufP chunks, seg_c0, V, w, alpha, beta, coef, coef2, sv, work, st, partial, pv, pi, nrm, fac;
    // b32 (an FP32 basis) needs m + 1 <= 32, the rows of the fused passes
    void setup(Dev* dev, const std::vector<int64_t>& seg_off, int64_t N, int m, bool b32);
    // enqueue one cycle on `s` (no host synchronisation: capturable);
    // apply(v, v32, y): y = H v with the basis vector in FP64 (v) or, for an
    // FP32 basis, in FP32 (v32; v null)
    void cycle(const std::function<void(const double*, const float*, double*)>& apply, double* x,
               hipStream_t s);
};

// ---- autotuner of the GEMM tile shape and pipeline per plan stage --------
struct Tuner {
    bool on = false;
    std::string path;
    std::map<std::string, int> cache;
    void load();
    void save() const;
    void tune(Dev* dev, Plan& P, void* ws, void* x, void* y);
};

// ---- batched node-level H_eff -------------------------------------------
struct HeffBatch {
    Ctx* ctx = nullptr;
    int nn = 0;
    std::vector<std::array<Leg, 3>> legs;
    std::vector<BlockTable> tabs;
    std::vector<int64_t> off;      // nn + 1 offsets into the concatenated vector
    std::vector<std::vector<HTerm>> terms;
    Plan plan;
    BufP ws, xc, yc;
    SegLanczos lz;
    hipStream_t stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    double* gx = nullptr;
    int gm = 0;
    void matvec(const double* x, double* y, hipStream_t s);
    // y = H x with x already in the plan's FP32 compute type
    void matvec32(const float* x, double* y, hipStream_t s);
    ~HeffBatch();
};

struct Ctx {
    Dev dev;
    Prof prof;
    Tuner tuner;
    double mv_flops = 0.0;
    long long mv_count = 0;
    bool host_only = true;
    std::string err;
    Params prm;
    std::unique_ptr<Engine> eng;
    bool built = false;
};

}  // namespace qed
