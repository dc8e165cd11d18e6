// HIP kernels of the TTN node update for gfx950 (CDNA4, wave64).
//
//  * k_brgemm: grouped batch-reduce GEMM.  Every contraction of the hot
//    path (H_eff mode products, the term-summed output accumulation, the
//    environment renormalisation) is a list of jobs, each a sum of
//    products of dense symmetry blocks; one workgroup owns one output tile
//    (64x64, 128x32 or 32x128), stages A/B through double-buffered LDS and
//    runs 16x16x4 MFMA on four waves.  FP64 and FP32 instances; FP32
//    accumulates in FP32.  k_sum_stage runs stages of identity products.
//  * FP64 Lanczos vector kernels: multi-row dot products with wave64
//    shuffle reductions in a fixed order (deterministic); the recurrence,
//    both Gram-Schmidt passes and the norm fused with their dot products.
//  * k_tridiag_lowest: lowest eigenpair of the Lanczos tridiagonal
//    (Sturm-count multisection on one wave + inverse iteration with
//    partial pivoting).
//  * k_householder_qr: per-sector blocked Householder QR (compact WY
//    panels in LDS), one workgroup per sector matrix, diag(R) >= 0;
//    k_householder_qr_wide for sectors wider than 256 columns.
#include "kernels.h"
#include "qedttn.h"

namespace qed {

template <typename T> struct Mfma;

// Operand layout of both 16x16x4 instructions: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  The accumulator layout differs:
// FP32 keeps rows 4 (l / 16) + i in item i, FP64 keeps rows 4 i + l / 16.
template <> struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 step(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return 4 * i + (lane >> 4); }
};

template <> struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 step(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// Operand and output blocks of the GEMM kernels live in device (global)
// memory; pointers read from the job lists are generic to the compiler,
// which would emit flat loads, and a flat load also counts against the LDS
// wait counter: every LDS wait of the MFMA loop would then wait for the
// next chunk's operand prefetch too.  resolve() returns the pointer in the
// global address space.
template <typename T>
using gmem = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ gmem<T>* resolve(const GRef& r, const Bases& bs) {
    if (r.tag == TAG_ABS) return (gmem<T>*)r.abs;
    return (gmem<T>*)bs.b[r.tag] + r.off;
}

// word 3 of a raw (untyped, stride 0) buffer resource on gfx9-family
// parts, and a byte offset beyond every resource's range
constexpr int DMA_RSRC_W3 = 0x00020000;
constexpr uint32_t DMA_OOB = 0x80000000u;

// one element through a raw buffer resource; an offset past the resource's
// range reads as zero
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
    return __hiloint2double((int)v.y, (int)v.x);
}
// one element stored through a raw buffer resource; a store past the
// resource's range is dropped
template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ void buf_store<float>(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, 0, 0);
}
template <>
__device__ __forceinline__ void buf_store<double>(double v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const u2 w = {(unsigned)__double2loint(v), (unsigned)__double2hiint(v)};
    __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)off, 0, 0);
}

// ---------------------------------------------------------------------
// grouped batch-reduce GEMM
// ---------------------------------------------------------------------
// Workgroup tile (16 WM BM) x (16 WN BN) on 4 waves in a WM x WN grid;
// every wave owns BM x BN MFMA 16x16 blocks.  K advances in chunks of
// KC = 16 staged k-major in LDS (As[k][m], Bs[k][n]:
// the MFMA operand reads of a wave hit 16 consecutive words).  The LDS
// stage is double-buffered: chunk c + 1 is fetched into registers while
// chunk c is multiplied, then stored into the other buffer, so a chunk
// costs one barrier.  Each thread's element offsets are computed once per
// product; a chunk only adds its k offset.
// An empty asm statement per prefetched operand register (no instruction):
// the values stay untouched until the stage that stores them to LDS, so the
// compiler cannot place their first use, and the wait for their loads,
// before the MFMAs that the prefetch is meant to overlap.
template <typename T, int NA, int NB>
__device__ __forceinline__ void hold_regs(T (&ra)[NA], T (&rb)[NB]) {
#pragma unroll
    for (int e = 0; e < NA; ++e) asm volatile("" : "+v"(ra[e]));
#pragma unroll
    for (int e = 0; e < NB; ++e) asm volatile("" : "+v"(rb[e]));
}

template <typename T> struct GemmK;
template <> struct GemmK<float> { static constexpr int KC = 16; };
template <> struct GemmK<double> { static constexpr int KC = 16; };

// Occupancy hint of five waves per SIMD: the FP32 instances fit in 96 VGPRs
// without spills (four waves otherwise); measured faster on the sweep, the
// batched matvec and the adjoint.
// FLAT selects the flat pipeline (operands and output through buffer
// resources, below); BUF gives the register-staged loop the same buffer
// access (the host sets it where every block fits 2^31-byte offsets).
template <typename T, int WM, int WN, int BM, int BN, bool FLAT, bool BUF>
__global__ __launch_bounds__(256, 5) void k_brgemm(const GJob* __restrict__ jobs,
                                                const GProd* __restrict__ prods,
                                                const GTile* __restrict__ tiles, Bases bases) {
    typedef typename Mfma<T>::v4 v4;
    constexpr int KC = GemmK<T>::KC;
    constexpr int TM = 16 * WM * BM, TN = 16 * WN * BN;
    constexpr int PAD = 4;
    constexpr int AE = TM * KC / 256;   // A elements per thread per chunk
    constexpr int BE = TN * KC / 256;
    __shared__ T As[2][KC][TM + PAD];
    __shared__ T Bs[2][KC][TN + PAD];
    const GTile tl = tiles[blockIdx.x];
    if (tl.job < 0) return;   // padding of the XCD-ordered tile list
    const GJob J = jobs[tl.job];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm0 = (wave / WN) * 16 * BM;
    const int wn0 = (wave % WN) * 16 * BN;
    const int m0 = tl.tm * TM;
    const int n0 = tl.tn * TN;
    const int lr = lane & 15, lk = lane >> 4;
    v4 acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) acc[i][j] = v4{0, 0, 0, 0};
    T ra[AE], rb[BE];
    // every tile extent divides 256, so element e of a thread sits at a
    // fixed stride from its element 0: one base offset per operand
    constexpr int ASA = 256 / KC, ASB = 256 / TM;    // A rows (A^T k) per e
    constexpr int BSB = 256 / KC, BSN = 256 / TN;    // B^T rows (B k) per e
    const int t_kc = tid % KC, t_kq = tid / KC;
    const int t_tm = tid % TM, t_tq = tid / TM;
    const int t_tn = tid % TN, t_nq = tid / TN;
    if constexpr (!FLAT) {
        // one product after the other, each with its own pipeline prologue
        for (int p = J.p0; p < J.p1; ++p) {
            const GProd P = prods[p];
            gmem<const T>* Bb = resolve<T>(P.B, bases) + (int64_t)tl.b * P.bsB;
            const T alpha = (T)P.alpha;
            if (P.ident) {
    #pragma unroll
                for (int bi = 0; bi < BM; ++bi)
    #pragma unroll
                    for (int bj = 0; bj < BN; ++bj) {
                        const int col = n0 + wn0 + bj * 16 + lr;
                        const int64_t co = P.nsb ? (int64_t)(col / P.nsb) * P.nob + col % P.nsb : col;
    #pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int row = m0 + wm0 + bi * 16 + Mfma<T>::row(lane, i);
                            if (row < J.M && col < J.N)
                                acc[bi][bj][i] += alpha * Bb[(int64_t)row * P.ldb + co];
                        }
                    }
                continue;
            }
            gmem<const T>* Ab = resolve<T>(P.A, bases) + (int64_t)tl.b * P.bsA;
            const int nchunk = (P.K + KC - 1) / KC;
            // element e of this thread: A row am0 + e amE, A column (k) ak0 + e akE
            // within the chunk (and likewise for B), one branch-free form for
            // both storage orders
            const int am0 = P.tA ? t_tm : t_kq, amE = P.tA ? 0 : ASA;
            const int ak0 = P.tA ? t_tq : t_kc, akE = P.tA ? ASB : 0;
            const int64_t akm = P.tA ? (int64_t)P.lda : 1;
            const int64_t aes = (int64_t)(P.tA ? ASB : ASA) * P.lda;
            const int64_t abase = P.tA ? (int64_t)ak0 * P.lda + m0 + am0 : (int64_t)(m0 + am0) * P.lda + ak0;
            const int bn0 = P.tB ? t_kq : t_tn, bnE = P.tB ? BSB : 0;
            const int bk0 = P.tB ? t_kc : t_nq, bkE = P.tB ? 0 : BSN;
            const int64_t bkm = P.tB ? 1 : (int64_t)P.ldb;
            const int64_t bes = (int64_t)(P.tB ? BSB : BSN) * P.ldb;
            int64_t bbase;
            if (P.tB) {
                bbase = (int64_t)(n0 + bn0) * P.ldb + bk0;
            } else {
                const int gn = n0 + bn0;
                const int64_t col = P.nsb ? (int64_t)(gn / P.nsb) * P.nob + gn % P.nsb : gn;
                bbase = (int64_t)bk0 * P.ldb + col;
            }
            for (int r = 0; r < P.nred; ++r) {
                gmem<const T>* A = Ab + (int64_t)r * P.rsA + abase;
                gmem<const T>* B = Bb + (int64_t)r * P.rsB + bbase;
                const __amdgpu_buffer_rsrc_t rsa =
                    __builtin_amdgcn_make_buffer_rsrc((void*)(Ab + (int64_t)r * P.rsA), (short)0, 0x7fffffff, DMA_RSRC_W3);
                const __amdgpu_buffer_rsrc_t rsb =
                    __builtin_amdgcn_make_buffer_rsrc((void*)(Bb + (int64_t)r * P.rsB), (short)0, 0x7fffffff, DMA_RSRC_W3);
                auto fetch = [&](int c) {
                    const int k0 = c * KC;
                    if constexpr (BUF) {
                        const uint32_t pa = (uint32_t)((abase + k0 * akm) * (int64_t)sizeof(T));
                        const uint32_t pb = (uint32_t)((bbase + k0 * bkm) * (int64_t)sizeof(T));
                        const uint32_t aeb = (uint32_t)(aes * (int64_t)sizeof(T));
                        const uint32_t beb = (uint32_t)(bes * (int64_t)sizeof(T));
    #pragma unroll
                        for (int e = 0; e < AE; ++e) {
                            const bool ok = (m0 + am0 + e * amE < J.M) & (k0 + ak0 + e * akE < P.K);
                            ra[e] = buf_load<T>(rsa, ok ? pa + (uint32_t)e * aeb : DMA_OOB);
                        }
    #pragma unroll
                        for (int e = 0; e < BE; ++e) {
                            const bool ok = (n0 + bn0 + e * bnE < J.N) & (k0 + bk0 + e * bkE < P.K);
                            rb[e] = buf_load<T>(rsb, ok ? pb + (uint32_t)e * beb : DMA_OOB);
                        }
                    } else {
                        gmem<const T>* pa = A + k0 * akm;
                        gmem<const T>* pb = B + k0 * bkm;
    #pragma unroll
                        for (int e = 0; e < AE; ++e) {
                            T v = (T)0;
                            if (m0 + am0 + e * amE < J.M && k0 + ak0 + e * akE < P.K) v = pa[e * aes];
                            ra[e] = v;
                        }
    #pragma unroll
                        for (int e = 0; e < BE; ++e) {
                            T v = (T)0;
                            if (n0 + bn0 + e * bnE < J.N && k0 + bk0 + e * bkE < P.K) v = pb[e * bes];
                            rb[e] = v;
                        }
                    }
                };
                // alpha is applied here, not at the load: a use right after
                // the load would make the prefetch wait before the MFMAs
                auto stash = [&](int buf) {
                    hold_regs(ra, rb);
    #pragma unroll
                    for (int e = 0; e < AE; ++e) As[buf][ak0 + e * akE][am0 + e * amE] = ra[e] * alpha;
    #pragma unroll
                    for (int e = 0; e < BE; ++e) Bs[buf][bk0 + e * bkE][bn0 + e * bnE] = rb[e];
                };
                // the previous product's last chunk may still be read from
                // buffer 0 by other waves
                __syncthreads();
                fetch(0);
                stash(0);
                __syncthreads();
                for (int c = 0; c < nchunk; ++c) {
                    const int cur = c & 1;
                    if (c + 1 < nchunk) fetch(c + 1);
    #pragma unroll
                    for (int kk = 0; kk < KC; kk += 4) {
                        T a[BM], bb[BN];
    #pragma unroll
                        for (int i = 0; i < BM; ++i) a[i] = As[cur][kk + lk][wm0 + i * 16 + lr];
    #pragma unroll
                        for (int j = 0; j < BN; ++j) bb[j] = Bs[cur][kk + lk][wn0 + j * 16 + lr];
    #pragma unroll
                        for (int i = 0; i < BM; ++i)
    #pragma unroll
                            for (int j = 0; j < BN; ++j) acc[i][j] = Mfma<T>::step(a[i], bb[j], acc[i][j]);
                    }
                    if (c + 1 < nchunk) stash(cur ^ 1);
                    __syncthreads();
                }
            }
        }
    } else {
        // identity products first (they need no LDS stage)
        for (int p = J.p0; p < J.p1; ++p) {
            const GProd P = prods[p];
            if (!P.ident) continue;
            gmem<const T>* Bb = resolve<T>(P.B, bases) + (int64_t)tl.b * P.bsB;
            const T alpha = (T)P.alpha;
    #pragma unroll
            for (int bi = 0; bi < BM; ++bi)
    #pragma unroll
                for (int bj = 0; bj < BN; ++bj) {
                    const int col = n0 + wn0 + bj * 16 + lr;
                    const int64_t co = P.nsb ? (int64_t)(col / P.nsb) * P.nob + col % P.nsb : col;
    #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = m0 + wm0 + bi * 16 + Mfma<T>::row(lane, i);
                        if (row < J.M && col < J.N) acc[bi][bj][i] += alpha * Bb[(int64_t)row * P.ldb + co];
                    }
                }
        }
        // The other products run as one flat sequence of (product, reduction,
        // chunk) steps: the next step's operands are fetched while the current
        // chunk is multiplied, also across product boundaries.
        // Operands are read through raw buffer resources over the product's
        // blocks, an element outside the tile's range at the out-of-range
        // offset (read as zero): every load is issued unconditionally, with
        // no branch around it (the host routes here only products whose
        // operands span less than 2^31 bytes).
        struct Step {
            __amdgpu_buffer_rsrc_t ra, rb;
            uint32_t ao, bo;            // byte offset of this thread's element 0 at k0 = 0
            uint32_t akb, aeb, bkb, beb;   // bytes per k and per element index e
            int am0, amE, ak0, akE, bn0, bnE, bk0, bkE;
            int K, nchunk, nred;
            T alpha;
        };
        auto describe = [&](int p, int r, Step& D) {
            const GProd P = prods[p];
            gmem<const T>* Ab = resolve<T>(P.A, bases) + (int64_t)tl.b * P.bsA;
            gmem<const T>* Bb = resolve<T>(P.B, bases) + (int64_t)tl.b * P.bsB;
            D.am0 = P.tA ? t_tm : t_kq;
            D.amE = P.tA ? 0 : ASA;
            D.ak0 = P.tA ? t_tq : t_kc;
            D.akE = P.tA ? ASB : 0;
            const int64_t akm = P.tA ? (int64_t)P.lda : 1;
            const int64_t aes = (int64_t)(P.tA ? ASB : ASA) * P.lda;
            const int64_t abase =
                P.tA ? (int64_t)D.ak0 * P.lda + m0 + D.am0 : (int64_t)(m0 + D.am0) * P.lda + D.ak0;
            D.bn0 = P.tB ? t_kq : t_tn;
            D.bnE = P.tB ? BSB : 0;
            D.bk0 = P.tB ? t_kc : t_nq;
            D.bkE = P.tB ? 0 : BSN;
            const int64_t bkm = P.tB ? 1 : (int64_t)P.ldb;
            const int64_t bes = (int64_t)(P.tB ? BSB : BSN) * P.ldb;
            int64_t bbase;
            if (P.tB) {
                bbase = (int64_t)(n0 + D.bn0) * P.ldb + D.bk0;
            } else {
                const int gn = n0 + D.bn0;
                const int64_t col = P.nsb ? (int64_t)(gn / P.nsb) * P.nob + gn % P.nsb : gn;
                bbase = (int64_t)D.bk0 * P.ldb + col;
            }
            D.ra = __builtin_amdgcn_make_buffer_rsrc((void*)(Ab + (int64_t)r * P.rsA), (short)0, 0x7fffffff,
                                                     DMA_RSRC_W3);
            D.rb = __builtin_amdgcn_make_buffer_rsrc((void*)(Bb + (int64_t)r * P.rsB), (short)0, 0x7fffffff,
                                                     DMA_RSRC_W3);
            D.ao = (uint32_t)(abase * (int64_t)sizeof(T));
            D.bo = (uint32_t)(bbase * (int64_t)sizeof(T));
            D.akb = (uint32_t)(akm * (int64_t)sizeof(T));
            D.aeb = (uint32_t)(aes * (int64_t)sizeof(T));
            D.bkb = (uint32_t)(bkm * (int64_t)sizeof(T));
            D.beb = (uint32_t)(bes * (int64_t)sizeof(T));
            D.K = P.K;
            D.nchunk = (P.K + KC - 1) / KC;
            D.nred = P.nred;
            D.alpha = (T)P.alpha;
        };
        auto fetch = [&](const Step& D, int c) {
            const int k0 = c * KC;
            const uint32_t pa = D.ao + (uint32_t)k0 * D.akb;
            const uint32_t pb = D.bo + (uint32_t)k0 * D.bkb;
    #pragma unroll
            for (int e = 0; e < AE; ++e) {
                const bool ok = (m0 + D.am0 + e * D.amE < J.M) & (k0 + D.ak0 + e * D.akE < D.K);
                ra[e] = buf_load<T>(D.ra, ok ? pa + (uint32_t)e * D.aeb : DMA_OOB);
            }
    #pragma unroll
            for (int e = 0; e < BE; ++e) {
                const bool ok = (n0 + D.bn0 + e * D.bnE < J.N) & (k0 + D.bk0 + e * D.bkE < D.K);
                rb[e] = buf_load<T>(D.rb, ok ? pb + (uint32_t)e * D.beb : DMA_OOB);
            }
        };
        // alpha is applied here (see the loop pipeline)
        auto stash = [&](const Step& D, int buf) {
            hold_regs(ra, rb);
    #pragma unroll
            for (int e = 0; e < AE; ++e) As[buf][D.ak0 + e * D.akE][D.am0 + e * D.amE] = ra[e] * D.alpha;
    #pragma unroll
            for (int e = 0; e < BE; ++e) Bs[buf][D.bk0 + e * D.bkE][D.bn0 + e * D.bnE] = rb[e];
        };
        auto next_product = [&](int p) {
            while (p < J.p1 && prods[p].ident) ++p;
            return p;
        };
        int p = next_product(J.p0);
        if (p < J.p1) {
            Step D;
            describe(p, 0, D);
            int r = 0, c = 0, cur = 0;
            fetch(D, 0);
            stash(D, 0);
            __syncthreads();
            while (true) {
                int np = p, nr = r, nc = c + 1;
                if (nc >= D.nchunk) {
                    nc = 0;
                    if (++nr >= D.nred) {
                        nr = 0;
                        np = next_product(p + 1);
                    }
                }
                const bool more = np < J.p1;
                // reduction indices of the current chunk (the steps past
                // them would multiply zero padding only)
                const int kv = D.K - c * KC;
                if (more) {
                    if (np != p || nr != r) describe(np, nr, D);
                    fetch(D, nc);
                }
    #pragma unroll
                for (int kk = 0; kk < KC; kk += 4) {
                    if (kk >= kv) break;
                    T a[BM], bb[BN];
    #pragma unroll
                    for (int i = 0; i < BM; ++i) a[i] = As[cur][kk + lk][wm0 + i * 16 + lr];
    #pragma unroll
                    for (int j = 0; j < BN; ++j) bb[j] = Bs[cur][kk + lk][wn0 + j * 16 + lr];
    #pragma unroll
                    for (int i = 0; i < BM; ++i)
    #pragma unroll
                        for (int j = 0; j < BN; ++j) acc[i][j] = Mfma<T>::step(a[i], bb[j], acc[i][j]);
                }
                if (!more) break;
                stash(D, cur ^ 1);
                __syncthreads();
                cur ^= 1;
                p = np;
                r = nr;
                c = nc;
            }
        }
    }
    gmem<T>* C = resolve<T>(J.C, bases) + (int64_t)tl.b * J.bsC;
    if constexpr (FLAT || BUF) {
        // the output through a buffer resource as well: an element outside
        // the job stores to the out-of-range offset, which drops the store
        const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc((void*)C, (short)0, 0x7fffffff,
                                                                            DMA_RSRC_W3);
#pragma unroll
        for (int bi = 0; bi < BM; ++bi)
#pragma unroll
            for (int bj = 0; bj < BN; ++bj) {
                const int col = n0 + wn0 + bj * 16 + lr;
                // unsigned arithmetic: exact wherever the element is in range
                const uint32_t co = J.nsc ? (uint32_t)(col / J.nsc) * (uint32_t)J.noc + (uint32_t)(col % J.nsc)
                                          : (uint32_t)col;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = m0 + wm0 + bi * 16 + Mfma<T>::row(lane, i);
                    const bool ok = (row < J.M) & (col < J.N);
                    const uint32_t o =
                        ok ? ((uint32_t)row * (uint32_t)J.ldc + co) * (uint32_t)sizeof(T) : DMA_OOB;
                    T v = acc[bi][bj][i];
                    if (J.acc) v += buf_load<T>(rc, o);
                    buf_store<T>(v, rc, o);
                }
            }
        return;
    }
#pragma unroll
    for (int bi = 0; bi < BM; ++bi)
#pragma unroll
        for (int bj = 0; bj < BN; ++bj) {
            const int col = n0 + wn0 + bj * 16 + lr;
            const int64_t co = J.nsc ? (int64_t)(col / J.nsc) * J.noc + col % J.nsc : col;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + wm0 + bi * 16 + Mfma<T>::row(lane, i);
                if (row < J.M && col < J.N) {
                    gmem<T>* c = C + (int64_t)row * J.ldc + co;
                    *c = J.acc ? *c + acc[bi][bj][i] : acc[bi][bj][i];
                }
            }
        }
}

// A stage whose products are all identity products: C (+)= sum_p alpha_p
// B_p elementwise, with the same column splits and the same order of
// additions as the GEMM kernel's identity path (so the same results), but
// coalesced: one workgroup per SUM_TILE consecutive elements of a job.
template <typename T>
__global__ __launch_bounds__(256) void k_sum_stage(const GJob* __restrict__ jobs,
                                                   const GProd* __restrict__ prods,
                                                   const GTile* __restrict__ tiles, Bases bases) {
    const GTile tl = tiles[blockIdx.x];
    if (tl.job < 0) return;
    const GJob J = jobs[tl.job];
    const int64_t total = (int64_t)J.M * J.N;
    const int64_t e0 = (int64_t)tl.tm * SUM_TILE;
    const int64_t e1 = e0 + SUM_TILE < total ? e0 + SUM_TILE : total;
    gmem<T>* C = resolve<T>(J.C, bases) + (int64_t)tl.b * J.bsC;
    // output and every input stored densely (no column split, leading
    // dimension N): element e sits at offset e everywhere, and each thread
    // sums SUM_TILE / 256 elements with all their loads issued together
    // (an index past the tile reads the tile's last element and is not
    // stored)
    bool dense = J.nsc == 0 && J.ldc == J.N;
    for (int p = J.p0; p < J.p1 && dense; ++p) dense = prods[p].nsb == 0 && prods[p].ldb == J.N;
    if (dense) {
        constexpr int U = SUM_TILE / 256;
        int64_t ix[U];
        T acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + threadIdx.x + 256 * u;
            ix[u] = e < e1 ? e : e1 - 1;
            acc[u] = (T)0;
        }
        int p = J.p0;
        for (; p + 2 <= J.p1; p += 2) {
            const GProd& P0 = prods[p];
            const GProd& P1 = prods[p + 1];
            gmem<const T>* B0 = resolve<T>(P0.B, bases) + (int64_t)tl.b * P0.bsB;
            gmem<const T>* B1 = resolve<T>(P1.B, bases) + (int64_t)tl.b * P1.bsB;
            T v0[U], v1[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                v0[u] = B0[ix[u]];
                v1[u] = B1[ix[u]];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                acc[u] += (T)P0.alpha * v0[u];
                acc[u] += (T)P1.alpha * v1[u];
            }
        }
        if (p < J.p1) {
            const GProd& P0 = prods[p];
            gmem<const T>* B0 = resolve<T>(P0.B, bases) + (int64_t)tl.b * P0.bsB;
#pragma unroll
            for (int u = 0; u < U; ++u) acc[u] += (T)P0.alpha * B0[ix[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + threadIdx.x + 256 * u;
            if (e < e1) C[e] = J.acc ? C[e] + acc[u] : acc[u];
        }
        return;
    }
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        const int row = (int)(e / J.N), col = (int)(e % J.N);
        T acc = (T)0;
        // four loads in flight, then the additions in product order
        int p = J.p0;
        for (; p + 4 <= J.p1; p += 4) {
            T v[4], al[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const GProd& P = prods[p + u];
                gmem<const T>* Bb = resolve<T>(P.B, bases) + (int64_t)tl.b * P.bsB;
                const int64_t co = P.nsb ? (int64_t)(col / P.nsb) * P.nob + col % P.nsb : col;
                v[u] = Bb[(int64_t)row * P.ldb + co];
                al[u] = (T)P.alpha;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += al[u] * v[u];
        }
        for (; p < J.p1; ++p) {
            const GProd P = prods[p];
            gmem<const T>* Bb = resolve<T>(P.B, bases) + (int64_t)tl.b * P.bsB;
            const int64_t co = P.nsb ? (int64_t)(col / P.nsb) * P.nob + col % P.nsb : col;
            acc += (T)P.alpha * Bb[(int64_t)row * P.ldb + co];
        }
        const int64_t cc = J.nsc ? (int64_t)(col / J.nsc) * J.noc + col % J.nsc : col;
        gmem<T>* c = C + (int64_t)row * J.ldc + cc;
        *c = J.acc ? *c + acc : acc;
    }
}

void launch_sum_stage_bf16(const GJob*, const GProd*, const GTile*, int, const Bases&, hipStream_t);

void launch_sum_stage(int dtype, const GJob* jobs, const GProd* prods, const GTile* tiles, int ntiles,
                      const Bases& bases, hipStream_t st) {
    if (ntiles <= 0) return;
    if (dtype == QED_FP64)
        hipLaunchKernelGGL(k_sum_stage<double>, dim3(ntiles), dim3(256), 0, st, jobs, prods, tiles, bases);
    else if (dtype == QED_FP32)
        hipLaunchKernelGGL(k_sum_stage<float>, dim3(ntiles), dim3(256), 0, st, jobs, prods, tiles, bases);
    else
        launch_sum_stage_bf16(jobs, prods, tiles, ntiles, bases, st);
}

// ---------------------------------------------------------------------
// FP32 grouped batch-reduce GEMM with direct global -> LDS loads
// ---------------------------------------------------------------------
// The same job/product/tile contract as k_brgemm, for stages whose
// products read A row-major along K (tA = 0) and B row-major along N
// (tB = 0): the mode products on the two child legs, with reductions of a
// full child sector (K up to 141).  Operands travel from global memory
// straight into LDS (buffer loads with the LDS destination: each
// instruction fills 64 consecutive LDS words, lane by lane), NS chunks of
// KC = 16 live in an LDS ring, and a chunk is requested NS - 1 chunks
// before it is multiplied, so no registers stage the operands and more of
// the load latency is covered.
// Elements outside the operands (M, N and K tails) are given an offset
// beyond the buffer resource's range, which reads as zero, so every lane
// issues every load and the per-wave count of loads in flight is exact (the
// waits are counted).  The product's coefficient
// multiplies the A operand as it is read from LDS.
// LDS layouts (conflict-free MFMA operand reads):
//   A: element (m, k) at (m / 4) 66 + (m % 4) 16 + (k ^ (8 [m % 4 >= 2]));
//      one load instruction fills 4 rows of 16 k;
//   B: element (k, n) at k (TN + 16) + n; one instruction fills 64 n of a row.
template <int N> struct VmWait {
    // s_waitcnt with vmcnt(N) only (expcnt and lgkmcnt left unconstrained)
    static constexpr int imm = (N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8);
};

#define QED_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

template <int WM, int WN, int BM, int BN, int NS>
__global__ __launch_bounds__(256, 4) void k_brgemm_dma(const GJob* __restrict__ jobs,
                                                     const GProd* __restrict__ prods,
                                                     const GTile* __restrict__ tiles, Bases bases) {
    typedef Mfma<float>::v4 v4;
    constexpr int KC = 16;
    constexpr int TM = 16 * WM * BM, TN = 16 * WN * BN;
    static_assert(TN % 64 == 0 && TM % 16 == 0, "tile shape");
    constexpr int A_SLOT = (TM / 4) * 66;
    constexpr int LDB = TN + 16;
    constexpr int B_SLOT = KC * LDB;
    constexpr int SLOT = A_SLOT + B_SLOT;
    constexpr int IA = TM / 16;          // A load instructions per wave and chunk
    constexpr int IB = TN / 16;          // B load instructions per wave and chunk
    constexpr int V = IA + IB;
    constexpr int D = NS - 1;            // chunks requested ahead
    __shared__ float lds[NS * SLOT];
    const GTile tl = tiles[blockIdx.x];
    if (tl.job < 0) return;
    const GJob J = jobs[tl.job];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm0 = (wave / WN) * 16 * BM;
    const int wn0 = (wave % WN) * 16 * BN;
    const int m0 = tl.tm * TM;
    const int n0 = tl.tn * TN;
    const int lr = lane & 15, lk = lane >> 4;
    v4 acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) acc[i][j] = v4{0, 0, 0, 0};
    // this lane's element of each of its load instructions: A instruction
    // j covers rows 4 q .. 4 q + 3 (q = wave IA + j); B instruction j is row
    // t / (TN / 64), segment t % (TN / 64) (t = wave IB + j)
    const int ar = lane >> 4;
    const int ak = (lane & 15) ^ ((ar & 2) << 2);
    // MFMA operand words: A row (wm0 + i 16 + lr), B column (wn0 + j 16 + lr)
    int aw[BM];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
        const int m = wm0 + i * 16 + lr;
        aw[i] = (m >> 2) * 66 + (m & 3) * 16;
    }
    const int sw = ((lr & 2) << 2);       // the A swizzle of row m (m % 4 = lr % 4)
    for (int p = J.p0; p < J.p1; ++p) {
        const GProd P = prods[p];
        gmem<const float>* Bb = resolve<float>(P.B, bases) + (int64_t)tl.b * P.bsB;
        if (P.ident) {
            const float alpha = (float)P.alpha;
#pragma unroll
            for (int bi = 0; bi < BM; ++bi)
#pragma unroll
                for (int bj = 0; bj < BN; ++bj) {
                    const int col = n0 + wn0 + bj * 16 + lr;
                    const int64_t co = P.nsb ? (int64_t)(col / P.nsb) * P.nob + col % P.nsb : col;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = m0 + wm0 + bi * 16 + Mfma<float>::row(lane, i);
                        if (row < J.M && col < J.N) acc[bi][bj][i] += alpha * Bb[(int64_t)row * P.ldb + co];
                    }
                }
            continue;
        }
        const float* Ab = (const float*)(resolve<float>(P.A, bases) + (int64_t)tl.b * P.bsA);
        const float alpha = (float)P.alpha;
        const int nchunk = (P.K + KC - 1) / KC;
        // B instruction j of this wave: row wave IB / HS + j / HS of the
        // chunk, 64-column segment j % HS (IB is a multiple of HS).  Byte
        // offsets relative to the chunk's first row (B) or column (A) are
        // fixed for the product; a chunk adds its k0 to them.
        constexpr int HS = TN / 64;
        const int brow0 = wave * (IB / HS);
        uint32_t boff[IB];
        bool bok[IB];
#pragma unroll
        for (int j = 0; j < IB; ++j) {
            const int n = n0 + (j % HS) * 64 + lane;
            const int row = brow0 + j / HS;
            bok[j] = n < J.N;
            const int co = P.nsb ? (n / P.nsb) * (int)P.nob + n % P.nsb : n;
            boff[j] = 4u * (uint32_t)(row * P.ldb + co);
        }
        // A instruction j of this wave: row am + 4 j (this lane's row)
        const int am = m0 + 4 * wave * IA + ar;
        uint32_t aoff[IA];
        bool aok[IA];
#pragma unroll
        for (int j = 0; j < IA; ++j) {
            aok[j] = am + 4 * j < J.M;
            aoff[j] = 4u * (uint32_t)((am + 4 * j) * P.lda + ak);
        }
        for (int r = 0; r < P.nred; ++r) {
            // raw buffer resources over the operands; an offset of 2^31 is
            // outside every operand (the host routes no product whose
            // operand spans 2^31 bytes here) and reads as zero
            const __amdgpu_buffer_rsrc_t ra =
                __builtin_amdgcn_make_buffer_rsrc((void*)(Ab + (int64_t)r * P.rsA), (short)0, 0x7fffffff, DMA_RSRC_W3);
            const __amdgpu_buffer_rsrc_t rb =
                __builtin_amdgcn_make_buffer_rsrc((void*)(Bb + (int64_t)r * P.rsB), (short)0, 0x7fffffff, DMA_RSRC_W3);
            // request chunk c into ring slot c % NS
            auto issue = [&](int c) {
                float* slot = lds + (c % NS) * SLOT;
                const int k0 = c * KC;
                const bool kin = k0 + ak < P.K;
#pragma unroll
                for (int j = 0; j < IA; ++j) {
                    const uint32_t o = (aok[j] && kin) ? aoff[j] + 4u * (uint32_t)k0 : DMA_OOB;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, QED_LDS_PTR(slot + (wave * IA + j) * 66), 4, o, 0, 0,
                                                             0);
                }
                const uint32_t kb = 4u * (uint32_t)(k0 * P.ldb);
#pragma unroll
                for (int j = 0; j < IB; ++j) {
                    const int row = brow0 + j / HS, h = j % HS;
                    const uint32_t o = (bok[j] && k0 + row < P.K) ? boff[j] + kb : DMA_OOB;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, QED_LDS_PTR(slot + A_SLOT + row * LDB + h * 64), 4, o,
                                                             0, 0, 0);
                }
            };
            // the previous product's last chunks may still be read from the
            // ring by other waves
            __syncthreads();
#pragma unroll
            for (int c = 0; c < D; ++c)
                if (c < nchunk) issue(c);
            for (int c = 0; c < nchunk; ++c) {
                // chunk c complete for this wave: the loads requested after
                // it (at most D - 1 chunks) may still be in flight
                const int after = nchunk - 1 - c < D - 1 ? nchunk - 1 - c : D - 1;
                if (after >= 2) __builtin_amdgcn_s_waitcnt(VmWait<2 * V>::imm);
                else if (after == 1) __builtin_amdgcn_s_waitcnt(VmWait<V>::imm);
                else __builtin_amdgcn_s_waitcnt(VmWait<0>::imm);
                __builtin_amdgcn_s_barrier();
                // every wave is past chunk c - 1: its slot takes chunk c + D
                if (c + D < nchunk) issue(c + D);
                const float* As = lds + (c % NS) * SLOT;
                const float* Bs = As + A_SLOT;
#pragma unroll
                for (int kk = 0; kk < KC; kk += 4) {
                    float a[BM], bb[BN];
                    const int k = kk + lk;
#pragma unroll
                    for (int i = 0; i < BM; ++i) a[i] = As[aw[i] + (k ^ sw)] * alpha;
#pragma unroll
                    for (int j = 0; j < BN; ++j) bb[j] = Bs[k * LDB + wn0 + j * 16 + lr];
#pragma unroll
                    for (int i = 0; i < BM; ++i)
#pragma unroll
                        for (int j = 0; j < BN; ++j) acc[i][j] = Mfma<float>::step(a[i], bb[j], acc[i][j]);
                }
            }
        }
    }
    // the output through a buffer resource: an element outside the job
    // stores to the out-of-range offset, which drops the store
    gmem<float>* C = resolve<float>(J.C, bases) + (int64_t)tl.b * J.bsC;
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc((void*)C, (short)0, 0x7fffffff, DMA_RSRC_W3);
#pragma unroll
    for (int bi = 0; bi < BM; ++bi)
#pragma unroll
        for (int bj = 0; bj < BN; ++bj) {
            const int col = n0 + wn0 + bj * 16 + lr;
            // unsigned arithmetic: exact wherever the element is in range
            const uint32_t co = J.nsc ? (uint32_t)(col / J.nsc) * (uint32_t)J.noc + (uint32_t)(col % J.nsc)
                                      : (uint32_t)col;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + wm0 + bi * 16 + Mfma<float>::row(lane, i);
                const bool ok = (row < J.M) & (col < J.N);
                const uint32_t o = ok ? ((uint32_t)row * (uint32_t)J.ldc + co) * 4u : DMA_OOB;
                float v = acc[bi][bj][i];
                if (J.acc) v += buf_load<float>(rc, o);
                buf_store<float>(v, rc, o);
            }
        }
}

// Skinny products: every product of the stage is A B^T with A the
// contiguous M x K panel of a block (lda = K, tA = 0), B an N x K operator
// block (ldb = K, tB = 1), K <= 64 and N <= 64, summed into a contiguous
// M x N output (ldc = N, overwritten).  This is the mode product on the
// parent leg: long M, short K and N, so the output written dominates.  A
// strip of SK_RS(T) rows and the whole output width is one unit of work:
// its output is one contiguous range of memory, staged through LDS and
// stored fully coalesced, once.  The kernel is persistent: workgroup w
// walks strips w, w + G, w + 2G, ... (G a multiple of 8, so a workgroup
// stays on the XCD the strip order assigns), and the operands of its next
// product, of this strip or the next, are fetched into registers while the
// current one is multiplied and its output stored, so the load latency of
// one strip hides behind the work of the previous one.  The MFMA column
// blocks are a compile-time count per job.  The order of the sums (k
// ascending in steps of 4, products in order) is the block GEMM's.
template <typename T> struct SkinnyRows;
template <> struct SkinnyRows<float> { static constexpr int BMR = 2; };
template <> struct SkinnyRows<double> { static constexpr int BMR = 1; };

template <typename T>
struct SkinnyRegs {
    static constexpr int RS = 64 * SkinnyRows<T>::BMR;
    static constexpr int UA = RS * SK_KMAX / 256, UB = SK_NMAX * SK_KMAX / 256;
    T ra[UA], rb[UB];
};

// operands of product p of job J for the strip at row m0 into registers;
// element e of the padded strip is (r, k) = (e / Kp, e % Kp), r = e / Kp
// exact in float for e < 2^13 (e + 1/2 is at least 1/(2 Kp) away from a
// multiple of Kp)
template <typename T>
__device__ __forceinline__ void skinny_fetch(SkinnyRegs<T>& R, const GJob& J, const GProd& P, int m0,
                                             const Bases& bases) {
    constexpr int RS = SkinnyRegs<T>::RS;
    const int tid = threadIdx.x;
    const int K = P.K, Kp = (K + 3) & ~3;
    const int rows = min(RS, J.M - m0);
    const float inv = 1.0f / (float)Kp;
    gmem<const T>* A = resolve<T>(P.A, bases) + (int64_t)m0 * K;
    gmem<const T>* B = resolve<T>(P.B, bases);
#pragma unroll
    for (int u = 0; u < SkinnyRegs<T>::UA; ++u) {
        const int e = tid + 256 * u;
        const int r = (int)(((float)e + 0.5f) * inv), k = e - r * Kp;
        R.ra[u] = (e < RS * Kp && r < rows && k < K) ? A[r * K + k] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < SkinnyRegs<T>::UB; ++u) {
        const int e = tid + 256 * u;
        const int n = (int)(((float)e + 0.5f) * inv), k = e - n * Kp;
        R.rb[u] = (e < SK_NMAX * Kp && n < J.N && k < K) ? B[n * K + k] : (T)0;
    }
}

template <typename T>
__device__ __forceinline__ void skinny_stash(const SkinnyRegs<T>& R, int K, T* As, T* Bs) {
    constexpr int RS = SkinnyRegs<T>::RS, LDA = SK_KMAX + 1;
    const int tid = threadIdx.x;
    const int Kp = (K + 3) & ~3;
    const float inv = 1.0f / (float)Kp;
#pragma unroll
    for (int u = 0; u < SkinnyRegs<T>::UA; ++u) {
        const int e = tid + 256 * u;
        const int r = (int)(((float)e + 0.5f) * inv), k = e - r * Kp;
        if (e < RS * Kp) As[r * LDA + k] = R.ra[u];
    }
#pragma unroll
    for (int u = 0; u < SkinnyRegs<T>::UB; ++u) {
        const int e = tid + 256 * u;
        const int n = (int)(((float)e + 0.5f) * inv), k = e - n * Kp;
        if (e < SK_NMAX * Kp) Bs[n * LDA + k] = R.rb[u];
    }
}

// one strip of job J; on return the registers hold the operands of the
// next strip's first product (job Jn at row mn), if there is one
template <typename T, int NB>
__device__ __forceinline__ void skinny_strip(const GJob& J, int m0, const GProd* __restrict__ prods,
                                             const Bases& bases, SkinnyRegs<T>& R, bool has_next,
                                             const GJob& Jn, int mn, T* As, T* Bs) {
    typedef typename Mfma<T>::v4 v4;
    constexpr int BMR = SkinnyRows<T>::BMR;
    constexpr int LDA = SK_KMAX + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    v4 acc[BMR][NB];
#pragma unroll
    for (int i = 0; i < BMR; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = v4{0, 0, 0, 0};
    for (int p = J.p0; p < J.p1; ++p) {
        const GProd P = prods[p];
        __syncthreads();   // the LDS stage is no longer read (previous product or output strip)
        skinny_stash<T>(R, P.K, As, Bs);
        __syncthreads();
        if (p + 1 < J.p1) skinny_fetch<T>(R, J, prods[p + 1], m0, bases);
        else if (has_next) skinny_fetch<T>(R, Jn, prods[Jn.p0], mn, bases);
        const int Kp = (P.K + 3) & ~3;
        const T alpha = (T)P.alpha;
        for (int kk = 0; kk < Kp; kk += 4) {
            const int k = kk + lk;
            T a[BMR], b[NB];
#pragma unroll
            for (int i = 0; i < BMR; ++i) a[i] = As[(wave * 16 * BMR + i * 16 + lr) * LDA + k] * alpha;
#pragma unroll
            for (int j = 0; j < NB; ++j) b[j] = Bs[(j * 16 + lr) * LDA + k];
#pragma unroll
            for (int i = 0; i < BMR; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[i][j] = Mfma<T>::step(a[i], b[j], acc[i][j]);
        }
    }
    // the output strip through LDS (it fits in the A stage), then stored as
    // one contiguous range
    __syncthreads();
    T* Cs = As;
    const int N = J.N;
#pragma unroll
    for (int i = 0; i < BMR; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int col = j * 16 + lr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = wave * 16 * BMR + i * 16 + Mfma<T>::row(lane, e);
                if (col < N) Cs[row * N + col] = acc[i][j][e];
            }
        }
    __syncthreads();
    const int rows = min(64 * BMR, J.M - m0);
    gmem<T>* C = resolve<T>(J.C, bases) + (int64_t)m0 * N;
    const int tot = rows * N;
#pragma unroll 8
    for (int e = tid; e < tot; e += 256) C[e] = Cs[e];
}

template <typename T>
__global__ __launch_bounds__(256) void k_skinny(const GJob* __restrict__ jobs, const GProd* __restrict__ prods,
                                                const GTile* __restrict__ tiles, int ntiles, Bases bases) {
    constexpr int RS = SkinnyRegs<T>::RS, LDA = SK_KMAX + 1;
    __shared__ T As[RS * LDA];
    __shared__ T Bs[SK_NMAX * LDA];
    const int G = gridDim.x;
    auto next_real = [&](int i) {
        while (i < ntiles && tiles[i].job < 0) i += G;
        return i;
    };
    int i = next_real(blockIdx.x);
    if (i >= ntiles) return;
    SkinnyRegs<T> R;
    {
        const GJob J0 = jobs[tiles[i].job];
        skinny_fetch<T>(R, J0, prods[J0.p0], tiles[i].tm * RS, bases);
    }
    while (i < ntiles) {
        const GTile tl = tiles[i];
        const GJob J = jobs[tl.job];
        const int in = next_real(i + G);
        const bool has_next = in < ntiles;
        const GJob Jn = jobs[has_next ? tiles[in].job : tl.job];
        const int mn = has_next ? tiles[in].tm * RS : 0;
        const int m0 = tl.tm * RS;
        switch ((J.N + 15) >> 4) {
            case 1: skinny_strip<T, 1>(J, m0, prods, bases, R, has_next, Jn, mn, As, Bs); break;
            case 2: skinny_strip<T, 2>(J, m0, prods, bases, R, has_next, Jn, mn, As, Bs); break;
            case 3: skinny_strip<T, 3>(J, m0, prods, bases, R, has_next, Jn, mn, As, Bs); break;
            default: skinny_strip<T, 4>(J, m0, prods, bases, R, has_next, Jn, mn, As, Bs); break;
        }
        i = in;
    }
}

int skinny_rows(int dtype) { return dtype == QED_FP64 ? 64 * SkinnyRows<double>::BMR : 64 * SkinnyRows<float>::BMR; }

// workgroups of a persistent skinny launch: as many as are resident at once
// (the occupancy of the kernel on this device, queried once), a multiple
// of 8, so that no workgroup starts after another has finished its list
template <typename T>
void launch_skinny(const GJob* jobs, const GProd* prods, const GTile* tiles, int ntiles, const Bases& bases,
                   hipStream_t st) {
    if (ntiles <= 0) return;
    static const int resident = [] {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_skinny<T>, 256, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 8)
            cus = 8;
        return per_cu * cus;
    }();
    int g = std::min(ntiles, resident);
    g = std::max(8, g & ~7);
    hipLaunchKernelGGL(k_skinny<T>, dim3(g), dim3(256), 0, st, jobs, prods, tiles, ntiles, bases);
}
template void launch_skinny<float>(const GJob*, const GProd*, const GTile*, int, const Bases&, hipStream_t);
template void launch_skinny<double>(const GJob*, const GProd*, const GTile*, int, const Bases&, hipStream_t);

// FP64 instance of the LDS-DMA ring (same contract and pipeline as
// k_brgemm_dma): every double travels as two 4-byte buffer-to-LDS loads,
// so each lane addresses exactly one half of one element (the middle-leg
// products split their columns at odd strides, so two adjacent doubles
// need not be adjacent in memory).  LDS layouts, in doubles:
//   A: element (m, k) at (m / 2) 34 + (m % 2) 16 + k; one instruction fills
//      two rows of 16 k (64 words) and the pad of 2 doubles per row pair
//      spreads the 16 rows an MFMA operand read touches over the banks;
//   B: element (k, n) at k (TN + 16) + n; one instruction fills 32 n of a
//      row.
template <int WM, int WN, int BM, int BN, int NS>
__global__ __launch_bounds__(256, 2) void k_brgemm_dma64(const GJob* __restrict__ jobs,
                                                       const GProd* __restrict__ prods,
                                                       const GTile* __restrict__ tiles, Bases bases) {
    typedef Mfma<double>::v4 v4;
    constexpr int KC = 16;
    constexpr int TM = 16 * WM * BM, TN = 16 * WN * BN;
    static_assert(TN % 32 == 0 && TM % 8 == 0, "tile shape");
    constexpr int A_SLOT = (TM / 2) * 34;
    constexpr int LDB = TN + 16;
    constexpr int B_SLOT = KC * LDB;
    constexpr int SLOT = A_SLOT + B_SLOT;
    constexpr int IA = TM / 8;            // A load instructions per wave and chunk
    constexpr int HS = TN / 32;           // B instructions per row
    constexpr int IB = KC * HS / 4;       // B load instructions per wave and chunk
    constexpr int V = IA + IB;
    constexpr int D = NS - 1;
    __shared__ double lds[NS * SLOT];
    const GTile tl = tiles[blockIdx.x];
    if (tl.job < 0) return;
    const GJob J = jobs[tl.job];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm0 = (wave / WN) * 16 * BM;
    const int wn0 = (wave % WN) * 16 * BN;
    const int m0 = tl.tm * TM;
    const int n0 = tl.tn * TN;
    const int lr = lane & 15, lk = lane >> 4;
    v4 acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) acc[i][j] = v4{0, 0, 0, 0};
    // this lane's word of an A instruction: row pair half (lane / 32), the
    // double lane % 32 / 2 of that row, half lane % 2
    const int ah = lane >> 5, ak = (lane & 31) >> 1, aw = lane & 1;
    int arow[BM];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
        const int m = wm0 + i * 16 + lr;
        arow[i] = (m >> 1) * 34 + (m & 1) * 16;
    }
    for (int p = J.p0; p < J.p1; ++p) {
        const GProd P = prods[p];
        gmem<const double>* Bb = resolve<double>(P.B, bases) + (int64_t)tl.b * P.bsB;
        if (P.ident) {
            const double alpha = P.alpha;
#pragma unroll
            for (int bi = 0; bi < BM; ++bi)
#pragma unroll
                for (int bj = 0; bj < BN; ++bj) {
                    const int col = n0 + wn0 + bj * 16 + lr;
                    const int64_t co = P.nsb ? (int64_t)(col / P.nsb) * P.nob + col % P.nsb : col;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = m0 + wm0 + bi * 16 + Mfma<double>::row(lane, i);
                        if (row < J.M && col < J.N) acc[bi][bj][i] += alpha * Bb[(int64_t)row * P.ldb + co];
                    }
                }
            continue;
        }
        const double* Ab = (const double*)(resolve<double>(P.A, bases) + (int64_t)tl.b * P.bsA);
        const double alpha = P.alpha;
        const int nchunk = (P.K + KC - 1) / KC;
        // byte offsets of this lane's words relative to the chunk's first
        // row (B) or column (A), fixed for the product
        uint32_t boff[IB];
        bool bok[IB];
        const int brow0 = wave * (KC / 4);
#pragma unroll
        for (int j = 0; j < IB; ++j) {
            const int n = n0 + (j % HS) * 32 + (lane >> 1);
            const int row = brow0 + j / HS;
            bok[j] = n < J.N;
            const int co = P.nsb ? (n / P.nsb) * (int)P.nob + n % P.nsb : n;
            boff[j] = 8u * (uint32_t)(row * P.ldb + co) + 4u * (uint32_t)(lane & 1);
        }
        uint32_t aoff[IA];
        bool aok[IA];
#pragma unroll
        for (int j = 0; j < IA; ++j) {
            const int m = m0 + 2 * (wave * IA + j) + ah;
            aok[j] = m < J.M;
            aoff[j] = 8u * (uint32_t)(m * P.lda + ak) + 4u * (uint32_t)aw;
        }
        for (int r = 0; r < P.nred; ++r) {
            const __amdgpu_buffer_rsrc_t ra =
                __builtin_amdgcn_make_buffer_rsrc((void*)(Ab + (int64_t)r * P.rsA), (short)0, 0x7fffffff, DMA_RSRC_W3);
            const __amdgpu_buffer_rsrc_t rb =
                __builtin_amdgcn_make_buffer_rsrc((void*)(Bb + (int64_t)r * P.rsB), (short)0, 0x7fffffff, DMA_RSRC_W3);
            auto issue = [&](int c) {
                double* slot = lds + (c % NS) * SLOT;
                const int k0 = c * KC;
                const bool kin = k0 + ak < P.K;
#pragma unroll
                for (int j = 0; j < IA; ++j) {
                    const uint32_t o = (aok[j] && kin) ? aoff[j] + 8u * (uint32_t)k0 : DMA_OOB;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, QED_LDS_PTR(slot + (wave * IA + j) * 34), 4, o, 0, 0,
                                                             0);
                }
                const uint32_t kb = 8u * (uint32_t)(k0 * P.ldb);
#pragma unroll
                for (int j = 0; j < IB; ++j) {
                    const int row = brow0 + j / HS, h = j % HS;
                    const uint32_t o = (bok[j] && k0 + row < P.K) ? boff[j] + kb : DMA_OOB;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, QED_LDS_PTR(slot + A_SLOT + row * LDB + h * 32), 4, o,
                                                             0, 0, 0);
                }
            };
            __syncthreads();
#pragma unroll
            for (int c = 0; c < D; ++c)
                if (c < nchunk) issue(c);
            for (int c = 0; c < nchunk; ++c) {
                const int after = nchunk - 1 - c < D - 1 ? nchunk - 1 - c : D - 1;
                if (after >= 2) __builtin_amdgcn_s_waitcnt(VmWait<2 * V>::imm);
                else if (after == 1) __builtin_amdgcn_s_waitcnt(VmWait<V>::imm);
                else __builtin_amdgcn_s_waitcnt(VmWait<0>::imm);
                __builtin_amdgcn_s_barrier();
                if (c + D < nchunk) issue(c + D);
                const double* As = lds + (c % NS) * SLOT;
                const double* Bs = As + A_SLOT;
#pragma unroll
                for (int kk = 0; kk < KC; kk += 4) {
                    double a[BM], bb[BN];
                    const int k = kk + lk;
#pragma unroll
                    for (int i = 0; i < BM; ++i) a[i] = As[arow[i] + k] * alpha;
#pragma unroll
                    for (int j = 0; j < BN; ++j) bb[j] = Bs[k * LDB + wn0 + j * 16 + lr];
#pragma unroll
                    for (int i = 0; i < BM; ++i)
#pragma unroll
                        for (int j = 0; j < BN; ++j) acc[i][j] = Mfma<double>::step(a[i], bb[j], acc[i][j]);
                }
            }
        }
    }
    gmem<double>* C = resolve<double>(J.C, bases) + (int64_t)tl.b * J.bsC;
#pragma unroll
    for (int bi = 0; bi < BM; ++bi)
#pragma unroll
        for (int bj = 0; bj < BN; ++bj) {
            const int col = n0 + wn0 + bj * 16 + lr;
            const int64_t co = J.nsc ? (int64_t)(col / J.nsc) * J.noc + col % J.nsc : col;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + wm0 + bi * 16 + Mfma<double>::row(lane, i);
                if (row < J.M && col < J.N) {
                    gmem<double>* c = C + (int64_t)row * J.ldc + co;
                    *c = J.acc ? *c + acc[bi][bj][i] : acc[bi][bj][i];
                }
            }
        }
}

bool brgemm_dma_shape(int shape) { return shape == GEMM_SHAPE_SQUARE || shape == GEMM_SHAPE_WIDE; }

void launch_brgemm_dma64(const GJob* jobs, const GProd* prods, const GTile* tiles, int ntiles,
                         const Bases& bases, int shape, hipStream_t st) {
    if (ntiles <= 0) return;
    if (shape == GEMM_SHAPE_WIDE)
        hipLaunchKernelGGL((k_brgemm_dma64<1, 4, 2, 2, 3>), dim3(ntiles), dim3(256), 0, st, jobs, prods, tiles,
                           bases);
    else
        hipLaunchKernelGGL((k_brgemm_dma64<2, 2, 2, 2, 3>), dim3(ntiles), dim3(256), 0, st, jobs, prods, tiles,
                           bases);
}

void launch_brgemm_dma(const GJob* jobs, const GProd* prods, const GTile* tiles, int ntiles,
                       const Bases& bases, int shape, hipStream_t st) {
    if (ntiles <= 0) return;
    if (shape == GEMM_SHAPE_WIDE)
        hipLaunchKernelGGL((k_brgemm_dma<1, 4, 2, 2, 3>), dim3(ntiles), dim3(256), 0, st, jobs, prods, tiles,
                           bases);
    else
        hipLaunchKernelGGL((k_brgemm_dma<2, 2, 2, 2, 3>), dim3(ntiles), dim3(256), 0, st, jobs, prods, tiles,
                           bases);
}

template <typename T>
void launch_brgemm(const GJob* jobs, const GProd* prods, const GTile* tiles, int ntiles,
                   const Bases& bases, int shape, bool flat, bool buf, hipStream_t st) {
    if (ntiles <= 0) return;
#define QED_LAUNCH(WM, WN, F, B) \
    hipLaunchKernelGGL((k_brgemm<T, WM, WN, 2, 2, F, B>), dim3(ntiles), dim3(256), 0, st, jobs, prods, tiles, bases)
#define QED_LAUNCH3(WM, WN)                 \
    do {                                    \
        if (flat) QED_LAUNCH(WM, WN, true, true);   \
        else if (buf) QED_LAUNCH(WM, WN, false, true); \
        else QED_LAUNCH(WM, WN, false, false);      \
    } while (0)
    switch (shape) {
        case GEMM_SHAPE_TALL: QED_LAUNCH3(4, 1); break;
        case GEMM_SHAPE_WIDE: QED_LAUNCH3(1, 4); break;
        default: QED_LAUNCH3(2, 2);
    }
#undef QED_LAUNCH3
#undef QED_LAUNCH
}

template void launch_brgemm<double>(const GJob*, const GProd*, const GTile*, int, const Bases&, int,
                                    bool, bool, hipStream_t);
template void launch_brgemm<float>(const GJob*, const GProd*, const GTile*, int, const Bases&, int,
                                   bool, bool, hipStream_t);

// ---------------------------------------------------------------------
// element-wise helpers
// ---------------------------------------------------------------------
__global__ void k_fill(double* x, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void k_f64_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

__global__ void k_f32_to_f64(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}

static int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return (int)g;
}

void launch_fill(double* x, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, st, x, n, v);
}
// FP32 copies of several FP64 arrays in one launch, one workgroup per array
// (the same rounding as k_f64_to_f32)
__global__ __launch_bounds__(256) void k_f64_to_f32_segs(const ConvSeg* __restrict__ segs) {
    const ConvSeg S = segs[blockIdx.x];
    float* d = (float*)S.dst;
    for (int64_t i = threadIdx.x; i < S.n; i += 256) d[i] = (float)S.src[i];
}

void launch_f64_to_f32_segs(const ConvSeg* segs, int nseg, hipStream_t st) {
    if (nseg > 0) hipLaunchKernelGGL(k_f64_to_f32_segs, dim3(nseg), dim3(256), 0, st, segs);
}

void launch_f64_to_f32(const double* a, float* b, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(n)), dim3(256), 0, st, a, b, n);
}
void launch_f32_to_f64(const float* a, double* b, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(n)), dim3(256), 0, st, a, b, n);
}

// ---------------------------------------------------------------------
// FP64 reductions (fixed partition and order: bitwise reproducible)
// ---------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

constexpr int DOT_ROWS = 8;

int dot_grid(int64_t n) {
    int64_t g = (n + 1023) / 1024;
    if (g > 512) g = 512;
    if (g < 1) g = 1;
    return (int)g;
}

// partial[r * G + block] = sum over the block's slice of V[r] . w, r < nrows
__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ V, int64_t ldv,
                                                     int nrows, const double* __restrict__ w,
                                                     int64_t n, double* __restrict__ partial,
                                                     const LState* st, int skip_if_broken) {
    if (skip_if_broken && st && st->broken) return;
    __shared__ double sh[DOT_ROWS][4];
    const int G = gridDim.x;
    const int64_t chunk = (n + G - 1) / G;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int r0 = 0; r0 < nrows; r0 += DOT_ROWS) {
        double s[DOT_ROWS];
#pragma unroll
        for (int q = 0; q < DOT_ROWS; ++q) s[q] = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
            const double wi = w[i];
#pragma unroll
            for (int q = 0; q < DOT_ROWS; ++q)
                if (r0 + q < nrows) s[q] += V[(int64_t)(r0 + q) * ldv + i] * wi;
        }
#pragma unroll
        for (int q = 0; q < DOT_ROWS; ++q) {
            double v = wave_sum(s[q]);
            if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x >> 6] = v;
        }
        __syncthreads();
        if (threadIdx.x < DOT_ROWS && r0 + (int)threadIdx.x < nrows) {
            const int q = threadIdx.x;
            partial[(int64_t)(r0 + q) * G + blockIdx.x] = ((sh[q][0] + sh[q][1]) + sh[q][2]) + sh[q][3];
        }
        __syncthreads();
    }
}

// out[r] = sum_b partial[r * G + b]; one workgroup per row, fixed
// strided partition and fixed reduction tree; mode 1: sqrt
__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ partial, int G,
                                                   int nrows, double* __restrict__ out, int mode,
                                                   const LState* st, int skip_if_broken) {
    if (skip_if_broken && st && st->broken) return;
    __shared__ double sh[4];
    const int r = blockIdx.x;
    if (r >= nrows) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < G; b += 256) s += partial[(int64_t)r * G + b];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = ((sh[0] + sh[1]) + sh[2]) + sh[3];
        out[r] = mode == 1 ? sqrt(t) : t;
    }
}

void launch_dots(const double* V, int64_t ldv, int nrows, const double* w, int64_t n,
                 double* partial, double* out, int mode, const LState* st, int skip,
                 hipStream_t stream) {
    const int G = dot_grid(n);
    hipLaunchKernelGGL(k_dot_partial, dim3(G), dim3(256), 0, stream, V, ldv, nrows, w, n, partial,
                       st, skip);
    hipLaunchKernelGGL(k_dot_final, dim3(nrows), dim3(256), 0, stream, partial, G, nrows, out,
                       mode, st, skip);
}

// w = (double) a, and the partials of v . w with the partition and
// reduction of k_dot_partial (one row): the FP32 matvec's conversion and
// the Lanczos alpha dot in one pass, with the same results as the two
// separate kernels
template <typename TV>
__global__ __launch_bounds__(256) void k_f32_to_f64_dot(const float* __restrict__ a,
                                                        double* __restrict__ w,
                                                        const TV* __restrict__ v, int64_t n,
                                                        double* __restrict__ partial,
                                                        const LState* st) {
    if (st->broken) return;
    __shared__ double sh[4];
    const int G = gridDim.x;
    const int64_t chunk = (n + G - 1) / G;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
        const double wi = (double)a[i];
        w[i] = wi;
        s += (double)v[i] * wi;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

template <typename TV>
void launch_f32_to_f64_dot(const float* a, double* w, const TV* v, int64_t n, double* partial,
                           const LState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_f32_to_f64_dot<TV>, dim3(dot_grid(n)), dim3(256), 0, s, a, w, v, n, partial, st);
}
template void launch_f32_to_f64_dot<double>(const float*, double*, const double*, int64_t, double*, const LState*,
                                            hipStream_t);
template void launch_f32_to_f64_dot<float>(const float*, double*, const float*, int64_t, double*, const LState*,
                                           hipStream_t);

void launch_dot_final(const double* partial, int64_t n, int nrows, double* out, int mode,
                      const LState* st, int skip, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_final, dim3(nrows), dim3(256), 0, s, partial, dot_grid(n), nrows, out,
                       mode, st, skip);
}

// ---------------------------------------------------------------------
// Lanczos step kernels (all no-ops once the state has broken down)
// ---------------------------------------------------------------------
// w -= alpha[j] v_j + beta[j-1] v_{j-1}
__global__ void k_lz_three_term(double* __restrict__ w, const double* __restrict__ V, int64_t ldv,
                                int j, const double* __restrict__ alpha,
                                const double* __restrict__ beta, int64_t n, const LState* st) {
    if (st->broken) return;
    const double a = alpha[j];
    const double b = j > 0 ? beta[j - 1] : 0.0;
    const double* vj = V + (int64_t)j * ldv;
    const double* vm = j > 0 ? V + (int64_t)(j - 1) * ldv : nullptr;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double t = a * vj[i];
        if (vm) t += b * vm[i];
        w[i] -= t;
    }
}

// w -= sum_{r < nrows} c[r] V[r]
__global__ void k_lz_subtract(double* __restrict__ w, const double* __restrict__ V, int64_t ldv,
                              int nrows, const double* __restrict__ c, int64_t n,
                              const LState* st) {
    if (st->broken) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double t = 0.0;
        for (int r = 0; r < nrows; ++r) t += c[r] * V[(int64_t)r * ldv + i];
        w[i] -= t;
    }
}

// beta[j] = sqrt(ww); breakdown test against the scale of T
__global__ void k_lz_beta(const double* ww, double* alpha, double* beta, int j, LState* st,
                          double tol) {
    if (st->broken) return;
    double b = sqrt(*ww);
    double scale = 1.0;
    for (int i = 0; i <= j; ++i) scale = fmax(scale, fabs(alpha[i]));
    for (int i = 0; i < j; ++i) scale = fmax(scale, beta[i]);
    if (b <= tol * scale) {
        beta[j] = 0.0;
        st->broken = 1;
        st->k = j + 1;
    } else {
        beta[j] = b;
    }
}

// V[j+1] = w / beta[j]
// (and, with vc, its FP32 copy for the next matvec: the value the separate
// conversion would write)
// (an FP32 basis stores the rounded value itself: the basis vector is then
// exactly the matvec's input)
template <typename TV>
__global__ void k_lz_next(TV* __restrict__ V, int64_t ldv, int j,
                          const double* __restrict__ w, const double* __restrict__ beta,
                          int64_t n, const LState* st, float* __restrict__ vc) {
    if (st->broken) return;
    const double inv = 1.0 / beta[j];
    TV* v = V + (int64_t)(j + 1) * ldv;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double t = w[i] * inv;
        v[i] = (TV)t;
        if (vc) vc[i] = (float)t;
    }
}

// dst = src / *nrm  (start vector); records the norm
template <typename TV>
__global__ void k_lz_start(TV* __restrict__ dst, const double* __restrict__ src,
                           const double* nrm, int64_t n, LState* st, int m) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->broken = 0;
        st->k = m;
        st->norm = *nrm;
    }
    const double inv = 1.0 / *nrm;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (TV)(src[i] * inv);
}

// lowest eigenpair of the k x k tridiagonal (alpha, beta): Sturm-count
// multisection on one wave (64 shifts per round, the interval shrinks 65x),
// to full precision, then inverse iteration with a pivoted tridiagonal LU
// by lane 0.  Writes s[0..k), st->theta and st->resid.
// alpha, beta, the LU factors and the vector live in LDS (k <= 64): the
// serial steps below read no global memory
__global__ void k_tridiag_lowest(const double* alpha_g, const double* beta_g, double* s_g, LState* st,
                                 double* work) {
    (void)work;
    if (blockIdx.x != 0) return;
    __shared__ double alpha[64], beta[64], dl[64], dd[64], du[64], du2[64], s[64];
    __shared__ int piv[64];
    const int lane = threadIdx.x;
    const int k = st->k;
    if (lane < k) {
        alpha[lane] = alpha_g[lane];
        beta[lane] = beta_g[lane];
    }
    __syncthreads();
    double lo = 0.0, hi = 0.0, tnorm = 0.0;
    for (int i = 0; i < k; ++i) {
        double r = (i > 0 ? fabs(beta[i - 1]) : 0.0) + (i < k - 1 ? fabs(beta[i]) : 0.0);
        double a = alpha[i] - r, b = alpha[i] + r;
        if (i == 0 || a < lo) lo = a;
        if (i == 0 || b > hi) hi = b;
        tnorm = fmax(tnorm, fabs(alpha[i]) + r);
    }
    const double tiny = 1e-300;
    // invariant: no eigenvalue below lo, at least one below hi
    for (int it = 0; it < 64; ++it) {
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        int cnt = 0;
        double d = alpha[0] - x;
        if (d == 0.0) d = -tiny;
        if (d < 0) ++cnt;
        for (int i = 1; i < k; ++i) {
            d = alpha[i] - x - beta[i - 1] * beta[i - 1] / d;
            if (d == 0.0) d = -tiny;
            if (d < 0) ++cnt;
        }
        // the first shift with an eigenvalue below it bounds the lowest one
        const unsigned long long m = __ballot(cnt >= 1 && x > lo && x <= hi);
        const int f = m ? __ffsll((long long)m) - 1 : 64;
        const double nhi = f < 64 ? __shfl(x, f, 64) : hi;
        const double nlo = f > 0 ? __shfl(x, f - 1 < 64 ? f - 1 : 63, 64) : lo;
        const double lo2 = (f > 0 && f <= 64 && nlo > lo && nlo < nhi) ? nlo : lo;
        if (nhi >= hi && lo2 <= lo) break;   // no representable progress
        lo = lo2;
        hi = nhi;
    }
    if (lane != 0) return;
    const double theta = 0.5 * (lo + hi);
    // inverse iteration on (T - theta I)
    for (int i = 0; i < k; ++i) s[i] = 1.0;
    const double eps = 2.3e-16 * (tnorm > 0 ? tnorm : 1.0);
    for (int iter = 0; iter < 3; ++iter) {
        for (int i = 0; i < k; ++i) {
            dd[i] = alpha[i] - theta;
            if (i < k - 1) { dl[i] = beta[i]; du[i] = beta[i]; }
            du2[i] = 0.0;
            piv[i] = i;
        }
        for (int i = 0; i < k - 1; ++i) {
            if (fabs(dd[i]) >= fabs(dl[i])) {
                if (dd[i] == 0.0) dd[i] = eps;
                double f = dl[i] / dd[i];
                dl[i] = f;
                dd[i + 1] -= f * du[i];
            } else {
                double f = dd[i] / dl[i];
                dd[i] = dl[i];
                dl[i] = f;
                double tmp = du[i];
                du[i] = dd[i + 1];
                dd[i + 1] = tmp - f * dd[i + 1];
                if (i < k - 2) {
                    du2[i] = du[i + 1];
                    du[i + 1] = -f * du[i + 1];
                }
                piv[i] = i + 1;
            }
        }
        if (dd[k - 1] == 0.0) dd[k - 1] = eps;
        for (int i = 0; i < k - 1; ++i) {
            if (piv[i] == i) {
                s[i + 1] -= dl[i] * s[i];
            } else {
                double tmp = s[i];
                s[i] = s[i + 1];
                s[i + 1] = tmp - dl[i] * s[i];
            }
        }
        s[k - 1] /= dd[k - 1];
        if (k > 1) s[k - 2] = (s[k - 2] - du[k - 2] * s[k - 1]) / dd[k - 2];
        for (int i = k - 3; i >= 0; --i) s[i] = (s[i] - du[i] * s[i + 1] - du2[i] * s[i + 2]) / dd[i];
        double nrm = 0.0;
        for (int i = 0; i < k; ++i) nrm += s[i] * s[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < k; ++i) s[i] /= nrm;
    }
    for (int i = 0; i < k; ++i) s_g[i] = s[i];
    st->theta = theta;
    st->resid = fabs(beta[k - 1] * s[k - 1]);
}

// u = sum_{r < k} s[r] V[r]
template <typename TV>
__global__ void k_ritz(double* __restrict__ u, const TV* __restrict__ V, int64_t ldv,
                       const double* __restrict__ s, int64_t n, const LState* st) {
    const int k = st->k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double t = 0.0;
        for (int r = 0; r < k; ++r) t += s[r] * (double)V[(int64_t)r * ldv + i];
        u[i] = t;
    }
}

// per block: largest |u| and its first index
__global__ __launch_bounds__(256) void k_argmax_partial(const double* __restrict__ u, int64_t n,
                                                        double* pv, int64_t* pi) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    const int G = gridDim.x;
    const int64_t chunk = (n + G - 1) / G;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    double bv = -1.0;
    int64_t bi = -1;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
        double a = fabs(u[i]);
        if (a > bv) { bv = a; bi = i; }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            double v2 = sv[threadIdx.x + o];
            int64_t i2 = si[threadIdx.x + o];
            double v1 = sv[threadIdx.x];
            int64_t i1 = si[threadIdx.x];
            if (v2 > v1 || (v2 == v1 && i2 >= 0 && (i1 < 0 || i2 < i1))) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pv[blockIdx.x] = sv[0];
        pi[blockIdx.x] = si[0];
    }
}

// fac = sign(u[argmax |u|]) / nrm, decided once by a single thread before
// any element is rescaled
__global__ void k_sign_factor(const double* __restrict__ u, const double* nrm,
                              const double* pv, const int64_t* pi, int G, double* fac) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double bv = -1.0;
    int64_t bi = -1;
    for (int b = 0; b < G; ++b)
        if (pv[b] > bv || (pv[b] == bv && pi[b] >= 0 && (bi < 0 || pi[b] < bi))) {
            bv = pv[b];
            bi = pi[b];
        }
    const double sg = (bi >= 0 && u[bi] < 0) ? -1.0 : 1.0;
    *fac = sg / *nrm;
}

__global__ void k_scale_by(double* __restrict__ u, int64_t n, const double* fac) {
    const double f = *fac;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        u[i] *= f;
}

// Fused Lanczos vector update + dot products, one pass over the basis:
//   mode 0: w -= alpha_j v_j + beta_{j-1} v_{j-1}, then partials of V[r].w,
//           r <= j, and of w.w (row j + 1)
//   mode 1: w -= sum_{r < nrows} c[r] V[r], then, if a second Gram-Schmidt
//           pass is needed, partials of V[r].w, r < nrows; otherwise the
//           partial of w.w in row 0 (other rows zero)
//   mode 2: if the second pass is needed, w -= sum_{r < nrows} c[r] V[r]
//           and the partial of w.w; otherwise w is final and the partials
//           forward c[0] (the norm from mode 1) unchanged
// The second pass follows the criterion of Daniel, Gragg, Kaufman and
// Stewart (Math. Comp. 30, 1976): with a = |w|^2 before the projection and
// p = sum_r c_r^2 the squared length removed by it, |w'|^2 = a - p; the
// projection is repeated only when it removed more than half of |w|^2
// (|w'| < |w| / sqrt 2).  Both modes evaluate the test from the mode-0
// coefficients `cf` (c_r, r < nrows, and a in entry nrows) with the same
// arithmetic, so they agree everywhere.
// The element partition (contiguous slice per workgroup, stride 256 inside),
// the per-row accumulation order and the wave/block reduction are those of
// k_dot_partial, and the update expressions those of k_lz_three_term and
// k_lz_subtract; each basis element is loaded once for both the update and
// the dots.
__device__ __forceinline__ bool lz_second_pass(const double* cf, int nrows) {
    double p = 0.0;
    for (int r = 0; r < nrows; ++r) p += cf[r] * cf[r];
    return 2.0 * p > cf[nrows];
}

template <int MAXR, typename TV>
__global__ __launch_bounds__(256) void k_lz_fused(double* __restrict__ w, const TV* __restrict__ V,
                                                  int64_t ldv, int mode, int nrows, int j,
                                                  const double* __restrict__ alpha,
                                                  const double* __restrict__ beta,
                                                  const double* __restrict__ c,
                                                  const double* __restrict__ cf, int64_t n,
                                                  double* __restrict__ partial, const LState* st) {
    if (st->broken) return;
    __shared__ double sh[MAXR][4];
    const int G = gridDim.x;
    const bool second = mode == 0 || lz_second_pass(cf, nrows);
    if (mode == 2 && !second) {
        if (threadIdx.x == 0) partial[blockIdx.x] = blockIdx.x == 0 ? c[0] : 0.0;
        return;
    }
    const int64_t chunk = (n + G - 1) / G;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    const int nr = mode == 0 ? j + 1 : nrows;          // rows in the update / dots
    const int nd = mode == 0 ? j + 2 : mode == 2 ? 1 : nr;   // partial rows written
    const bool norm_only = mode == 2 || !second;         // mode 1 without a second pass
    const double a = mode == 0 ? alpha[j] : 0.0;
    const double b = (mode == 0 && j > 0) ? beta[j - 1] : 0.0;
    double s[MAXR];
#pragma unroll
    for (int q = 0; q < MAXR; ++q) s[q] = 0.0;
    // up to 32 rows the element's basis entries stay in registers between
    // the update and the dots
    constexpr bool CACHE = MAXR <= 32;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
        constexpr int NV = CACHE ? MAXR : 1;
        double v[NV];
        if constexpr (CACHE) {
            // every row's load is issued before any is converted: left to
            // itself the compiler converts a float row inside its guarded load
            // and so waits for each load in turn; the empty asm statements
            // (no instruction) hold the loaded values until all are issued
            TV vt[NV];
#pragma unroll
            for (int r = 0; r < NV; ++r) vt[r] = r < nr ? V[(int64_t)r * ldv + i] : (TV)0;
            if constexpr (sizeof(TV) == 4) {
#pragma unroll
                for (int r = 0; r < NV; ++r) asm volatile("" : "+v"(vt[r]));
            }
#pragma unroll
            for (int r = 0; r < NV; ++r) v[r] = (double)vt[r];
        }
#define QED_ROW(r) (CACHE ? v[(r) < NV ? (r) : 0] : (double)V[(int64_t)(r) * ldv + i])
        double wi = w[i];
        if (mode == 0) {
            // rows j and j-1 are cached from the loads above
            double t = a * (double)V[(int64_t)j * ldv + i];
            if (j > 0) t += b * (double)V[(int64_t)(j - 1) * ldv + i];
            wi -= t;
        } else {
            double t = 0.0;
#pragma unroll
            for (int r = 0; r < MAXR; ++r)
                if (r < nr) t += c[r] * QED_ROW(r);
            wi -= t;
        }
        w[i] = wi;
        if (norm_only) {
            s[0] += wi * wi;
        } else {
#pragma unroll
            for (int r = 0; r < MAXR; ++r)
                if (r < nr) s[r] += QED_ROW(r) * wi;
            if (mode == 0) {
#pragma unroll
                for (int r = 0; r < MAXR; ++r)
                    if (r == nr) s[r] += wi * wi;
            }
        }
    }
#undef QED_ROW
#pragma unroll
    for (int q = 0; q < MAXR; ++q) {
        if (q < nd) {
            double t = wave_sum(s[q]);
            if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x >> 6] = t;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nd)
        partial[(int64_t)threadIdx.x * G + blockIdx.x] =
            ((sh[threadIdx.x][0] + sh[threadIdx.x][1]) + sh[threadIdx.x][2]) + sh[threadIdx.x][3];
}

// The mode-2 pass's final sum (|w|^2 into *ww) followed by the step of
// k_lz_beta (beta_j = |w|, or breakdown) in the same single workgroup.
__global__ __launch_bounds__(256) void k_dot_final_beta(const double* __restrict__ partial, int G,
                                                        double* __restrict__ ww, double* alpha,
                                                        double* beta, int j, LState* st,
                                                        double tol) {
    if (st->broken) return;
    __shared__ double sh[4];
    double s = 0.0;
    for (int b = threadIdx.x; b < G; b += 256) s += partial[b];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double t = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    *ww = t;
    const double b = sqrt(t);
    double scale = 1.0;
    for (int i = 0; i <= j; ++i) scale = fmax(scale, fabs(alpha[i]));
    for (int i = 0; i < j; ++i) scale = fmax(scale, beta[i]);
    if (b <= tol * scale) {
        beta[j] = 0.0;
        st->broken = 1;
        st->k = j + 1;
    } else {
        beta[j] = b;
    }
}

template <typename TV>
bool launch_lz_fused(int mode, double* w, const TV* V, int64_t ldv, int nrows, int j,
                     const double* alpha, const double* beta, const double* c, const double* cf,
                     int64_t n, double* partial, double* out, const LState* st, hipStream_t s) {
    const int nr = mode == 0 ? j + 1 : nrows;
    if (nr + 1 > 32) return false;   // mode 0 also needs the row of w.w
    const int G = dot_grid(n);
    if (nr + 1 <= 16)
        hipLaunchKernelGGL((k_lz_fused<16, TV>), dim3(G), dim3(256), 0, s, w, V, ldv, mode, nrows, j, alpha,
                           beta, c, cf, n, partial, st);
    else
        hipLaunchKernelGGL((k_lz_fused<32, TV>), dim3(G), dim3(256), 0, s, w, V, ldv, mode, nrows, j, alpha,
                           beta, c, cf, n, partial, st);
    const int nd = mode == 0 ? j + 2 : mode == 2 ? 1 : nr;
    hipLaunchKernelGGL(k_dot_final, dim3(nd), dim3(256), 0, s, partial, G, nd, out, 0, st, 1);
    return true;
}
template bool launch_lz_fused<double>(int, double*, const double*, int64_t, int, int, const double*, const double*,
                                      const double*, const double*, int64_t, double*, double*, const LState*,
                                      hipStream_t);
template bool launch_lz_fused<float>(int, double*, const float*, int64_t, int, int, const double*, const double*,
                                     const double*, const double*, int64_t, double*, double*, const LState*,
                                     hipStream_t);

template <typename TV>
bool launch_lz_norm_beta(double* w, const TV* V, int64_t ldv, int nrows, int j, double* alpha,
                         double* beta, const double* c, const double* cf, int64_t n, double* partial,
                         double* ww, LState* st, double tol, hipStream_t s) {
    if (nrows + 1 > 32) return false;
    const int G = dot_grid(n);
    if (nrows + 1 <= 16)
        hipLaunchKernelGGL((k_lz_fused<16, TV>), dim3(G), dim3(256), 0, s, w, V, ldv, 2, nrows, j, alpha,
                           beta, c, cf, n, partial, st);
    else
        hipLaunchKernelGGL((k_lz_fused<32, TV>), dim3(G), dim3(256), 0, s, w, V, ldv, 2, nrows, j, alpha,
                           beta, c, cf, n, partial, st);
    hipLaunchKernelGGL(k_dot_final_beta, dim3(1), dim3(256), 0, s, partial, G, ww, alpha, beta, j, st,
                       tol);
    return true;
}
template bool launch_lz_norm_beta<double>(double*, const double*, int64_t, int, int, double*, double*,
                                          const double*, const double*, int64_t, double*, double*, LState*, double,
                                          hipStream_t);
template bool launch_lz_norm_beta<float>(double*, const float*, int64_t, int, int, double*, double*,
                                         const double*, const double*, int64_t, double*, double*, LState*, double,
                                         hipStream_t);

void launch_lz_three_term(double* w, const double* V, int64_t ldv, int j, const double* alpha,
                          const double* beta, int64_t n, const LState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_three_term, dim3(grid_for(n)), dim3(256), 0, s, w, V, ldv, j, alpha,
                       beta, n, st);
}
void launch_lz_subtract(double* w, const double* V, int64_t ldv, int nrows, const double* c,
                        int64_t n, const LState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_subtract, dim3(grid_for(n)), dim3(256), 0, s, w, V, ldv, nrows, c, n,
                       st);
}
void launch_lz_beta(const double* ww, double* alpha, double* beta, int j, LState* st, double tol,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_lz_beta, dim3(1), dim3(1), 0, s, ww, alpha, beta, j, st, tol);
}
template <typename TV>
void launch_lz_next(TV* V, int64_t ldv, int j, const double* w, const double* beta, int64_t n,
                    const LState* st, hipStream_t s, float* vc) {
    hipLaunchKernelGGL(k_lz_next<TV>, dim3(grid_for(n)), dim3(256), 0, s, V, ldv, j, w, beta, n, st, vc);
}
template void launch_lz_next<double>(double*, int64_t, int, const double*, const double*, int64_t, const LState*,
                                     hipStream_t, float*);
template void launch_lz_next<float>(float*, int64_t, int, const double*, const double*, int64_t, const LState*,
                                    hipStream_t, float*);
template <typename TV>
void launch_lz_start(TV* dst, const double* src, const double* nrm, int64_t n, LState* st,
                     int m, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_start<TV>, dim3(grid_for(n)), dim3(256), 0, s, dst, src, nrm, n, st, m);
}
template void launch_lz_start<double>(double*, const double*, const double*, int64_t, LState*, int, hipStream_t);
template void launch_lz_start<float>(float*, const double*, const double*, int64_t, LState*, int, hipStream_t);
void launch_tridiag(const double* alpha, const double* beta, double* sv, LState* st, double* work,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_tridiag_lowest, dim3(1), dim3(64), 0, s, alpha, beta, sv, st, work);
}
template <typename TV>
void launch_ritz(double* u, const TV* V, int64_t ldv, const double* sv, int64_t n,
                 const LState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_ritz<TV>, dim3(grid_for(n)), dim3(256), 0, s, u, V, ldv, sv, n, st);
}
template void launch_ritz<double>(double*, const double*, int64_t, const double*, int64_t, const LState*,
                                  hipStream_t);
template void launch_ritz<float>(double*, const float*, int64_t, const double*, int64_t, const LState*, hipStream_t);
void launch_normalise_sign(double* u, int64_t n, const double* nrm, double* pv, int64_t* pi,
                           double* fac, hipStream_t s) {
    const int G = dot_grid(n);
    hipLaunchKernelGGL(k_argmax_partial, dim3(G), dim3(256), 0, s, u, n, pv, pi);
    hipLaunchKernelGGL(k_sign_factor, dim3(1), dim3(1), 0, s, u, nrm, pv, pi, G, fac);
    hipLaunchKernelGGL(k_scale_by, dim3(grid_for(n)), dim3(256), 0, s, u, n, fac);
}

// ---------------------------------------------------------------------
// one-sided Jacobi SVD (Hestenes) of small matrices
// ---------------------------------------------------------------------
// One workgroup per matrix.  A sweep visits every column pair once in the
// round-robin (tournament) order, m' - 1 rounds of m'/2 disjoint pairs
// (m' = m rounded up to even, the extra column a dummy); each wave rotates
// its pairs: with a = |x_p|^2, b = |x_q|^2, g = x_p . x_q, the rotation with
// zeta = (b - a) / 2g, t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// c = 1 / sqrt(1 + t^2), s = c t makes the two columns orthogonal, and is
// applied to the same columns of V.  Sweeps stop when no pair had
// |g| > 1e-15 sqrt(a b), or after 60; numerically zero columns are skipped.
// Fixed order: reproducible.
__global__ __launch_bounds__(256) void k_jacobi_svd(const SvdMat* __restrict__ mats) {
    const SvdMat S = mats[blockIdx.x];
    const int n = S.n, m = S.m;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ int rotated;
    __shared__ double fro[4];
    for (int i = threadIdx.x; i < m * m; i += 256) S.v[i] = (i % m == i / m) ? 1.0 : 0.0;
    // columns below 1e-16 of the Frobenius norm are left alone (they are
    // numerically zero and get dropped by any truncation)
    double f2 = 0.0;
    for (int64_t i = threadIdx.x; i < (int64_t)n * m; i += 256) f2 += S.x[i] * S.x[i];
    f2 = wave_sum(f2);
    if (lane == 0) fro[wave] = f2;
    __syncthreads();
    const double tiny = 1e-32 * (((fro[0] + fro[1]) + fro[2]) + fro[3]);
    const int mp = (m + 1) & ~1;
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (threadIdx.x == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < mp - 1; ++r) {
            for (int k = wave; k < mp / 2; k += 4) {
                // tournament pairing: position 0 fixed, the others rotate
                const int a0 = k == 0 ? 0 : 1 + (k - 1 + r) % (mp - 1);
                const int b0 = 1 + (mp - 2 - k + r) % (mp - 1);
                const int p = a0 < b0 ? a0 : b0, q = a0 < b0 ? b0 : a0;
                if (q >= m) continue;
                double* xp = S.x + (int64_t)p * n;
                double* xq = S.x + (int64_t)q * n;
                double sa = 0.0, sb = 0.0, sg = 0.0;
                for (int i = lane; i < n; i += 64) {
                    const double u = xp[i], w = xq[i];
                    sa += u * u;
                    sb += w * w;
                    sg += u * w;
                }
                sa = wave_sum(sa);
                sb = wave_sum(sb);
                sg = wave_sum(sg);
                sa = __shfl(sa, 0, 64);
                sb = __shfl(sb, 0, 64);
                sg = __shfl(sg, 0, 64);
                if (sa <= tiny || sb <= tiny || fabs(sg) <= 1e-15 * sqrt(sa) * sqrt(sb)) continue;
                const double zeta = (sb - sa) / (2.0 * sg);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int i = lane; i < n; i += 64) {
                    const double u = xp[i], w = xq[i];
                    xp[i] = c * u - s * w;
                    xq[i] = s * u + c * w;
                }
                double* vp = S.v + (int64_t)p * m;
                double* vq = S.v + (int64_t)q * m;
                for (int i = lane; i < m; i += 64) {
                    const double u = vp[i], w = vq[i];
                    vp[i] = c * u - s * w;
                    vq[i] = s * u + c * w;
                }
                if (lane == 0) rotated = 1;
            }
            __syncthreads();
        }
        const int any = rotated;
        __syncthreads();
        if (!any) break;
    }
    for (int j = wave; j < m; j += 4) {
        const double* x = S.x + (int64_t)j * n;
        double s2 = 0.0;
        for (int i = lane; i < n; i += 64) s2 += x[i] * x[i];
        s2 = wave_sum(s2);
        if (lane == 0) S.sigma[j] = sqrt(s2);
    }
}

void launch_jacobi_svd(const SvdMat* mats, int nmats, hipStream_t s) {
    if (nmats <= 0) return;
    hipLaunchKernelGGL(k_jacobi_svd, dim3(nmats), dim3(256), 0, s, mats);
}

// y += f x
__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double f, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] += f * x[i];
}

void launch_axpy(double* y, const double* x, double f, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, s, y, x, f, n);
}

// ---------------------------------------------------------------------
// QR of the sector matrices of a node matricised along one leg
// ---------------------------------------------------------------------
// pack (dir = 0): tensor -> column-major sector matrices; unpack (dir = 1)
__global__ void k_pack(const PackBlk* __restrict__ blks, double* __restrict__ tensor,
                       double* __restrict__ packed, int dir) {
    const PackBlk B = blks[blockIdx.x];
    const int64_t size = (int64_t)B.n[0] * B.n[1] * B.n[2];
    for (int64_t e = blockIdx.y * (int64_t)blockDim.x + threadIdx.x; e < size;
         e += (int64_t)gridDim.y * blockDim.x) {
        const int ip = (int)(e % B.n[2]);
        const int64_t t = e / B.n[2];
        const int ir = (int)(t % B.n[1]);
        const int il = (int)(t / B.n[1]);
        int row, col;
        if (B.leg == 2) { col = ip; row = il * B.n[1] + ir; }
        else if (B.leg == 0) { col = il; row = ir * B.n[2] + ip; }
        else { col = ir; row = il * B.n[2] + ip; }
        const int64_t pidx = B.mat + (int64_t)col * B.rows + B.row0 + row;
        if (dir == 0) packed[pidx] = tensor[B.off + e];
        else tensor[B.off + e] = packed[pidx];
    }
}

void launch_pack(const PackBlk* blks, int nblk, int64_t maxsize, double* tensor, double* packed,
                 int dir, hipStream_t s) {
    if (nblk <= 0) return;
    int64_t gy = (maxsize + 255) / 256;
    if (gy > 256) gy = 256;
    if (gy < 1) gy = 1;
    hipLaunchKernelGGL(k_pack, dim3(nblk, (int)gy), dim3(256), 0, s, blks, tensor, packed, dir);
}

// Householder QR of one column-major rows x cols matrix (leading dimension
// ld) per workgroup, cols <= rows <= QR_ROWS, cols <= QR_COLS.  On exit the
// matrix holds the explicit Q with orthonormal columns and R is written
// through (rout, rrs, rcs); signs are fixed so that diag(R) >= 0.  `qbuf` is
// scratch with the same layout as the input.  Zero columns (rank
// deficiency) get tau = 0 and R_jj = 0, and Q still has orthonormal columns.
//
// Blocked (compact WY) form: panels of QB columns are staged in LDS and
// factored there; the panel's reflectors H_1..H_w are combined into
// I - V T V^T (T upper triangular, from the Gram matrix of V and the tau),
// and the trailing columns get (I - V T^T V^T) in one pass each, a wave per
// pair of columns held in registers.  Q is accumulated backwards by panels
// with the same one-pass update.  Each trailing column is thus read and
// written once per panel instead of once per reflector.
constexpr int QB = 8;
constexpr int QR_RPL = QR_ROWS / 64;   // rows per lane in the column passes
constexpr int QB_PAIRS = QB * (QB - 1) / 2;

// Sum over the 64 lanes, the same value in every lane.  A butterfly whose
// every step adds the partner lane's partial, so both partners form the
// same sum (addition commutes) and all lanes end bit-identical: the first
// four steps move data inside rows of 16 lanes with DPP (quad_perm [1,0,3,2]
// and [2,3,0,1], row_half_mirror, row_mirror; no LDS traffic), the last two
// exchange across rows with shuffles.  Needs every lane active.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_allsum(double v) {
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_move<0x141>(v);   // row_half_mirror: the other quad of 8 lanes
    v += dpp_move<0x140>(v);   // row_mirror: the other half of 16 lanes
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}
__device__ __forceinline__ double wave_bcast_sum(double v) { return wave_allsum(v); }

// y <- y - V S y for the QB-column panel V in LDS (rows r >= k of column k;
// r relative to the panel's first row), S = T^T (trans = 1) or T, on the
// columns c0 and c0 + 1 (if present) of the column-major matrix X.
template <bool TRANS>
__device__ __forceinline__ void apply_panel(double* X, int64_t ld, int row0, int mr, int c0, bool two,
                                            const double* Vp, const double* T, int lane) {
    double a0[QR_RPL], a1[QR_RPL];
    double* x0 = X + (int64_t)c0 * ld + row0;
    double* x1 = x0 + ld;
#pragma unroll
    for (int t = 0; t < QR_RPL; ++t) {
        if (64 * t >= mr) break;   // uniform: the wave's rows end here
        const int r = lane + 64 * t;
        a0[t] = r < mr ? x0[r] : 0.0;
        a1[t] = (two && r < mr) ? x1[r] : 0.0;
    }
    double w0[QB], w1[QB];
#pragma unroll
    for (int k = 0; k < QB; ++k) w0[k] = w1[k] = 0.0;
#pragma unroll
    for (int t = 0; t < QR_RPL; ++t) {
        if (64 * t >= mr) break;
        const int r = lane + 64 * t;
        if (r < mr) {
#pragma unroll
            for (int k = 0; k < QB; ++k) {
                const double v = r >= k ? Vp[r * QB + k] : 0.0;
                w0[k] += v * a0[t];
                w1[k] += v * a1[t];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < QB; ++k) {
        w0[k] = wave_bcast_sum(w0[k]);
        w1[k] = wave_bcast_sum(w1[k]);
    }
    double s0[QB], s1[QB];
#pragma unroll
    for (int k = 0; k < QB; ++k) {
        s0[k] = s1[k] = 0.0;
#pragma unroll
        for (int a = 0; a < QB; ++a) {
            const double tk = TRANS ? T[a * QB + k] : T[k * QB + a];
            s0[k] += tk * w0[a];
            s1[k] += tk * w1[a];
        }
    }
#pragma unroll
    for (int t = 0; t < QR_RPL; ++t) {
        if (64 * t >= mr) break;
        const int r = lane + 64 * t;
        if (r < mr) {
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int k = 0; k < QB; ++k) {
                const double v = r >= k ? Vp[r * QB + k] : 0.0;
                d0 += v * s0[k];
                d1 += v * s1[k];
            }
            x0[r] = a0[t] - d0;
            if (two) x1[r] = a1[t] - d1;
        }
    }
}

__global__ __launch_bounds__(256) void k_householder_qr(const QRMat* __restrict__ mats) {
    __shared__ double Vp[QR_ROWS * QB];                    // panel, row-major
    __shared__ double Ts[(QR_COLS / QB) * QB * QB];        // T of every panel
    __shared__ double tau[QR_COLS], diag[QR_COLS];
    __shared__ double red[4][QB_PAIRS > QB ? QB_PAIRS : QB];
    const QRMat Mt = mats[blockIdx.x];
    const int m = Mt.rows, n = Mt.cols;
    const int64_t ld = Mt.ld;
    double* A = Mt.a;
    double* Qm = Mt.q;
    double* R = Mt.r;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int npan = (n + QB - 1) / QB;
    for (int p = 0; p < npan; ++p) {
        const int j0 = p * QB, w = min(QB, n - j0), mr = m - j0;
        for (int e = tid; e < mr * QB; e += 256) {
            const int k = e / mr, r = e % mr;
            Vp[r * QB + k] = k < w ? A[(int64_t)(j0 + k) * ld + j0 + r] : 0.0;
        }
        __syncthreads();
        // unblocked factorisation of the panel
        for (int i = 0; i < w; ++i) {
            double s = 0.0;
            for (int r = i + tid; r < mr; r += 256) s += Vp[r * QB + i] * Vp[r * QB + i];
            s = wave_allsum(s);
            if (lane == 0) red[wave][0] = s;
            __syncthreads();
            if (tid == 0) {
                const double norm2 = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
                const double x0 = Vp[i * QB + i];
                const double nrm = sqrt(norm2);
                if (nrm == 0.0) {
                    tau[j0 + i] = 0.0;
                    diag[j0 + i] = 0.0;
                } else {
                    const double al = x0 >= 0.0 ? -nrm : nrm;
                    const double v0 = x0 - al;
                    const double vtv = v0 * v0 + (norm2 - x0 * x0);
                    tau[j0 + i] = vtv > 0.0 ? 2.0 / vtv : 0.0;
                    diag[j0 + i] = al;
                    Vp[i * QB + i] = v0;
                }
            }
            __syncthreads();
            const double ti = tau[j0 + i];
            if (ti != 0.0 && i + 1 < w) {
                double d[QB];
#pragma unroll
                for (int k = 0; k < QB; ++k) d[k] = 0.0;
                for (int r = i + tid; r < mr; r += 256) {
                    const double v = Vp[r * QB + i];
#pragma unroll
                    for (int k = 0; k < QB; ++k)
                        if (k > i) d[k] += v * Vp[r * QB + k];
                }
#pragma unroll
                for (int k = 0; k < QB; ++k) {
                    if (k <= i) continue;
                    const double t = wave_allsum(d[k]);
                    if (lane == 0) red[wave][k] = t;
                }
                __syncthreads();
                double f[QB];
#pragma unroll
                for (int k = 0; k < QB; ++k)
                    f[k] = k > i ? ti * (((red[0][k] + red[1][k]) + red[2][k]) + red[3][k]) : 0.0;
                for (int r = i + tid; r < mr; r += 256) {
                    const double v = Vp[r * QB + i];
#pragma unroll
                    for (int k = 0; k < QB; ++k)
                        if (k > i) Vp[r * QB + k] -= f[k] * v;
                }
                __syncthreads();
            }
        }
        // the panel back to the matrix: v below the diagonal, v0 on it,
        // the panel's part of R above it
        for (int e = tid; e < mr * w; e += 256) {
            const int k = e / mr, r = e % mr;
            A[(int64_t)(j0 + k) * ld + j0 + r] = Vp[r * QB + k];
        }
        // compact WY factor T from the Gram matrix of the panel's V
        double g[QB_PAIRS];
#pragma unroll
        for (int q = 0; q < QB_PAIRS; ++q) g[q] = 0.0;
        for (int r = tid; r < mr; r += 256) {
            int q = 0;
#pragma unroll
            for (int b = 1; b < QB; ++b)
#pragma unroll
                for (int a = 0; a < b; ++a, ++q)
                    if (r >= b) g[q] += Vp[r * QB + a] * Vp[r * QB + b];
        }
#pragma unroll
        for (int q = 0; q < QB_PAIRS; ++q) {
            const double t = wave_allsum(g[q]);
            if (lane == 0) red[wave][q] = t;
        }
        __syncthreads();
        double* T = Ts + p * QB * QB;
        if (tid == 0) {
            for (int e = 0; e < QB * QB; ++e) T[e] = 0.0;
            for (int i = 0; i < w; ++i) {
                const double ti = tau[j0 + i];
                T[i * QB + i] = ti;
                double z[QB];
                for (int a = 0; a < i; ++a) {
                    const int q = i * (i - 1) / 2 + a;   // pair (a, b = i)
                    z[a] = -ti * (((red[0][q] + red[1][q]) + red[2][q]) + red[3][q]);
                }
                for (int a = 0; a < i; ++a) {
                    double s = 0.0;
                    for (int b = a; b < i; ++b) s += T[a * QB + b] * z[b];
                    T[a * QB + i] = s;
                }
            }
        }
        __syncthreads();
        // trailing columns: A <- (I - V T^T V^T) A
        for (int c0 = j0 + w + 2 * wave; c0 < n; c0 += 8)
            apply_panel<true>(A, ld, j0, mr, c0, c0 + 1 < n, Vp, T, lane);
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += 256) {
        const int r = e / n, c = e % n;
        R[r * Mt.rrs + c * Mt.rcs] = c > r ? A[(int64_t)c * ld + r] : (c == r ? diag[r] : 0.0);
    }
    for (int64_t e = tid; e < (int64_t)m * n; e += 256) {
        const int c = (int)(e / m), r = (int)(e % m);
        Qm[(int64_t)c * ld + r] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    // Q = H_1 ... H_n [I; 0], panels applied last to first: Q <- (I - V T V^T) Q
    for (int p = npan - 1; p >= 0; --p) {
        const int j0 = p * QB, w = min(QB, n - j0), mr = m - j0;
        for (int e = tid; e < mr * QB; e += 256) {
            const int k = e / mr, r = e % mr;
            Vp[r * QB + k] = (k < w && r >= k) ? A[(int64_t)(j0 + k) * ld + j0 + r] : 0.0;
        }
        __syncthreads();
        for (int c0 = j0 + 2 * wave; c0 < n; c0 += 8)
            apply_panel<false>(Qm, ld, j0, mr, c0, c0 + 1 < n, Vp, Ts + p * QB * QB, lane);
        __syncthreads();
    }
    for (int64_t e = tid; e < (int64_t)m * n; e += 256) {
        const int c = (int)(e / m), r = (int)(e % m);
        const double q = Qm[(int64_t)c * ld + r];
        A[(int64_t)c * ld + r] = diag[c] < 0.0 ? -q : q;
    }
    for (int e = tid; e < n * n; e += 256) {
        const int r = e / n, c = e % n;
        if (diag[r] < 0.0) R[r * Mt.rrs + c * Mt.rcs] = -R[r * Mt.rrs + c * Mt.rcs];
    }
}

// Unblocked Householder QR for sectors wider than QR_COLS (no size limit
// beyond LDS for 2 cols + 4 doubles): one column-major rows x cols matrix
// (leading dimension ld) per workgroup, rows >= cols, reflectors applied
// to the trailing columns one at a time, waves over columns.  On exit the matrix holds the explicit Q
// with orthonormal columns and R is written through (rout, rrs, rcs); signs
// are fixed so that diag(R) >= 0.  `qbuf` is scratch with the same layout
// as the input.  Zero columns (rank deficiency) get tau = 0 and R_jj = 0,
// and Q still has orthonormal columns.
__global__ __launch_bounds__(256) void k_householder_qr_wide(const QRMat* __restrict__ mats) {
    extern __shared__ double lds[];
    const QRMat Mt = mats[blockIdx.x];
    const int m = Mt.rows, n = Mt.cols;
    const int64_t ld = Mt.ld;
    double* A = Mt.a;
    double* Qm = Mt.q;
    double* R = Mt.r;
    double* tau = lds;          // n
    double* diag = lds + n;     // n  (R_jj)
    double* red = lds + 2 * n;  // 4
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = j + tid; i < m; i += 256) s += A[(int64_t)j * ld + i] * A[(int64_t)j * ld + i];
        s = wave_sum(s);
        if (lane == 0) red[wave] = s;
        __syncthreads();
        if (tid == 0) {
            const double norm2 = ((red[0] + red[1]) + red[2]) + red[3];
            const double x0 = A[(int64_t)j * ld + j];
            const double nrm = sqrt(norm2);
            if (nrm == 0.0) {
                tau[j] = 0.0;
                diag[j] = 0.0;
            } else {
                const double al = x0 >= 0.0 ? -nrm : nrm;
                const double v0 = x0 - al;
                const double vtv = v0 * v0 + (norm2 - x0 * x0);
                tau[j] = vtv > 0.0 ? 2.0 / vtv : 0.0;
                diag[j] = al;
                A[(int64_t)j * ld + j] = v0;
            }
        }
        __syncthreads();
        const double tj = tau[j];
        if (tj != 0.0) {
            for (int k = j + 1 + wave; k < n; k += 4) {
                double d = 0.0;
                for (int i = j + lane; i < m; i += 64) d += A[(int64_t)j * ld + i] * A[(int64_t)k * ld + i];
                d = wave_sum(d);
                d = __shfl(d, 0, 64);
                const double f = tj * d;
                for (int i = j + lane; i < m; i += 64) A[(int64_t)k * ld + i] -= f * A[(int64_t)j * ld + i];
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += 256) {
        const int r = e / n, c = e % n;
        R[r * Mt.rrs + c * Mt.rcs] = c > r ? A[(int64_t)c * ld + r] : (c == r ? diag[r] : 0.0);
    }
    for (int64_t e = tid; e < (int64_t)m * n; e += 256) {
        const int c = (int)(e / m), r = (int)(e % m);
        Qm[(int64_t)c * ld + r] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = n - 1; j >= 0; --j) {
        const double tj = tau[j];
        if (tj != 0.0) {
            for (int k = j + wave; k < n; k += 4) {
                double d = 0.0;
                for (int i = j + lane; i < m; i += 64) d += A[(int64_t)j * ld + i] * Qm[(int64_t)k * ld + i];
                d = wave_sum(d);
                d = __shfl(d, 0, 64);
                const double f = tj * d;
                for (int i = j + lane; i < m; i += 64) Qm[(int64_t)k * ld + i] -= f * A[(int64_t)j * ld + i];
            }
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < (int64_t)m * n; e += 256) {
        const int c = (int)(e / m), r = (int)(e % m);
        const double q = Qm[(int64_t)c * ld + r];
        A[(int64_t)c * ld + r] = diag[c] < 0.0 ? -q : q;
    }
    for (int e = tid; e < n * n; e += 256) {
        const int r = e / n, c = e % n;
        if (diag[r] < 0.0) R[r * Mt.rrs + c * Mt.rcs] = -R[r * Mt.rrs + c * Mt.rcs];
    }
}

// ---------------------------------------------------------------------
// CholeskyQR: factor of the Gram matrix, its inverse, the running R
// ---------------------------------------------------------------------
// One workgroup per sector.  G (+ the shift) is copied to LDS and factored
// in place column by column (right-looking: row j of R is formed from its
// pivot, the trailing upper triangle takes one rank-1 update); the pivot
// test uses the largest diagonal entry.  R^-1 is formed in LDS by back
// substitution, one column per thread (each column's triangular solve is
// independent), and written out once complete.
__global__ __launch_bounds__(256) void k_chol_inv(const CholMat* __restrict__ mats) {
    extern __shared__ double sh[];
    const CholMat M = mats[blockIdx.x];
    const int n = M.n, ld = n + 1;
    double* G = sh;                    // n x ld: G, then R in its upper triangle
    double* X = sh + n * ld;           // n x ld: R^-1
    __shared__ double gmax, sft;
    __shared__ int bad;
    const int tid = threadIdx.x;
    for (int i = tid; i < n * n; i += blockDim.x) G[(i / n) * ld + i % n] = M.g[i];
    __syncthreads();
    if (tid == 0) {
        double m = 0.0, tr = 0.0;
        for (int i = 0; i < n; ++i) {
            m = fmax(m, G[i * ld + i]);
            tr += G[i * ld + i];
        }
        sft = M.shift * tr;
        gmax = m + sft;
        bad = 0;
    }
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) G[i * ld + i] += sft;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double d = G[j * ld + j];
        if (!(d > 1e-12 * gmax)) {
            if (tid == 0) bad = 1;
            break;
        }
        const double r = sqrt(d);
        __syncthreads();
        for (int k = j + tid; k < n; k += blockDim.x) G[j * ld + k] = (k == j) ? r : G[j * ld + k] / r;
        __syncthreads();
        const int t = n - j - 1;
        for (int e = tid; e < t * t; e += blockDim.x) {
            const int i = j + 1 + e / t, k = j + 1 + e % t;
            if (k >= i) G[i * ld + k] -= G[j * ld + i] * G[j * ld + k];
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) *M.status = 1;
        return;
    }
    if (tid == 0) *M.status = 0;
    // R^-1: column c solves R x = e_c (x[i] = 0 for i > c)
    for (int c = tid; c < n; c += blockDim.x) {
        for (int i = n - 1; i > c; --i) X[i * ld + c] = 0.0;
        X[c * ld + c] = 1.0 / G[c * ld + c];
        for (int i = c - 1; i >= 0; --i) {
            double acc = 0.0;
            for (int k = i + 1; k <= c; ++k) acc += G[i * ld + k] * X[k * ld + c];
            X[i * ld + c] = -acc / G[i * ld + i];
        }
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) M.rinv[e] = X[(e / n) * ld + e % n];
    // the running R: R rprev (both upper triangular), or R itself
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        double v = 0.0;
        if (j >= i) {
            if (M.rprev) {
                for (int k = i; k <= j; ++k) v += G[i * ld + k] * M.rprev[(int64_t)k * n + j];
            } else {
                v = G[i * ld + j];
            }
        }
        M.rout[i * M.rrs + j * M.rcs] = v;
    }
}

// Householder QR of one column-major rows x cols chunk per workgroup with
// the whole chunk resident in LDS (qr_lds_fits); the same contract as
// k_householder_qr (explicit Q written over the input, R through (rout,
// rrs, rcs), diag(R) >= 0, tau = 0 and R_jj = 0 for a zero column).
// The rows below the diagonal are split into four ranges, one per wave.
// With more than 64 trailing columns lane l of every wave owns column
// k = i + 1 + l and k + 64; with at most 64 the wave's lanes are spread
// over the trailing columns and slices of its rows (qrl_lanes), so that the
// per-lane loops shrink with the trailing matrix instead of idling lanes
// (the loops are bound by the LDS instructions a wave issues).  The
// products v^T a_k are per-lane sums over a lane's rows (eight rows' loads
// issued together), summed over the slices by lane exchanges and across
// the waves through LDS in a fixed order (one barrier).  The norm of the
// next column is gathered while its update is written.  Q is then formed in place from the reflectors,
// last to first (column i becomes H_i e_i once the columns right of it
// hold H_i+1 ... [I; 0]), with the same column-per-lane products.  The
// leading dimension in LDS is odd, so the lanes of a wave read different
// banks.
__device__ __forceinline__ void qrl_rows(int r0, int m, int wave, int& rb, int& re) {
    const int nr = m - r0;
    rb = r0 + (nr * wave) / 4;
    re = r0 + (nr * (wave + 1)) / 4;
}

// Lanes of a column step with nc <= 64 trailing columns: lane = s * ncp + c
// with ncp the power of two at or above nc, so each of the 64 / ncp slices
// s of the wave takes column c on its share [sb, se) of the wave's rows
// [rb, re) (every lane busy however few columns are left); the slices'
// sums meet by exchanges across the lane bits at and above ncp.
struct QRLanes {
    int ncp, c, s, sb, se;
    bool act;
};
__device__ __forceinline__ QRLanes qrl_lanes(int nc, int lane, int rb, int re) {
    QRLanes L;
    L.ncp = nc <= 1 ? 1 : 1 << (32 - __clz(nc - 1));
    const int f = 64 / L.ncp;
    L.c = lane & (L.ncp - 1);
    L.s = lane / L.ncp;
    L.act = L.c < nc;
    L.sb = rb + ((re - rb) * L.s) / f;
    L.se = rb + ((re - rb) * (L.s + 1)) / f;
    return L;
}
__device__ __forceinline__ double qrl_slices_sum(double v, int ncp) {
    for (int o = ncp; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sum over rows [rb, re) of v[r] c[r]
__device__ __forceinline__ double qrl_dot(const double* v, const double* c, int rb, int re) {
    double p = 0.0;
    int r = rb;
    for (; r + 8 <= re; r += 8) {
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a[u] = v[r + u];
            b[u] = c[r + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) p += a[u] * b[u];
    }
    for (; r < re; ++r) p += v[r] * c[r];
    return p;
}

// c[r] -= w v[r] over rows [rb, re); returns the sum of the new c[r]^2 over
// rows r > skip
__device__ __forceinline__ double qrl_axpy(double* c, const double* v, double w, int rb, int re, int skip) {
    double s = 0.0;
    int r = rb;
    for (; r + 8 <= re; r += 8) {
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a[u] = v[r + u];
            b[u] = c[r + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            b[u] -= w * a[u];
            if (r + u > skip) s += b[u] * b[u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) c[r + u] = b[u];
    }
    for (; r < re; ++r) {
        const double u = c[r] - w * v[r];
        c[r] = u;
        if (r > skip) s += u * u;
    }
    return s;
}

__global__ __launch_bounds__(256) void k_qr_lds(const QRMat* __restrict__ mats) {
    extern __shared__ double qs[];
    const QRMat Mt = mats[blockIdx.x];
    const int m = Mt.rows, n = Mt.cols;
    const int64_t ldg = Mt.ld;
    const int ld = m | 1;
    double* As = qs;                          // column k at As + k ld
    double* tau = As + (int64_t)ld * n;
    double* vd = tau + n;                     // v on the diagonal
    double* dg = vd + n;                      // R_ii before the sign fix
    double* red = dg + n;                     // [4]
    double* part = red + 4;                   // [4][128]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // (m n fits 32 bits here: 32-bit index arithmetic)
    for (int e = tid; e < m * n; e += 256) {
        const int c = e / m, r = e - c * m;
        As[c * ld + r] = Mt.a[(int64_t)c * ldg + r];
    }
    __syncthreads();
    {
        double s0 = 0.0;
        for (int r = 1 + tid; r < m; r += 256) s0 += As[r] * As[r];
        s0 = wave_allsum(s0);
        if (lane == 0) red[wave] = s0;
    }
    __syncthreads();
    for (int i = 0; i < n; ++i) {
        const double* ci = As + (int64_t)i * ld;
        const double sb = ((red[0] + red[1]) + red[2]) + red[3];
        const double x0 = ci[i];
        const double nrm = sqrt(x0 * x0 + sb);
        double ti = 0.0, v0 = 0.0, al = 0.0;
        if (nrm != 0.0) {
            al = x0 >= 0.0 ? -nrm : nrm;
            v0 = x0 - al;
            const double vtv = v0 * v0 + sb;
            ti = vtv > 0.0 ? 2.0 / vtv : 0.0;
        }
        int rb, re;
        qrl_rows(i + 1, m, wave, rb, re);
        if (tid == 0) {
            tau[i] = ti;
            vd[i] = v0;
            dg[i] = al;
        }
        double nx = 0.0;
        if (n - i - 1 > 64) {
            const int k0 = i + 1 + lane, k1 = k0 + 64;
            const bool a0 = k0 < n, a1 = k1 < n;
            double* c0 = As + (int64_t)(a0 ? k0 : i) * ld;
            double* c1 = As + (int64_t)(a1 ? k1 : i) * ld;
            if (ti != 0.0) {
                double p0 = 0.0, p1 = 0.0;
                if (wave == 0) {
                    p0 = v0 * c0[i];
                    p1 = v0 * c1[i];
                }
                p0 += qrl_dot(ci, c0, rb, re);
                p1 += qrl_dot(ci, c1, rb, re);
                part[wave * 128 + lane] = p0;
                part[wave * 128 + 64 + lane] = p1;
            }
            __syncthreads();
            // updates, and the next column's squares below its diagonal
            if (ti != 0.0) {
                const double w0 =
                    ti * (((part[lane] + part[128 + lane]) + part[256 + lane]) + part[384 + lane]);
                const double w1 =
                    ti * (((part[64 + lane] + part[192 + lane]) + part[320 + lane]) + part[448 + lane]);
                nx = qrl_axpy(c0, ci, w0, rb, re, i + 1);
                if (wave == 0) c0[i] -= w0 * v0;
                if (a1) {
                    (void)qrl_axpy(c1, ci, w1, rb, re, m);
                    if (wave == 0) c1[i] -= w1 * v0;
                }
            } else {
                for (int r = rb; r < re; ++r)
                    if (r > i + 1) nx += c0[r] * c0[r];
            }
        } else {
            const QRLanes L = qrl_lanes(n - i - 1, lane, rb, re);
            double* ck = As + (int64_t)(L.act ? i + 1 + L.c : i) * ld;
            if (ti != 0.0) {
                double p = 0.0;
                if (L.act) {
                    if (wave == 0 && L.s == 0) p = v0 * ck[i];
                    p += qrl_dot(ci, ck, L.sb, L.se);
                }
                p = qrl_slices_sum(p, L.ncp);
                if (L.s == 0) part[wave * 128 + L.c] = p;
            }
            __syncthreads();
            if (ti != 0.0) {
                const double w =
                    ti * (((part[L.c] + part[128 + L.c]) + part[256 + L.c]) + part[384 + L.c]);
                if (L.act) {
                    nx = qrl_axpy(ck, ci, w, L.sb, L.se, i + 1);
                    if (wave == 0 && L.s == 0) ck[i] -= w * v0;
                }
            } else if (L.act) {
                for (int r = L.sb; r < L.se; ++r)
                    if (r > i + 1) nx += ck[r] * ck[r];
            }
            nx = qrl_slices_sum(nx, L.ncp);
        }
        if (lane == 0) red[wave] = nx;   // lane 0 holds column i + 1
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += 256) {
        const int r = e / n, c = e % n;
        const double v = c > r ? As[(int64_t)c * ld + r] : (c == r ? dg[r] : 0.0);
        Mt.r[r * Mt.rrs + c * Mt.rcs] = dg[r] < 0.0 ? -v : v;
    }
    __syncthreads();
    // Q in place: step i turns columns k > i (rows > i hold H_i+1 ... e_k,
    // row i still R) into H_i applied to them, then column i into H_i e_i
    for (int i = n - 1; i >= 0; --i) {
        double* ci = As + (int64_t)i * ld;
        const double ti = tau[i], v0 = vd[i];
        int rb, re;
        qrl_rows(i + 1, m, wave, rb, re);
        if (n - i - 1 > 64) {
            const int k0 = i + 1 + lane, k1 = k0 + 64;
            const bool a1 = k1 < n;
            double* c0 = As + (int64_t)k0 * ld;
            double* c1 = As + (int64_t)(a1 ? k1 : i) * ld;
            if (ti != 0.0) {
                part[wave * 128 + lane] = qrl_dot(ci, c0, rb, re);
                part[wave * 128 + 64 + lane] = qrl_dot(ci, c1, rb, re);
            }
            __syncthreads();
            if (ti != 0.0) {
                const double w0 =
                    ti * (((part[lane] + part[128 + lane]) + part[256 + lane]) + part[384 + lane]);
                const double w1 =
                    ti * (((part[64 + lane] + part[192 + lane]) + part[320 + lane]) + part[448 + lane]);
                (void)qrl_axpy(c0, ci, w0, rb, re, m);
                if (wave == 0) c0[i] = -w0 * v0;
                if (a1) {
                    (void)qrl_axpy(c1, ci, w1, rb, re, m);
                    if (wave == 0) c1[i] = -w1 * v0;
                }
            } else if (wave == 0) {
                c0[i] = 0.0;
                if (a1) c1[i] = 0.0;
            }
        } else {
            const QRLanes L = qrl_lanes(n - i - 1, lane, rb, re);
            double* ck = As + (int64_t)(L.act ? i + 1 + L.c : i) * ld;
            if (ti != 0.0) {
                double p = L.act ? qrl_dot(ci, ck, L.sb, L.se) : 0.0;
                p = qrl_slices_sum(p, L.ncp);
                if (L.s == 0) part[wave * 128 + L.c] = p;
            }
            __syncthreads();
            if (ti != 0.0) {
                const double w =
                    ti * (((part[L.c] + part[128 + L.c]) + part[256 + L.c]) + part[384 + L.c]);
                if (L.act) {
                    (void)qrl_axpy(ck, ci, w, L.sb, L.se, m);
                    if (wave == 0 && L.s == 0) ck[i] = -w * v0;
                }
            } else if (wave == 0 && L.s == 0 && L.act) {
                ck[i] = 0.0;
            }
        }
        __syncthreads();
        // column i: H_i e_i (every row of it is read above, by every wave)
        for (int r = tid; r < m; r += 256) {
            double q;
            if (r < i) q = 0.0;
            else if (r == i) q = 1.0 - ti * v0 * v0;
            else q = -ti * v0 * ci[r];
            ci[r] = q;
        }
        __syncthreads();
    }
    for (int e = tid; e < m * n; e += 256) {
        const int c = e / m, r = e - c * m;
        const double q = As[c * ld + r];
        Mt.a[(int64_t)c * ldg + r] = dg[c] < 0.0 ? -q : q;
    }
}

void launch_qr_lds(const QRMat* mats, int nmats, size_t lds, hipStream_t s) {
    if (nmats <= 0) return;
    (void)hipFuncSetAttribute((const void*)k_qr_lds, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_qr_lds, dim3(nmats), dim3(256), lds, s, mats);
}

void launch_chol_inv(const CholMat* mats, int nmats, int maxn, hipStream_t s) {
    if (nmats <= 0) return;
    const size_t lds = (size_t)2 * maxn * (maxn + 1) * sizeof(double);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_chol_inv, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    hipLaunchKernelGGL(k_chol_inv, dim3(nmats), dim3(256), lds, s, mats);
}

void launch_qr(const QRMat* mats, int nmats, int64_t maxrows, int maxcols, hipStream_t s) {
    if (nmats <= 0) return;
    if (maxrows <= QR_ROWS && maxcols <= QR_COLS) {
        hipLaunchKernelGGL(k_householder_qr, dim3(nmats), dim3(256), 0, s, mats);
        return;
    }
    const size_t lds = (size_t)(2 * maxcols + 4) * sizeof(double);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_householder_qr_wide,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_householder_qr_wide, dim3(nmats), dim3(256), lds, s, mats);
}

// ---------------------------------------------------------------------
// local expectation values: out[c] = sum_i rho_ii rows[i][c], c < 7
// ---------------------------------------------------------------------
__global__ void k_site_expect(const double* __restrict__ rho, const int64_t* __restrict__ diag_pos,
                              const signed char* __restrict__ rows, int d, double* __restrict__ out) {
    __shared__ double acc[7][64];
    const int t = threadIdx.x;
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = t; i < d; i += 64) {
        const double w = rho[diag_pos[i]];
        for (int c = 0; c < 7; ++c) s[c] += w * rows[i * 7 + c];
    }
    for (int c = 0; c < 7; ++c) acc[c][t] = s[c];
    __syncthreads();
    if (t < 7) {
        double v = 0.0;
        for (int i = 0; i < 64; ++i) v += acc[t][i];
        out[t] = v;
    }
}

void launch_site_expect(const double* rho, const int64_t* diag_pos, const signed char* rows, int d,
                        double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_site_expect, dim3(1), dim3(64), 0, s, rho, diag_pos, rows, d, out);
}

}  // namespace qed

namespace qed {

// ---------------------------------------------------------------------
// adjoint helpers
// ---------------------------------------------------------------------
void launch_bf16_to_f64(const void* a, double* b, int64_t n, double f, hipStream_t s);

// dst block (cols x rows) = transpose of src block (rows x cols), one
// workgroup per block; blk = {src_off, dst_off, rows, cols}
__global__ void k_transpose_blocks(const double* __restrict__ src, double* __restrict__ dst,
                                   const int64_t* __restrict__ blk) {
    const int64_t so = blk[4 * blockIdx.x], d0 = blk[4 * blockIdx.x + 1];
    const int rows = (int)blk[4 * blockIdx.x + 2], cols = (int)blk[4 * blockIdx.x + 3];
    for (int64_t e = threadIdx.x; e < (int64_t)rows * cols; e += blockDim.x) {
        const int r = (int)(e / cols), c = (int)(e % cols);
        dst[d0 + (int64_t)c * rows + r] = src[so + e];
    }
}

void launch_transpose_blocks(const double* src, double* dst, const int64_t* blk, int nblk,
                             hipStream_t s) {
    if (nblk <= 0) return;
    hipLaunchKernelGGL(k_transpose_blocks, dim3(nblk), dim3(256), 0, s, src, dst, blk);
}

// Scaling pass of the adjoint: blockIdx.y selects the segment.
__global__ __launch_bounds__(256) void k_adj_scale(const AdjSeg* __restrict__ segs) {
    const AdjSeg S = segs[blockIdx.y];
    if (!S.dst) return;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < S.n; i += (int64_t)gridDim.x * 256)
        S.dst[i] = S.scale * S.src[i];
}

// Dot pass: one workgroup per segment, strided partial sums and a fixed
// tree, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_adj_dots(const AdjSeg* __restrict__ segs, double* out) {
    const AdjSeg S = segs[blockIdx.x];
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < S.n; i += 256) acc += S.src[i] * S.a[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && S.dot >= 0) out[S.dot] = red[0];
}

void launch_adj_scale(const AdjSeg* segs, int nseg, int64_t maxn, hipStream_t s) {
    if (nseg <= 0 || maxn <= 0) return;
    const int g = (int)std::min<int64_t>(256, (maxn + 255) / 256);
    hipLaunchKernelGGL(k_adj_scale, dim3(g, nseg), dim3(256), 0, s, segs);
}

void launch_adj_dots(const AdjSeg* segs, int nseg, double* out, hipStream_t s) {
    if (nseg <= 0) return;
    hipLaunchKernelGGL(k_adj_dots, dim3(nseg), dim3(256), 0, s, segs, out);
}

template <typename S>
__global__ void k_scale_to_f64(const S* __restrict__ a, double* __restrict__ b, int64_t n, double f) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = f * (double)a[i];
}

void launch_scale_to_f64(const void* a, int dtype, double* b, int64_t n, double f, hipStream_t s) {
    if (n <= 0) return;
    if (dtype == QED_BF16) {
        launch_bf16_to_f64(a, b, n, f, s);
        return;
    }
    const int g = (int)std::min<int64_t>(2048, (n + 255) / 256);
    if (dtype == QED_FP32)
        hipLaunchKernelGGL(k_scale_to_f64<float>, dim3(g), dim3(256), 0, s, (const float*)a, b, n, f);
    else
        hipLaunchKernelGGL(k_scale_to_f64<double>, dim3(g), dim3(256), 0, s, (const double*)a, b, n, f);
}

}  // namespace qed
