// Fused H_eff stage for gfx950 (CDNA4, wave64, 16x16x4 MFMA).
//
// The effective Hamiltonian of a node is a sum of products of leg
// operators (Methods, "Tensor Networks", step (i)).  Most of its terms
// carry a factor C on the bond leg p, whose sectors are short (tens of
// states), together with a factor F on a child leg, whose sectors are long
// (up to 141 states per dressed-site charge).  Applying C in a stage of its
// own writes one node-sized intermediate per term and block to HBM and
// reads it back, at a few flops per byte.  Here one workgroup owns a tile
// of the output block (64 rows of the child leg times ng groups of the
// other child leg's index, each group a full bond sector) and runs every
// term of that block through it:
//   W = alpha F X          MFMA over the long child sector (K up to 141),
//                          accumulated in registers,
//   W -> LDS,
//   Y += W (I (x) C^T)     MFMA over the short bond sector, one block of
//                          16 output columns never straddles a group
//                          because groups are padded to 16 columns in Y.
// Y stays in registers across all terms and is written once.  Terms without
// a bond factor add W directly (remapped from dense to padded groups), and
// an identity F loads X straight into the W tile.
//
// Tile: 64 rows (wave w owns rows 16w..16w+15 and every column block), W
// up to WC dense columns, Y up to WC padded columns.  K advances in chunks
// of 16 staged in LDS (F m-major, X k-major, both double-buffered; the
// paddings make the MFMA operand reads free of bank conflicts); the W tile
// reuses the stage's LDS, and each term's bond factor is copied into LDS
// (transposed) when the term starts.  The next term's first chunk is
// fetched from global memory while the current term's epilogue runs.  Row
// blocks beyond M and column blocks beyond the tile's groups skip their
// MFMAs.  Global loads are issued in batches held in registers, so their
// latencies overlap.
#include <algorithm>

#include "kernels.h"

namespace qed {

template <typename T> struct FMfma;

// operand layout of both 16x16x4 instructions: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator item i of lane l is
// row 4 (l / 16) + i (FP32) or 4 i + l / 16 (FP64), column l % 16
template <> struct FMfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 step(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <> struct FMfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 step(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return 4 * i + (lane >> 4); }
};

// compile-time count for the column-block loops: a runtime guard on
// every MFMA of an unrolled loop makes the compiler keep all guarded
// accumulators alive in select form (hundreds of spilled registers), so
// each loop runs as one of eight instances chosen by a switch
template <int N> struct IC {
    static constexpr int value = N;
};
#define QED_FUSED_DISPATCH(n, f)          \
    switch (n) {                          \
        case 1: f(IC<1>{}); break;        \
        case 2: f(IC<2>{}); break;        \
        case 3: f(IC<3>{}); break;        \
        case 4: f(IC<4>{}); break;        \
        case 5: f(IC<5>{}); break;        \
        case 6: f(IC<6>{}); break;        \
        case 7: f(IC<7>{}); break;        \
        case 8: f(IC<8>{}); break;        \
        default: break;                   \
    }

// the same for the epilogues, on (groups of the tile, 16-column blocks per
// group): accumulator j = g Q + jj covers group g, columns 16 jj..
#define QED_FUSED_DISPATCH_GQ(q, ng, f)   \
    switch ((q) * 16 + (ng)) {            \
        case 17: f(IC<1>{}, IC<1>{}); break;        \
        case 18: f(IC<2>{}, IC<1>{}); break;        \
        case 19: f(IC<3>{}, IC<1>{}); break;        \
        case 20: f(IC<4>{}, IC<1>{}); break;        \
        case 21: f(IC<5>{}, IC<1>{}); break;        \
        case 22: f(IC<6>{}, IC<1>{}); break;        \
        case 23: f(IC<7>{}, IC<1>{}); break;        \
        case 24: f(IC<8>{}, IC<1>{}); break;        \
        case 33: f(IC<1>{}, IC<2>{}); break;        \
        case 34: f(IC<2>{}, IC<2>{}); break;        \
        case 35: f(IC<3>{}, IC<2>{}); break;        \
        case 36: f(IC<4>{}, IC<2>{}); break;        \
        case 49: f(IC<1>{}, IC<3>{}); break;        \
        case 50: f(IC<2>{}, IC<3>{}); break;        \
        case 65: f(IC<1>{}, IC<4>{}); break;        \
        case 66: f(IC<2>{}, IC<4>{}); break;        \
        case 81: f(IC<1>{}, IC<5>{}); break;        \
        case 97: f(IC<1>{}, IC<6>{}); break;        \
        case 113: f(IC<1>{}, IC<7>{}); break;        \
        case 129: f(IC<1>{}, IC<8>{}); break;        \
        default: break;                   \
    }

// blocks in device (global) memory: global rather than flat loads, so that
// the LDS waits of the MFMA loops and epilogues do not also wait for the
// operand prefetch (flat loads count against the LDS counter)
template <typename T>
using gmem = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ gmem<const T>* fres(const GRef& r, const Bases& bs) {
    if (r.tag == TAG_ABS) return (gmem<const T>*)r.abs;
    return (gmem<const T>*)bs.b[r.tag] + r.off;
}

template <typename T, int WC>
__global__ __launch_bounds__(256, 3) void k_heff_fused(const FJob* __restrict__ jobs,
                                                      const FProd* __restrict__ prods,
                                                      const GTile* __restrict__ tiles, Bases bases,
                                                      int cs_ld) {
    typedef typename FMfma<T>::v4 v4;
    constexpr int KC = 16;
    constexpr int TM = FUSED_TM;
    constexpr int NB = WC / 16;              // column blocks of W and of Y
    constexpr int LDA = KC + 2;              // F stage: m-major rows of KC (+2)
    constexpr int LDX = WC + 16;             // X stage: k-major rows of WC (+16)
    constexpr int LDW = WC + 2;              // W tile: row-major rows of WC (+2)
    constexpr int A_WORDS = TM * LDA;
    constexpr int X_WORDS = KC * LDX;
    constexpr int STAGE = 2 * (A_WORDS + X_WORDS);
    constexpr int WTILE = TM * LDW;
    constexpr int UNION = STAGE > WTILE ? STAGE : WTILE;
    constexpr int AE = TM * KC / 256;        // F elements per thread and chunk
    constexpr int XR = 256 / WC;             // X rows covered by one pass of the threads
    constexpr int XE = KC / XR;              // X elements per thread and chunk
    constexpr int IB = 8;                    // identity-F rows loaded per batch and thread
    constexpr int CE = 8;                    // bond-factor elements per thread and batch
    // dynamic LDS: the operand stage / W tile union, then the bond factor of
    // the current product, transposed (row k = input bond index, cs_ld
    // columns), so its MFMA operand reads are conflict-free
    extern __shared__ __align__(16) unsigned char smem[];
    T* lds = (T*)smem;
    T* Cs = lds + UNION;

    const GTile tl = tiles[blockIdx.x];
    if (tl.job < 0) return;   // padding of the XCD-ordered tile list
    const FJob J = jobs[tl.job];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int m0 = tl.tm * TM;
    const int g0 = tl.tn * J.ng;
    const int ngv = J.ng < J.G - g0 ? J.ng : J.G - g0;   // groups of this tile
    const int p16 = (J.np + 15) & ~15;
    const int q16 = p16 / 16;                            // column blocks per group
    const int nyb = ngv * q16;                           // Y column blocks in use
    const int wr0 = 16 * wave;                           // this wave's rows in the tile
    const bool wrows = m0 + wr0 < J.M;

    v4 accy[NB], accw[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) accy[j] = v4{0, 0, 0, 0};

    // per-thread fetch coordinates: F element (row fm + 16 e, column fk) of
    // a chunk; X element (row xk + XR e, column xc) of a chunk
    const int fk = tid % KC, fm = tid / KC;
    const int xc = tid % WC, xk = tid / WC;
    T ra[AE], rx[XE];

    // operand pointers of the product being fetched
    struct Src {
        gmem<const T>* F;   // row fm, column fk of chunk 0 (rows m0 + fm)
        gmem<const T>* X;   // row xk, column xc of chunk 0
        int64_t fes;     // F stride between this thread's elements
        int64_t xkm;     // X stride per k row
        int K, nchunk;
        bool xok;        // this thread's X column is inside the tile's groups
        T alpha;
    };
    Src S{};   // the product whose chunks are fetched
    auto describe = [&](const FProd& P, Src& S) {
        gmem<const T>* Fb = fres<T>(P.F, bases);
        gmem<const T>* Xb = fres<T>(P.X, bases);
        S.F = Fb + (int64_t)(m0 + fm) * P.lda + fk;
        S.fes = (int64_t)16 * P.lda;
        S.xok = xc < ngv * P.np_in;
        const int g = xc / P.np_in, cc = xc - g * P.np_in;
        S.X = Xb + (int64_t)xk * P.ldx + (int64_t)(g0 + g) * P.gox + cc;
        S.xkm = P.ldx;
        S.K = P.K;
        S.nchunk = (P.K + KC - 1) / KC;
        S.alpha = (T)P.alpha;
    };
    auto fetch = [&](const Src& S, int c) {
        const int k0 = c * KC;
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            T v = (T)0;
            if (m0 + fm + 16 * e < J.M && k0 + fk < S.K) v = S.F[e * S.fes + k0];
            ra[e] = v;
        }
#pragma unroll
        for (int e = 0; e < XE; ++e) {
            T v = (T)0;
            if (S.xok && k0 + xk + XR * e < S.K) v = S.X[(int64_t)(k0 + XR * e) * S.xkm];
            rx[e] = v;
        }
    };
    // the product's alpha is applied here, not at the load: a use right after
    // the load would make the prefetch wait before the work it overlaps; the
    // empty asm statements (no instruction) hold the loaded values until now.
    // S describes the fetched chunk's product whenever a chunk is stashed.
    auto stash = [&](int buf) {
#pragma unroll
        for (int e = 0; e < AE; ++e) asm volatile("" : "+v"(ra[e]));
#pragma unroll
        for (int e = 0; e < XE; ++e) asm volatile("" : "+v"(rx[e]));
        T* As = lds + buf * (A_WORDS + X_WORDS);
        T* Xs = As + A_WORDS;
#pragma unroll
        for (int e = 0; e < AE; ++e) As[(fm + 16 * e) * LDA + fk] = ra[e] * S.alpha;
#pragma unroll
        for (int e = 0; e < XE; ++e) Xs[(xk + XR * e) * LDX + xc] = rx[e];
    };
    // the bond factor of product P into Cs: Cs[k * cs_ld + c'] = C(c', k)
    // for k < np_in, c' < p16 (zero beyond np); loads of a batch in flight
    // together
    auto load_c = [&](const FProd& P) {
        gmem<const T>* Cb = fres<T>(P.Cb, bases);
        const int npi = P.np_in, n = npi * p16;
        for (int base = 0; base < n; base += 256 * CE) {
            T cr[CE];
#pragma unroll
            for (int e = 0; e < CE; ++e) {
                const int idx = base + tid + 256 * e;
                T v = (T)0;
                if (idx < n) {
                    const int k = idx / p16, cp = idx - k * p16;
                    if (cp < J.np) v = Cb[(int64_t)cp * npi + k];
                }
                cr[e] = v;
            }
#pragma unroll
            for (int e = 0; e < CE; ++e) {
                const int idx = base + tid + 256 * e;
                if (idx < n) {
                    const int k = idx / p16, cp = idx - k * p16;
                    Cs[k * cs_ld + cp] = cr[e];
                }
            }
        }
    };

    bool have = false;   // ra/rx hold the first chunk of product p
    for (int p = J.p0; p < J.p1; ++p) {
        const FProd P = prods[p];
        const int npi = P.np_in;
        const int nwb = (ngv * npi + 15) >> 4;   // W column blocks in use
        __syncthreads();   // the previous product's epilogue is done with the LDS
        if (P.hasC) load_c(P);
        if (P.identF) {
            // W = alpha X: rows m0.. of the tile straight from X; this thread
            // keeps one column and loads IB rows at a time
            gmem<const T>* Xb = fres<T>(P.X, bases);
            const T alpha = (T)P.alpha;
            const bool cok = xc < ngv * npi;
            const int g = xc / npi, cc = xc - g * npi;
            gmem<const T>* xp = Xb + (int64_t)(g0 + g) * P.gox + cc;
#pragma unroll
            for (int r0 = 0; r0 < TM; r0 += XR * IB) {
                T v[IB];
#pragma unroll
                for (int e = 0; e < IB; ++e) {
                    const int r = r0 + xk + XR * e;
                    v[e] = (cok && m0 + r < J.M) ? alpha * xp[(int64_t)(m0 + r) * P.ldx] : (T)0;
                }
#pragma unroll
                for (int e = 0; e < IB; ++e) lds[(r0 + xk + XR * e) * LDW + xc] = v[e];
            }
            __syncthreads();
        } else {
            if (!have) {
                describe(P, S);
                fetch(S, 0);
            }
            have = false;
            stash(0);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < NB; ++j) accw[j] = v4{0, 0, 0, 0};
            for (int c = 0; c < S.nchunk; ++c) {
                const int cur = c & 1;
                if (c + 1 < S.nchunk) fetch(S, c + 1);
                const T* As = lds + cur * (A_WORDS + X_WORDS);
                const T* Xs = As + A_WORDS;
                if (wrows) {
                    auto mm = [&](auto nbv) {
                        constexpr int NBV = decltype(nbv)::value;
                        if constexpr (NBV <= NB) {
#pragma unroll
                            for (int kk = 0; kk < KC; kk += 4) {
                                const T a = As[(wr0 + lr) * LDA + kk + lk];
#pragma unroll
                                for (int j = 0; j < NBV; ++j) {
                                    const T b = Xs[(kk + lk) * LDX + 16 * j + lr];
                                    accw[j] = FMfma<T>::step(a, b, accw[j]);
                                }
                            }
                        }
                    };
                    QED_FUSED_DISPATCH(nwb, mm)
                }
                if (c + 1 < S.nchunk) stash(cur ^ 1);
                __syncthreads();
            }
            // W -> LDS (the stage buffers are free after the last barrier)
            if (wrows) {
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    if (j < nwb) {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            lds[(wr0 + FMfma<T>::row(lane, i)) * LDW + 16 * j + lr] = accw[j][i];
                    }
            }
            __syncthreads();
        }
        // the next product's first chunk is fetched while this epilogue runs
        if (p + 1 < J.p1) {
            const FProd Pn = prods[p + 1];
            if (!Pn.identF) {
                describe(Pn, S);
                fetch(S, 0);
                have = true;
            }
        }
        if (!wrows) continue;
        if (P.hasC) {
            // Y(m, g, c') += sum_c W(m, g, c) C(c', c): per k step, one W
            // operand per group and one C operand per column block
            auto ep = [&](auto ngc, auto qc) {
                constexpr int G = decltype(ngc)::value, Q = decltype(qc)::value;
                if constexpr (G * Q <= NB) {
                    for (int kk = 0; kk < npi; kk += 4) {
                        const int k = kk + lk;
                        const bool kin = k < npi;
                        T a[G], b[Q];
#pragma unroll
                        for (int g = 0; g < G; ++g) a[g] = kin ? lds[(wr0 + lr) * LDW + g * npi + k] : (T)0;
#pragma unroll
                        for (int jj = 0; jj < Q; ++jj) b[jj] = kin ? Cs[k * cs_ld + 16 * jj + lr] : (T)0;
#pragma unroll
                        for (int g = 0; g < G; ++g)
#pragma unroll
                            for (int jj = 0; jj < Q; ++jj)
                                accy[g * Q + jj] = FMfma<T>::step(a[g], b[jj], accy[g * Q + jj]);
                    }
                }
            };
            QED_FUSED_DISPATCH_GQ(q16, ngv, ep)
        } else {
            // Y(m, g, c') += W(m, g, c'), dense groups of np into padded
            // ones (padding columns of Y receive values that are never
            // stored; every index stays inside the W tile)
            auto add = [&](auto ngc, auto qc) {
                constexpr int G = decltype(ngc)::value, Q = decltype(qc)::value;
                if constexpr (G * Q <= NB) {
#pragma unroll
                    for (int g = 0; g < G; ++g)
#pragma unroll
                        for (int jj = 0; jj < Q; ++jj)
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                accy[g * Q + jj][i] +=
                                    lds[(wr0 + FMfma<T>::row(lane, i)) * LDW + g * J.np + 16 * jj + lr];
                }
            };
            QED_FUSED_DISPATCH_GQ(q16, ngv, add)
        }
    }
    if (!wrows) return;
    gmem<T>* Y = (gmem<T>*)fres<T>(J.Y, bases);
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if (j < nyb) {
            const int g = (16 * j) / p16, cp = (16 * j) % p16 + lr;
            if (cp >= J.np) continue;
            gmem<T>* yg = Y + (int64_t)(g0 + g) * J.goy + cp;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + wr0 + FMfma<T>::row(lane, i);
                if (row < J.M) {
                    gmem<T>* y = yg + (int64_t)row * J.ldy;
                    *y = J.acc ? *y + accy[j][i] : accy[j][i];
                }
            }
        }
}

template <typename T>
void launch_heff_fused(const FJob* jobs, const FProd* prods, const GTile* tiles, int ntiles,
                       const Bases& bases, int cs_rows, int cs_cols, hipStream_t st) {
    if (ntiles <= 0) return;
    constexpr int WC = sizeof(T) == 4 ? FUSED_COLS_F32 : FUSED_COLS_F64;
    constexpr int KC = 16, TM = FUSED_TM;
    constexpr int STAGE = 2 * (TM * (KC + 2) + KC * (WC + 16));
    constexpr int WTILE = TM * (WC + 2);
    constexpr int UNION = STAGE > WTILE ? STAGE : WTILE;
    // bond-factor rows of cs_ld = cs_cols + 16 words (conflict-free reads)
    const int cs_ld = cs_cols + 16;
    const size_t lds = (size_t)(UNION + (size_t)std::max(cs_rows, 1) * cs_ld) * sizeof(T);
    hipLaunchKernelGGL((k_heff_fused<T, WC>), dim3(ntiles), dim3(256), lds, st, jobs, prods, tiles,
                       bases, cs_ld);
}

template void launch_heff_fused<float>(const FJob*, const FProd*, const GTile*, int, const Bases&,
                                       int, int, hipStream_t);
template void launch_heff_fused<double>(const FJob*, const FProd*, const GTile*, int, const Bases&,
                                        int, int, hipStream_t);

}  // namespace qed
