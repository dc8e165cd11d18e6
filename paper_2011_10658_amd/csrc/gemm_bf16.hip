// Grouped batch-reduce GEMM with bfloat16 operands and FP32 accumulation
// (MFMA 16x16x32 bf16 on CDNA4), the same job/product/tile contract as the
// FP32 and FP64 kernels: C[job] (+)= sum_p alpha_p op(A_p) op(B_p), every
// output element written by exactly one workgroup.  Storage is raw
// bfloat16 bits (uint16_t); results are rounded to nearest even once, when
// the FP32 accumulator is stored.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace qed {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// blocks in device (global) memory: global rather than flat loads and
// stores, so that the MFMA loop's LDS waits do not also wait for the next
// chunk's operand prefetch (flat loads count against the LDS counter)
template <typename P>
using gmem = __attribute__((address_space(1))) P;

template <typename P>
__device__ __forceinline__ gmem<P>* at(const GRef& r, const Bases& bs) {
    if (r.tag == TAG_ABS) return (gmem<P>*)r.abs;
    return (gmem<P>*)bs.b[r.tag] + r.off;
}

// K advances in chunks of KB = 32, one MFMA depth.  LDS holds the chunk
// row-major with k contiguous (As[m][k], Bs[n][k]) so that every lane reads
// its 8 consecutive k of one row as a single 16-byte access; rows are
// padded by 8 elements to spread the rows over the banks.  The stage is
// double-buffered (one barrier per chunk) and every thread's elements sit
// at fixed strides from its first one (all tile extents divide 256).
constexpr int KB = 32;
constexpr int KP = KB + 8;

// Occupancy hint of four waves per SIMD (three otherwise): the compiler
// keeps 128 VGPRs with a 12-byte spill in the 128x32 and 32x128 instances;
// measured 7% faster on the BF16 sweep.
template <int WM, int WN, int BM, int BN>
__global__ __launch_bounds__(256, 4) void k_brgemm_bf16(const GJob* __restrict__ jobs,
                                                     const GProd* __restrict__ prods,
                                                     const GTile* __restrict__ tiles, Bases bases) {
    constexpr int TM = 16 * WM * BM, TN = 16 * WN * BN;
    constexpr int AE = TM * KB / 256;
    constexpr int BE = TN * KB / 256;
    __shared__ __attribute__((aligned(16))) uint16_t As[2][TM][KP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][TN][KP];
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
    f32x4 acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    uint16_t ra[AE], rb[BE];
    constexpr int ASA = 256 / KB, ASB = 256 / TM;
    constexpr int BSB = 256 / KB, BSN = 256 / TN;
    const int t_kc = tid % KB, t_kq = tid / KB;
    const int t_tm = tid % TM, t_tq = tid / TM;
    const int t_tn = tid % TN, t_nq = tid / TN;
    for (int p = J.p0; p < J.p1; ++p) {
        const GProd P = prods[p];
        gmem<const uint16_t>* Bb = at<const uint16_t>(P.B, bases) + (int64_t)tl.b * P.bsB;
        const float alpha = (float)P.alpha;
        if (P.ident) {
#pragma unroll
            for (int bi = 0; bi < BM; ++bi)
#pragma unroll
                for (int bj = 0; bj < BN; ++bj) {
                    const int col = n0 + wn0 + bj * 16 + lr;
                    const int64_t co = P.nsb ? (int64_t)(col / P.nsb) * P.nob + col % P.nsb : col;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = m0 + wm0 + bi * 16 + 4 * lk + i;
                        if (row < J.M && col < J.N)
                            acc[bi][bj][i] += alpha * bf2f(Bb[(int64_t)row * P.ldb + co]);
                    }
                }
            continue;
        }
        gmem<const uint16_t>* Ab = at<const uint16_t>(P.A, bases) + (int64_t)tl.b * P.bsA;
        const bool scale = alpha != 1.0f;
        const int nchunk = (P.K + KB - 1) / KB;
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
            gmem<const uint16_t>* A = Ab + (int64_t)r * P.rsA + abase;
            gmem<const uint16_t>* B = Bb + (int64_t)r * P.rsB + bbase;
            auto fetch = [&](int c) {
                const int k0 = c * KB;
                gmem<const uint16_t>* pa = A + k0 * akm;
                gmem<const uint16_t>* pb = B + k0 * bkm;
#pragma unroll
                for (int e = 0; e < AE; ++e) {
                    uint16_t v = 0;
                    if (m0 + am0 + e * amE < J.M && k0 + ak0 + e * akE < P.K) v = pa[e * aes];
                    ra[e] = v;
                }
#pragma unroll
                for (int e = 0; e < BE; ++e) {
                    uint16_t v = 0;
                    if (n0 + bn0 + e * bnE < J.N && k0 + bk0 + e * bkE < P.K) v = pb[e * bes];
                    rb[e] = v;
                }
            };
            // the scaling is applied here, not at the load: a use right after
            // the load would make the prefetch wait before the MFMAs; the
            // empty asm statements (no instruction) hold the loaded values
            // until this point
            auto stash = [&](int buf) {
#pragma unroll
                for (int e = 0; e < AE; ++e) {
                    uint32_t t = ra[e];
                    asm volatile("" : "+v"(t));
                    ra[e] = (uint16_t)t;
                }
#pragma unroll
                for (int e = 0; e < BE; ++e) {
                    uint32_t t = rb[e];
                    asm volatile("" : "+v"(t));
                    rb[e] = (uint16_t)t;
                }
#pragma unroll
                for (int e = 0; e < AE; ++e)
                    As[buf][am0 + e * amE][ak0 + e * akE] = scale ? f2bf(alpha * bf2f(ra[e])) : ra[e];
#pragma unroll
                for (int e = 0; e < BE; ++e) Bs[buf][bn0 + e * bnE][bk0 + e * bkE] = rb[e];
            };
            __syncthreads();
            fetch(0);
            stash(0);
            __syncthreads();
            for (int c = 0; c < nchunk; ++c) {
                const int cur = c & 1;
                if (c + 1 < nchunk) fetch(c + 1);
                bf16x8 a[BM], b[BN];
#pragma unroll
                for (int i = 0; i < BM; ++i)
                    a[i] = __builtin_bit_cast(bf16x8, *(const u16x8*)&As[cur][wm0 + i * 16 + lr][8 * lk]);
#pragma unroll
                for (int j = 0; j < BN; ++j)
                    b[j] = __builtin_bit_cast(bf16x8, *(const u16x8*)&Bs[cur][wn0 + j * 16 + lr][8 * lk]);
#pragma unroll
                for (int i = 0; i < BM; ++i)
#pragma unroll
                    for (int j = 0; j < BN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
                if (c + 1 < nchunk) stash(cur ^ 1);
                __syncthreads();
            }
        }
    }
    gmem<uint16_t>* C = at<uint16_t>(J.C, bases) + (int64_t)tl.b * J.bsC;
#pragma unroll
    for (int bi = 0; bi < BM; ++bi)
#pragma unroll
        for (int bj = 0; bj < BN; ++bj) {
            const int col = n0 + wn0 + bj * 16 + lr;
            const int64_t co = J.nsc ? (int64_t)(col / J.nsc) * J.noc + col % J.nsc : col;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + wm0 + bi * 16 + 4 * lk + i;
                if (row < J.M && col < J.N) {
                    gmem<uint16_t>* c = C + (int64_t)row * J.ldc + co;
                    *c = f2bf(J.acc ? bf2f(*c) + acc[bi][bj][i] : acc[bi][bj][i]);
                }
            }
        }
}

// identity-only stage (see k_sum_stage): BF16 storage, FP32 sums
__global__ __launch_bounds__(256) void k_sum_stage_bf16(const GJob* __restrict__ jobs,
                                                        const GProd* __restrict__ prods,
                                                        const GTile* __restrict__ tiles, Bases bases) {
    const GTile tl = tiles[blockIdx.x];
    if (tl.job < 0) return;
    const GJob J = jobs[tl.job];
    const int64_t total = (int64_t)J.M * J.N;
    const int64_t e0 = (int64_t)tl.tm * SUM_TILE;
    const int64_t e1 = e0 + SUM_TILE < total ? e0 + SUM_TILE : total;
    gmem<uint16_t>* C = at<uint16_t>(J.C, bases) + (int64_t)tl.b * J.bsC;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        const int row = (int)(e / J.N), col = (int)(e % J.N);
        float acc = 0.0f;
        for (int p = J.p0; p < J.p1; ++p) {
            const GProd P = prods[p];
            gmem<const uint16_t>* Bb = at<const uint16_t>(P.B, bases) + (int64_t)tl.b * P.bsB;
            const int64_t co = P.nsb ? (int64_t)(col / P.nsb) * P.nob + col % P.nsb : col;
            acc += (float)P.alpha * bf2f(Bb[(int64_t)row * P.ldb + co]);
        }
        const int64_t cc = J.nsc ? (int64_t)(col / J.nsc) * J.noc + col % J.nsc : col;
        gmem<uint16_t>* c = C + (int64_t)row * J.ldc + cc;
        *c = f2bf(J.acc ? bf2f(*c) + acc : acc);
    }
}

__global__ void k_f64_to_bf16(const double* __restrict__ a, uint16_t* __restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = f2bf((float)a[i]);
}

__global__ void k_bf16_to_f64(const uint16_t* __restrict__ a, double* __restrict__ b, int64_t n,
                              double f) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = f * (double)bf2f(a[i]);
}

int grid_of(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

void launch_brgemm_bf16(const GJob* jobs, const GProd* prods, const GTile* tiles, int ntiles,
                        const Bases& bases, int shape, hipStream_t st) {
    if (ntiles <= 0) return;
    switch (shape) {
        case GEMM_SHAPE_TALL:
            hipLaunchKernelGGL((k_brgemm_bf16<4, 1, 2, 2>), dim3(ntiles), dim3(256), 0, st, jobs, prods, tiles, bases);
            break;
        case GEMM_SHAPE_WIDE:
            hipLaunchKernelGGL((k_brgemm_bf16<1, 4, 2, 2>), dim3(ntiles), dim3(256), 0, st, jobs, prods, tiles, bases);
            break;
        default:
            hipLaunchKernelGGL((k_brgemm_bf16<2, 2, 2, 2>), dim3(ntiles), dim3(256), 0, st, jobs, prods, tiles, bases);
    }
}

void launch_sum_stage_bf16(const GJob* jobs, const GProd* prods, const GTile* tiles, int ntiles,
                           const Bases& bases, hipStream_t st) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_sum_stage_bf16, dim3(ntiles), dim3(256), 0, st, jobs, prods, tiles, bases);
}

void launch_f64_to_bf16(const double* a, void* b, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_f64_to_bf16, dim3(grid_of(n)), dim3(256), 0, st, a, (uint16_t*)b, n);
}

void launch_bf16_to_f64(const void* a, double* b, int64_t n, double f, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bf16_to_f64, dim3(grid_of(n)), dim3(256), 0, st, (const uint16_t*)a, b, n, f);
}

}  // namespace qed
