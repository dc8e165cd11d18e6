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

template <typename P>
__device__ __forceinline__ P* at(const GRef& r, const Bases& bs) {
    if (r.tag == TAG_ABS) return (P*)r.abs;
    return (P*)bs.b[r.tag] + r.off;
}

// K advances in chunks of KB = 32, one MFMA depth.  LDS holds the chunk
// row-major with k contiguous (As[m][k], Bs[n][k]) so that every lane reads
// its 8 consecutive k of one row as a single 16-byte access; rows are
// padded by 8 elements to spread the rows over the banks.
constexpr int KB = 32;
constexpr int KP = KB + 8;

template <int WM, int WN, int BM, int BN>
__global__ __launch_bounds__(256) void k_brgemm_bf16(const GJob* __restrict__ jobs,
                                                     const GProd* __restrict__ prods,
                                                     const GTile* __restrict__ tiles, Bases bases) {
    constexpr int TM = 16 * WM * BM, TN = 16 * WN * BN;
    constexpr int AE = TM * KB / 256;
    constexpr int BE = TN * KB / 256;
    __shared__ __attribute__((aligned(16))) uint16_t As[TM][KP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][KP];
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
    int bcol[BE];
    for (int p = J.p0; p < J.p1; ++p) {
        const GProd P = prods[p];
        const uint16_t* Bb = at<const uint16_t>(P.B, bases) + (int64_t)tl.b * P.bsB;
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
        const uint16_t* Ab = at<const uint16_t>(P.A, bases) + (int64_t)tl.b * P.bsA;
        const bool scale = alpha != 1.0f;
        const int nchunk = (P.K + KB - 1) / KB;
        if (!P.tB) {
#pragma unroll
            for (int e = 0; e < BE; ++e) {
                const int gn = n0 + (tid + e * 256) % TN;
                bcol[e] = P.nsb ? (int)((gn / P.nsb) * P.nob + gn % P.nsb) : gn;
            }
        }
        for (int r = 0; r < P.nred; ++r) {
            const uint16_t* A = Ab + (int64_t)r * P.rsA;
            const uint16_t* B = Bb + (int64_t)r * P.rsB;
            auto fetch = [&](int k0) {
#pragma unroll
                for (int e = 0; e < AE; ++e) {
                    const int idx = tid + e * 256;
                    int m, k;
                    if (P.tA) { m = idx % TM; k = idx / TM; }
                    else { k = idx % KB; m = idx / KB; }
                    const int gm = m0 + m, gk = k0 + k;
                    uint16_t v = 0;
                    if (gm < J.M && gk < P.K)
                        v = P.tA ? A[(int64_t)gk * P.lda + gm] : A[(int64_t)gm * P.lda + gk];
                    ra[e] = scale ? f2bf(alpha * bf2f(v)) : v;
                }
#pragma unroll
                for (int e = 0; e < BE; ++e) {
                    const int idx = tid + e * 256;
                    int k, n;
                    if (P.tB) { k = idx % KB; n = idx / KB; }
                    else { n = idx % TN; k = idx / TN; }
                    const int gn = n0 + n, gk = k0 + k;
                    uint16_t v = 0;
                    if (gn < J.N && gk < P.K)
                        v = P.tB ? B[(int64_t)gn * P.ldb + gk] : B[(int64_t)gk * P.ldb + bcol[e]];
                    rb[e] = v;
                }
            };
            auto stash = [&]() {
#pragma unroll
                for (int e = 0; e < AE; ++e) {
                    const int idx = tid + e * 256;
                    int m, k;
                    if (P.tA) { m = idx % TM; k = idx / TM; }
                    else { k = idx % KB; m = idx / KB; }
                    As[m][k] = ra[e];
                }
#pragma unroll
                for (int e = 0; e < BE; ++e) {
                    const int idx = tid + e * 256;
                    int k, n;
                    if (P.tB) { k = idx % KB; n = idx / KB; }
                    else { n = idx % TN; k = idx / TN; }
                    Bs[n][k] = rb[e];
                }
            };
            fetch(0);
            for (int c = 0; c < nchunk; ++c) {
                __syncthreads();
                stash();
                __syncthreads();
                if (c + 1 < nchunk) fetch((c + 1) * KB);
                bf16x8 a[BM], b[BN];
#pragma unroll
                for (int i = 0; i < BM; ++i)
                    a[i] = __builtin_bit_cast(bf16x8, *(const u16x8*)&As[wm0 + i * 16 + lr][8 * lk]);
#pragma unroll
                for (int j = 0; j < BN; ++j)
                    b[j] = __builtin_bit_cast(bf16x8, *(const u16x8*)&Bs[wn0 + j * 16 + lr][8 * lk]);
#pragma unroll
                for (int i = 0; i < BM; ++i)
#pragma unroll
                    for (int j = 0; j < BN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
    }
    uint16_t* C = at<uint16_t>(J.C, bases) + (int64_t)tl.b * J.bsC;
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
                    uint16_t* c = C + (int64_t)row * J.ldc + co;
                    *c = f2bf(J.acc ? bf2f(*c) + acc[bi][bj][i] : acc[bi][bj][i]);
                }
            }
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

void launch_f64_to_bf16(const double* a, void* b, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_f64_to_bf16, dim3(grid_of(n)), dim3(256), 0, st, a, (uint16_t*)b, n);
}

void launch_bf16_to_f64(const void* a, double* b, int64_t n, double f, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bf16_to_f64, dim3(grid_of(n)), dim3(256), 0, st, (const uint16_t*)a, b, n, f);
}

}  // namespace qed
