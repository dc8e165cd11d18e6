// Segmented Lanczos kernels: one independent recurrence per segment of a
// concatenated vector (many tree nodes optimised at once), in FP64; the
// basis is stored in FP64 or, for an FP32 matvec, in FP32 (TV, the basis
// element type).  Work is
// split into fixed chunks that never straddle a segment, so every
// reduction has a fixed partition and order (bitwise reproducible), and
// per-segment scalars (alpha, beta, coefficients, state) live on the
// device.  A segment that broke down skips all further updates.
#include "kernels.h"

namespace qed {

__device__ __forceinline__ double seg_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

constexpr int SROWS = 8;

// partial[r * nch + c] = sum over chunk c of V[r] . w   (r < nrows)
template <typename TV>
__global__ __launch_bounds__(256) void k_sdot_partial(const TV* __restrict__ V, int64_t ldv,
                                                      int nrows, const double* __restrict__ w,
                                                      const SegChunk* __restrict__ ch, int nch,
                                                      double* __restrict__ partial,
                                                      const LState* st, int skip) {
    const SegChunk C = ch[blockIdx.x];
    if (skip && st[C.seg].broken) return;
    __shared__ double sh[SROWS][4];
    for (int r0 = 0; r0 < nrows; r0 += SROWS) {
        double s[SROWS];
#pragma unroll
        for (int q = 0; q < SROWS; ++q) s[q] = 0.0;
        for (int64_t i = C.lo + threadIdx.x; i < C.hi; i += 256) {
            const double wi = w[i];
#pragma unroll
            for (int q = 0; q < SROWS; ++q)
                if (r0 + q < nrows) s[q] += (double)V[(int64_t)(r0 + q) * ldv + i] * wi;
        }
#pragma unroll
        for (int q = 0; q < SROWS; ++q) {
            const double v = seg_wave_sum(s[q]);
            if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x >> 6] = v;
        }
        __syncthreads();
        if ((int)threadIdx.x < SROWS && r0 + (int)threadIdx.x < nrows) {
            const int q = threadIdx.x;
            partial[(int64_t)(r0 + q) * nch + blockIdx.x] = ((sh[q][0] + sh[q][1]) + sh[q][2]) + sh[q][3];
        }
        __syncthreads();
    }
}

// out[seg * ldo + r] = sum over the segment's chunks (mode 1: sqrt);
// one workgroup per (segment, row)
__global__ __launch_bounds__(256) void k_sdot_final(const double* __restrict__ partial, int nch,
                                                    const int* __restrict__ seg_c0, int nrows,
                                                    double* __restrict__ out, int ldo, int mode,
                                                    const LState* st, int skip) {
    const int seg = blockIdx.x / nrows, r = blockIdx.x % nrows;
    if (skip && st[seg].broken) return;
    __shared__ double sh[4];
    const int c0 = seg_c0[seg], c1 = seg_c0[seg + 1];
    double s = 0.0;
    for (int c = c0 + threadIdx.x; c < c1; c += 256) s += partial[(int64_t)r * nch + c];
    s = seg_wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = ((sh[0] + sh[1]) + sh[2]) + sh[3];
        out[(int64_t)seg * ldo + r] = mode == 1 ? sqrt(t) : t;
    }
}

__global__ void k_s_init(LState* st, int nseg, int m, const double* nrm, int ldn) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    st[s].k = m;
    st[s].broken = 0;
    st[s].norm = nrm[(int64_t)s * ldn];
}

// dst = src / nrm[seg]
template <typename TV>
__global__ void k_s_start(TV* __restrict__ dst, const double* __restrict__ src,
                          const double* __restrict__ nrm, int ldn, const SegChunk* __restrict__ ch) {
    const SegChunk C = ch[blockIdx.x];
    const double inv = 1.0 / nrm[(int64_t)C.seg * ldn];
    for (int64_t i = C.lo + threadIdx.x; i < C.hi; i += 256) dst[i] = (TV)(src[i] * inv);
}

// w -= alpha[seg][j] v_j + beta[seg][j-1] v_{j-1}
__global__ void k_s_three_term(double* __restrict__ w, const double* __restrict__ V, int64_t ldv,
                               int j, const double* __restrict__ alpha,
                               const double* __restrict__ beta, int lds,
                               const SegChunk* __restrict__ ch, const LState* st) {
    const SegChunk C = ch[blockIdx.x];
    if (st[C.seg].broken) return;
    const double a = alpha[(int64_t)C.seg * lds + j];
    const double b = j > 0 ? beta[(int64_t)C.seg * lds + j - 1] : 0.0;
    const double* vj = V + (int64_t)j * ldv;
    const double* vm = V + (int64_t)(j > 0 ? j - 1 : 0) * ldv;
    for (int64_t i = C.lo + threadIdx.x; i < C.hi; i += 256) {
        double t = a * vj[i];
        if (j > 0) t += b * vm[i];
        w[i] -= t;
    }
}

// w -= sum_{r < nrows} coef[seg][r] V[r]
__global__ void k_s_subtract(double* __restrict__ w, const double* __restrict__ V, int64_t ldv,
                             int nrows, const double* __restrict__ coef, int lds,
                             const SegChunk* __restrict__ ch, const LState* st) {
    const SegChunk C = ch[blockIdx.x];
    if (st[C.seg].broken) return;
    const double* c = coef + (int64_t)C.seg * lds;
    for (int64_t i = C.lo + threadIdx.x; i < C.hi; i += 256) {
        double t = 0.0;
        for (int r = 0; r < nrows; ++r) t += c[r] * V[(int64_t)r * ldv + i];
        w[i] -= t;
    }
}

// beta[seg][j] = sqrt(ww[seg]); breakdown test against the scale of T
__global__ void k_s_beta(const double* ww, int ldw, double* alpha, double* beta, int lds, int j,
                         LState* st, int nseg, double tol) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg || st[s].broken) return;
    const double* a = alpha + (int64_t)s * lds;
    double* be = beta + (int64_t)s * lds;
    const double b = sqrt(ww[(int64_t)s * ldw]);
    double scale = 1.0;
    for (int i = 0; i <= j; ++i) scale = fmax(scale, fabs(a[i]));
    for (int i = 0; i < j; ++i) scale = fmax(scale, be[i]);
    if (b <= tol * scale) {
        be[j] = 0.0;
        st[s].broken = 1;
        st[s].k = j + 1;
    } else {
        be[j] = b;
    }
}

// V[j+1] = w / beta[seg][j]
template <typename TV>
__global__ void k_s_next(TV* __restrict__ V, int64_t ldv, int j, const double* __restrict__ w,
                         const double* __restrict__ beta, int lds, const SegChunk* __restrict__ ch,
                         const LState* st) {
    const SegChunk C = ch[blockIdx.x];
    if (st[C.seg].broken) return;
    const double inv = 1.0 / beta[(int64_t)C.seg * lds + j];
    TV* v = V + (int64_t)(j + 1) * ldv;
    for (int64_t i = C.lo + threadIdx.x; i < C.hi; i += 256) v[i] = (TV)(w[i] * inv);
}

// Fused vector update + dot products of one Lanczos step, segment by
// segment, one pass over the basis (each chunk's basis entries stay in
// registers between the update and the dots; rows <= MAXR):
//   mode 0: w -= alpha_j v_j + beta_{j-1} v_{j-1}, then partials of V[r].w,
//           r <= j, and of w.w (row j + 1)
//   mode 1: w -= sum_{r < nrows} c[r] V[r], then, where the segment needs a
//           second Gram-Schmidt pass, partials of V[r].w, r < nrows;
//           otherwise the partial of w.w in row 0
//   mode 2: where the second pass is needed, w -= sum_r c[r] V[r] and the
//           partial of w.w; otherwise the segment's first chunk forwards
//           c[0] (the norm from mode 1) and the others write 0
// The second pass follows the criterion of Daniel, Gragg, Kaufman and
// Stewart (Math. Comp. 30, 1976): with a = |w|^2 before the projection and
// p = sum_r c_r^2 the squared length it removed, the projection is
// repeated only when 2 p > a; every chunk of a segment evaluates it from
// the segment's mode-0 coefficients `cf` (a in entry nrows) with the same
// arithmetic, so a segment takes one decision.  Partials go to
// partial[r * nch + chunk], the layout k_sdot_final sums.
__device__ __forceinline__ bool s_second_pass(const double* cf, int nrows) {
    double p = 0.0;
    for (int r = 0; r < nrows; ++r) p += cf[r] * cf[r];
    return 2.0 * p > cf[nrows];
}

template <int MAXR, typename TV>
__global__ __launch_bounds__(256) void k_s_fused(double* __restrict__ w, const TV* __restrict__ V,
                                                 int64_t ldv, int mode, int nrows, int j,
                                                 const double* __restrict__ alpha,
                                                 const double* __restrict__ beta, int lds,
                                                 const double* __restrict__ c,
                                                 const double* __restrict__ cf,
                                                 const SegChunk* __restrict__ ch, int nch,
                                                 const int* __restrict__ seg_c0,
                                                 double* __restrict__ partial, const LState* st) {
    const SegChunk C = ch[blockIdx.x];
    if (st[C.seg].broken) return;
    __shared__ double sh[MAXR][4];
    const double* cs = mode == 0 ? nullptr : c + (int64_t)C.seg * lds;
    const double* cfs = mode == 0 ? nullptr : cf + (int64_t)C.seg * lds;
    const bool second = mode == 0 || s_second_pass(cfs, nrows);
    if (mode == 2 && !second) {
        if (threadIdx.x == 0) partial[blockIdx.x] = (int)blockIdx.x == seg_c0[C.seg] ? cs[0] : 0.0;
        return;
    }
    const int nr = mode == 0 ? j + 1 : nrows;                // rows in the update / dots
    const int nd = mode == 0 ? j + 2 : mode == 2 ? 1 : nr;   // partial rows written
    const bool norm_only = mode == 2 || !second;
    const double a = mode == 0 ? alpha[(int64_t)C.seg * lds + j] : 0.0;
    const double b = (mode == 0 && j > 0) ? beta[(int64_t)C.seg * lds + j - 1] : 0.0;
    double s[MAXR];
#pragma unroll
    for (int q = 0; q < MAXR; ++q) s[q] = 0.0;
    for (int64_t i = C.lo + threadIdx.x; i < C.hi; i += 256) {
        // every row's load is issued before any is converted (an FP32 row
        // converted inside its guarded load would wait for each load in
        // turn); the empty asm statements (no instruction) hold the values
        TV vt[MAXR];
#pragma unroll
        for (int r = 0; r < MAXR; ++r) vt[r] = r < nr ? V[(int64_t)r * ldv + i] : (TV)0;
        if constexpr (sizeof(TV) == 4) {
#pragma unroll
            for (int r = 0; r < MAXR; ++r) asm volatile("" : "+v"(vt[r]));
        }
        double v[MAXR];
#pragma unroll
        for (int r = 0; r < MAXR; ++r) v[r] = (double)vt[r];
        double wi = w[i];
        if (mode == 0) {
            double t = a * (double)V[(int64_t)j * ldv + i];
            if (j > 0) t += b * (double)V[(int64_t)(j - 1) * ldv + i];
            wi -= t;
        } else {
            double t = 0.0;
#pragma unroll
            for (int r = 0; r < MAXR; ++r)
                if (r < nr) t += cs[r] * v[r];
            wi -= t;
        }
        w[i] = wi;
        if (norm_only) {
            s[0] += wi * wi;
        } else {
#pragma unroll
            for (int r = 0; r < MAXR; ++r)
                if (r < nr) s[r] += v[r] * wi;
            if (mode == 0) {
#pragma unroll
                for (int r = 0; r < MAXR; ++r)
                    if (r == nr) s[r] += wi * wi;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < MAXR; ++q) {
        if (q < nd) {
            const double t = seg_wave_sum(s[q]);
            if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x >> 6] = t;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nd)
        partial[(int64_t)threadIdx.x * nch + blockIdx.x] =
            ((sh[threadIdx.x][0] + sh[threadIdx.x][1]) + sh[threadIdx.x][2]) + sh[threadIdx.x][3];
}

// lowest eigenpair of each segment's tridiagonal; one thread per segment
__global__ void k_s_tridiag(const double* alpha, const double* beta, int lds, double* sv,
                            LState* st, double* work, int nseg) {
    const int sidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (sidx >= nseg) return;
    const double* al = alpha + (int64_t)sidx * lds;
    const double* be = beta + (int64_t)sidx * lds;
    double* s = sv + (int64_t)sidx * lds;
    double* wk = work + (int64_t)sidx * 256;
    const int k = st[sidx].k;
    double lo = 0.0, hi = 0.0, tnorm = 0.0;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i < k - 1 ? fabs(be[i]) : 0.0);
        const double a = al[i] - r, b = al[i] + r;
        if (i == 0 || a < lo) lo = a;
        if (i == 0 || b > hi) hi = b;
        tnorm = fmax(tnorm, fabs(al[i]) + r);
    }
    const double tiny = 1e-300;
    for (int it = 0; it < 2000; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        int cnt = 0;
        double d = al[0] - mid;
        if (d == 0.0) d = -tiny;
        if (d < 0) ++cnt;
        for (int i = 1; i < k; ++i) {
            d = al[i] - mid - be[i - 1] * be[i - 1] / d;
            if (d == 0.0) d = -tiny;
            if (d < 0) ++cnt;
        }
        if (cnt >= 1) hi = mid; else lo = mid;
    }
    const double theta = 0.5 * (lo + hi);
    double* dl = wk;
    double* dd = wk + 64;
    double* du = wk + 128;
    double* du2 = wk + 192;
    int piv[64];
    for (int i = 0; i < k; ++i) s[i] = 1.0;
    const double eps = 2.3e-16 * (tnorm > 0 ? tnorm : 1.0);
    for (int iter = 0; iter < 3; ++iter) {
        for (int i = 0; i < k; ++i) {
            dd[i] = al[i] - theta;
            if (i < k - 1) { dl[i] = be[i]; du[i] = be[i]; }
            du2[i] = 0.0;
            piv[i] = i;
        }
        for (int i = 0; i < k - 1; ++i) {
            if (fabs(dd[i]) >= fabs(dl[i])) {
                if (dd[i] == 0.0) dd[i] = eps;
                const double f = dl[i] / dd[i];
                dl[i] = f;
                dd[i + 1] -= f * du[i];
            } else {
                const double f = dd[i] / dl[i];
                dd[i] = dl[i];
                dl[i] = f;
                const double tmp = du[i];
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
                const double tmp = s[i];
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
    st[sidx].theta = theta;
    st[sidx].resid = fabs(be[k - 1] * s[k - 1]);
}

// u = sum_{r < k_seg} s[seg][r] V[r]
template <typename TV>
__global__ void k_s_ritz(double* __restrict__ u, const TV* __restrict__ V, int64_t ldv,
                         const double* __restrict__ sv, int lds, const SegChunk* __restrict__ ch,
                         const LState* st) {
    const SegChunk C = ch[blockIdx.x];
    const int k = st[C.seg].k;
    const double* s = sv + (int64_t)C.seg * lds;
    for (int64_t i = C.lo + threadIdx.x; i < C.hi; i += 256) {
        double t = 0.0;
        for (int r = 0; r < k; ++r) t += s[r] * (double)V[(int64_t)r * ldv + i];
        u[i] = t;
    }
}

// largest |u| of each chunk and its first index
__global__ __launch_bounds__(256) void k_s_argmax(const double* __restrict__ u,
                                                  const SegChunk* __restrict__ ch, double* pv,
                                                  int64_t* pi) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    const SegChunk C = ch[blockIdx.x];
    double bv = -1.0;
    int64_t bi = -1;
    for (int64_t i = C.lo + threadIdx.x; i < C.hi; i += 256) {
        const double a = fabs(u[i]);
        if (a > bv) { bv = a; bi = i; }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double v2 = sv[threadIdx.x + o], v1 = sv[threadIdx.x];
            const int64_t i2 = si[threadIdx.x + o], i1 = si[threadIdx.x];
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

// fac[seg] = sign(u[argmax]) / nrm[seg]
__global__ void k_s_sign(const double* __restrict__ u, const double* pv, const int64_t* pi,
                         const int* seg_c0, const double* nrm, int ldn, double* fac, int nseg) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    double bv = -1.0;
    int64_t bi = -1;
    for (int c = seg_c0[s]; c < seg_c0[s + 1]; ++c)
        if (pv[c] > bv || (pv[c] == bv && pi[c] >= 0 && (bi < 0 || pi[c] < bi))) {
            bv = pv[c];
            bi = pi[c];
        }
    const double sg = (bi >= 0 && u[bi] < 0) ? -1.0 : 1.0;
    fac[s] = sg / nrm[(int64_t)s * ldn];
}

__global__ void k_s_scale(double* __restrict__ u, const double* __restrict__ fac,
                          const SegChunk* __restrict__ ch) {
    const SegChunk C = ch[blockIdx.x];
    const double f = fac[C.seg];
    for (int64_t i = C.lo + threadIdx.x; i < C.hi; i += 256) u[i] *= f;
}

// ---------------------------------------------------------------------
template <typename TV>
void seg_dots(const TV* V, int64_t ldv, int nrows, const double* w, const SegChunk* ch, int nch,
              const int* seg_c0, int nseg, double* partial, double* out, int ldo, int mode,
              const LState* st, int skip, hipStream_t s) {
    hipLaunchKernelGGL(k_sdot_partial<TV>, dim3(nch), dim3(256), 0, s, V, ldv, nrows, w, ch, nch,
                       partial, st, skip);
    hipLaunchKernelGGL(k_sdot_final, dim3(nseg * nrows), dim3(256), 0, s, partial, nch, seg_c0,
                       nrows, out, ldo, mode, st, skip);
}
template <typename TV>
bool seg_fused(int mode, double* w, const TV* V, int64_t ldv, int nrows, int j, const double* al,
               const double* be, int lds, const double* c, const double* cf, const SegChunk* ch, int nch,
               const int* seg_c0, int nseg, double* partial, double* out, int ldo, const LState* st,
               hipStream_t s) {
    const int nr = mode == 0 ? j + 1 : nrows;
    if (nr + 1 > 32) return false;   // mode 0 also needs the row of w.w
    if (nr + 1 <= 16)
        hipLaunchKernelGGL((k_s_fused<16, TV>), dim3(nch), dim3(256), 0, s, w, V, ldv, mode, nrows, j, al, be, lds, c,
                           cf, ch, nch, seg_c0, partial, st);
    else
        hipLaunchKernelGGL((k_s_fused<32, TV>), dim3(nch), dim3(256), 0, s, w, V, ldv, mode, nrows, j, al, be, lds, c,
                           cf, ch, nch, seg_c0, partial, st);
    const int nd = mode == 0 ? j + 2 : mode == 2 ? 1 : nr;
    hipLaunchKernelGGL(k_sdot_final, dim3(nseg * nd), dim3(256), 0, s, partial, nch, seg_c0, nd, out, ldo, 0,
                       st, 1);
    return true;
}
void seg_init(LState* st, int nseg, int m, const double* nrm, int ldn, hipStream_t s) {
    hipLaunchKernelGGL(k_s_init, dim3((nseg + 63) / 64), dim3(64), 0, s, st, nseg, m, nrm, ldn);
}
template <typename TV>
void seg_start(TV* dst, const double* src, const double* nrm, int ldn, const SegChunk* ch, int nch,
               hipStream_t s) {
    hipLaunchKernelGGL(k_s_start<TV>, dim3(nch), dim3(256), 0, s, dst, src, nrm, ldn, ch);
}
void seg_three_term(double* w, const double* V, int64_t ldv, int j, const double* al,
                    const double* be, int lds, const SegChunk* ch, int nch, const LState* st,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_s_three_term, dim3(nch), dim3(256), 0, s, w, V, ldv, j, al, be, lds, ch, st);
}
void seg_subtract(double* w, const double* V, int64_t ldv, int nrows, const double* coef, int lds,
                  const SegChunk* ch, int nch, const LState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_s_subtract, dim3(nch), dim3(256), 0, s, w, V, ldv, nrows, coef, lds, ch, st);
}
void seg_beta(const double* ww, int ldw, double* al, double* be, int lds, int j, LState* st,
              int nseg, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_s_beta, dim3((nseg + 63) / 64), dim3(64), 0, s, ww, ldw, al, be, lds, j, st,
                       nseg, tol);
}
template <typename TV>
void seg_next(TV* V, int64_t ldv, int j, const double* w, const double* be, int lds, const SegChunk* ch,
              int nch, const LState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_s_next<TV>, dim3(nch), dim3(256), 0, s, V, ldv, j, w, be, lds, ch, st);
}
void seg_tridiag(const double* al, const double* be, int lds, double* sv, LState* st, double* work,
                 int nseg, hipStream_t s) {
    hipLaunchKernelGGL(k_s_tridiag, dim3((nseg + 63) / 64), dim3(64), 0, s, al, be, lds, sv, st, work,
                       nseg);
}
template <typename TV>
void seg_ritz(double* u, const TV* V, int64_t ldv, const double* sv, int lds, const SegChunk* ch, int nch,
              const LState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_s_ritz<TV>, dim3(nch), dim3(256), 0, s, u, V, ldv, sv, lds, ch, st);
}
void seg_normalise_sign(double* u, const SegChunk* ch, int nch, const int* seg_c0, int nseg,
                        const double* nrm, int ldn, double* pv, int64_t* pi, double* fac,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_s_argmax, dim3(nch), dim3(256), 0, s, u, ch, pv, pi);
    hipLaunchKernelGGL(k_s_sign, dim3((nseg + 63) / 64), dim3(64), 0, s, u, pv, pi, seg_c0, nrm, ldn,
                       fac, nseg);
    hipLaunchKernelGGL(k_s_scale, dim3(nch), dim3(256), 0, s, u, fac, ch);
}

#define QED_SEG_TV(TV)                                                                                          \
    template void seg_dots<TV>(const TV*, int64_t, int, const double*, const SegChunk*, int, const int*, int,     \
                               double*, double*, int, int, const LState*, int, hipStream_t);                      \
    template bool seg_fused<TV>(int, double*, const TV*, int64_t, int, int, const double*, const double*, int,    \
                                const double*, const double*, const SegChunk*, int, const int*, int, double*,     \
                                double*, int, const LState*, hipStream_t);                                        \
    template void seg_start<TV>(TV*, const double*, const double*, int, const SegChunk*, int, hipStream_t);      \
    template void seg_next<TV>(TV*, int64_t, int, const double*, const double*, int, const SegChunk*, int,        \
                               const LState*, hipStream_t);                                                       \
    template void seg_ritz<TV>(double*, const TV*, int64_t, const double*, int, const SegChunk*, int,             \
                               const LState*, hipStream_t);
QED_SEG_TV(double)
QED_SEG_TV(float)
#undef QED_SEG_TV

}  // namespace qed
