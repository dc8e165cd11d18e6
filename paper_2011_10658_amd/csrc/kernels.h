// Device data structures shared by the host planner and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qed {

// Pointer into one of the buffers bound at launch time: tag 0 = absolute
// address `abs`; tag t > 0 = bases[t] + off elements of the compute type.
enum { TAG_ABS = 0, TAG_WS = 1, TAG_X = 2, TAG_Y = 3, NTAGS = 4 };

struct GRef {
    const void* abs;
    int64_t off;
    int tag;
    int pad;
};

struct Bases {
    void* b[NTAGS];
};

// One (batch-reduce) product alpha * sum_{r < nred} op(A_r) op(B_r),
// op(A) M x K, op(B) K x N.  tA = 1: op(A)[m][k] = A[k * lda + m];
// tB = 1: op(B)[k][n] = B[n * ldb + k].  ident = 1: A is the identity and
// op(B) (M x N, tB = 0) is added.  bsA/bsB: strides between batch items.
// nsb > 0 splits the column index of op(B) (tB = 0 only): column n lives
// at (n / nsb) * nob + (n % nsb) instead of n (a batch of matrices side by
// side read as one wide matrix).
struct GProd {
    GRef A, B;
    int64_t rsA, rsB, bsA, bsB, nob;
    double alpha;
    int K, lda, ldb, tA, tB, nred, ident, nsb;
};

// Output C (M x N, row-major, ldc) of `batch` items (stride bsC), the sum
// of products [p0, p1); acc = 1 adds into C, 0 overwrites.
// nsc > 0 splits the output column index the same way (stride noc).
struct GJob {
    GRef C;
    int64_t bsC, noc;
    int M, N, ldc, batch, p0, p1, acc, nsc;
};

// Fused H_eff stages (terms with a factor on the bond leg).  The output
// block Y is read as rows m < M (stride ldy) of G groups (stride goy) of np
// contiguous entries.  A product is  W = alpha F X  on the row leg (F:
// M x K row-major with leading dimension lda, or the identity), with X
// element (k, g, c) at k * ldx + g * gox + c (c < np_in), followed by
// Y(m, g, :) += W(m, g, :) C^T with C the np x np_in bond block (row-major,
// leading dimension np_in), or by Y += W when the product has no bond
// factor (then np_in = np).
struct FProd {
    GRef F, X, Cb;
    int64_t ldx, gox;
    double alpha;
    int K, lda, np_in, identF, hasC, pad;
};

// One output block of a fused stage: the sum of products [p0, p1), added
// to Y (acc = 1) or written over it.  A workgroup tile covers 64 rows and
// ng consecutive groups; in the tile every group takes np rounded up to a
// multiple of 16 columns, so that a bond-factor product is a whole number
// of MFMA column blocks per group.
struct FJob {
    GRef Y;
    int64_t ldy, goy;
    int M, G, np, ng, p0, p1, acc, pad;
};

// One array of a batched FP64 -> FP32 conversion.
struct ConvSeg {
    const double* src;
    void* dst;
    int64_t n;
};

// Work item of one workgroup: tile (tm, tn) of batch item b of job j.
struct GTile {
    int job, b, tm, tn;   // job < 0: an empty slot (the workgroup returns)
};

// One segment of the adjoint's gradient post-processing: dst[i] =
// scale * src[i] for i < n (scaling pass, dst may be null), and, in the
// dot pass, out[dot] = sum_i src[i] * a[i] (dot < 0: none).
struct AdjSeg {
    const double* src;
    double* dst;
    const double* a;
    int64_t n;
    double scale;
    int dot;
    int pad;
};

// One matrix of the one-sided Jacobi SVD: X (n x m, column-major, ld n) is
// overwritten by W = X V with mutually orthogonal columns, V (m x m,
// column-major) receives the rotations, sigma[j] = |W[:, j]|.
struct SvdMat {
    double* x;
    double* v;
    double* sigma;
    int n, m;
};

// Rows of a fused-stage tile, and its widest W (dense groups) and Y
// (16-padded groups) column spans per operand type.
constexpr int FUSED_TM = 64;
constexpr int FUSED_COLS_F32 = 128;
constexpr int FUSED_COLS_F64 = 64;

// Workgroup tile shapes of the block GEMM (rows x cols of the output).
enum {
    GEMM_SHAPE_SQUARE = 0,   //  64 x  64
    GEMM_SHAPE_TALL = 1,     // 128 x  32
    GEMM_SHAPE_WIDE = 2,     //  32 x 128
    GEMM_NSHAPES = 3
};
inline int gemm_tm(int s) {
    const int t[GEMM_NSHAPES] = {64, 128, 32};
    return t[s];
}
inline int gemm_tn(int s) {
    const int t[GEMM_NSHAPES] = {64, 32, 128};
    return t[s];
}
constexpr int GEMM_THREADS = 256;

// Operand pipelines of the block GEMM: register-staged double buffer
// (loop), one chunk per product across the products of a job (flat), and
// the LDS ring filled by buffer-to-LDS loads (dma: FP32 and FP64, tA = tB =
// 0, SQUARE and WIDE tiles, operands under 2^31 bytes).
// skinny: the whole stage is A B^T products with K, N <= 64 into contiguous
// outputs (one workgroup per row strip and the full output width).
enum { GEMM_PIPE_LOOP = 0, GEMM_PIPE_FLAT = 1, GEMM_PIPE_DMA = 2, GEMM_PIPE_SKINNY = 3, GEMM_NPIPES = 4 };
constexpr int SK_KMAX = 64;
constexpr int SK_NMAX = 64;

// Per-block description for packing a node tensor into the column-major
// matrices of its sectors along one leg (QR), and back.
struct PackBlk {
    int64_t off;       // block offset in the tensor
    int64_t mat;       // offset of the sector matrix in the packed buffer
    int n[3];          // block extents (l, r, p)
    int leg;           // leg whose index becomes the column
    int rows;          // rows of the sector matrix (its leading dimension)
    int row0;          // first row of this block inside the sector matrix
};

// One matrix for the QR kernel: column-major rows x cols with leading
// dimension ld at `mat` (in the packed buffer and, for the scratch copy of
// Q, in the scratch buffer); R(r, c) is written at rout + r*rrs + c*rcs.
// Output elements per workgroup of an identity-only (summation) stage.
constexpr int SUM_TILE = 1024;

// Sizes one QR workgroup handles (the panel and the T factors live in LDS).
constexpr int QR_ROWS = 2048;
constexpr int QR_COLS = 256;
// LDS-resident QR (k_qr_lds): matrices of at most QRL_MAXC columns, QR_ROWS
// rows and (rows + 1) x cols <= QRL_CAP
constexpr int QRL_MAXC = 96;
constexpr int QRL_CAP = 19456;
inline bool qr_lds_fits(int64_t rows, int cols) {
    return cols <= QRL_MAXC && rows <= QR_ROWS && (rows + 1) * cols <= QRL_CAP;
}
// LDS that k_qr_lds needs for one rows x cols matrix (a launch takes the
// largest over its matrices; at most 160 KiB whenever qr_lds_fits)
inline size_t qr_lds_bytes(int64_t rows, int cols) {
    return (size_t)(((rows | 1) * cols) + 3 * cols + 4 + 512) * sizeof(double);
}

struct QRMat {
    double* a;          // the matrix (column-major, leading dimension ld); Q on exit
    double* q;          // scratch with the same layout
    double* r;          // R written at r[i * rrs + j * rcs]
    int64_t ld;
    int64_t rrs, rcs;
    int rows, cols;
};

// One sector of a CholeskyQR pass: G (n x n, row-major) = A^T A of the
// sector matrix; the kernel factors G + shift trace(G) I = R^T R (R upper,
// positive diagonal), writes R^-1 (row-major n x n) to rinv and, when
// rprev is set, the product R rprev (row-major n x n) to rout at
// rout[i * rrs + j * rcs]; otherwise R itself.  status = 1 when a pivot
// fell below 1e-12 of the largest diagonal entry (not positive definite to
// working precision), else 0.
struct CholMat {
    const double* g;
    double* rinv;
    const double* rprev;
    double* rout;
    int* status;
    int64_t rrs, rcs;
    double shift;
    int n;
    int pad;
};
constexpr int CHOL_MAX_COLS = 96;

// A chunk of a segmented vector (never straddles a segment boundary).
struct SegChunk {
    int seg;
    int pad;
    int64_t lo, hi;
};

// Lanczos state living on the device.
struct LState {
    int k;             // number of valid steps (== m unless broken down)
    int broken;
    double theta, resid, norm;
};

}  // namespace qed
