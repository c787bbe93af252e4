// Dense 64 x 64 building blocks for kernels of one 256-thread workgroup
// (Cholesky QR of panels, Householder reconstruction, Cholesky-QR of
// eigenvector blocks, the Bethe-Salpeter Cholesky).  Matrices live in LDS
// (row r at r * 65) between the building blocks.
#pragma once
#include "common.h"

namespace {

// The eliminations below keep the matrix in registers: thread t owns the
// 4 x 4 block of rows 4 (t % 16) + i and columns 4 (t / 16) + k (i, k = 0..3).
// Step j needs the pivot row (and, without symmetry, the pivot column) of the
// working matrix; their owners publish them in a small LDS buffer at the end
// of the previous step, so each step costs one workgroup barrier and a few
// LDS accesses per thread.  The buffer sets rotate, so a set is rewritten only
// after every thread has passed the barrier that follows its last reader.
// The per-step update of an element is a single FMA: the masks sit on the
// per-row and per-column factors (zero outside the trailing part), and the
// divisions by the pivots are applied to whole rows or columns at the end.

// Four consecutive doubles from LDS (16-byte aligned), loaded
// unconditionally: the masks are applied to the values afterwards, so no
// load sits behind a branch with a wait of its own.
typedef double small64_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void lds4(const double *p, double v[4])
{
    const small64_d2 a = *(const small64_d2 *)p, b = *(const small64_d2 *)(p + 2);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
}

// Cholesky G = R^T R of the symmetric positive B x B matrix in M (row r at
// r * 65; rows and columns B..63 zero) together with R^{-1}: forward
// elimination of [G | I], whose step j subtracts (g_jr / g_jj) times row j
// from every row r > j, ends at D [R | R^{-T}] with D = diag(r_jj), and rows
// are divided by r_jj = sqrt of the pivot at the end.  Only the upper triangle
// of the working matrix is read, so the factor does not depend on the
// rounding of G's lower triangle.  Returns false (every thread, at the same
// step) when a pivot leaves (lo, hi); with clamp a pivot <= 0 is replaced by
// 1e-300 and the factorization never fails.  On success M holds R (zeros
// below the diagonal) and X holds R^{-1} (zeros below the diagonal).  The
// caller synchronizes after writing M; buf holds 320 doubles, 16-byte
// aligned.  The steps run
// in groups of four, so the row of a thread's block that step j touches
// (j % 4) is known at compile time.
__device__ __forceinline__ bool chol_inv64(double *M, double *X, int B, bool clamp, double lo, double hi,
                                           double *buf)
{
    const int r0 = 4 * (threadIdx.x & 15), c0 = 4 * (threadIdx.x >> 4);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double *dpiv = buf + 256;   // the pivots, for the row scaling at the end
    double e[4][4], y[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            e[i][k] = M[(r0 + i) * 65 + c0 + k];
            y[i][k] = (r0 + i == c0 + k) ? 1.0 : 0.0;
        }
    }
    if (r0 == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            buf[c0 + k] = e[0][k];
            buf[64 + c0 + k] = y[0][k];
        }
    }
    for (int jb = 0; jb < B; jb += 4) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int j = jb + jj;
            if (j < B) {   // uniform
                __syncthreads();
                const double *rb = buf + (jj & 1) * 128;
                const double d = rb[j];
                if (!clamp && !(d > lo && d < hi)) return false;   // uniform: every thread reads the same d
                const double dd = (clamp && !(d > 0.0)) ? 1e-300 : d;
                const double ip2 = recip(dd);   // the next pivot waits for this, not for a square root
                if (threadIdx.x == 0) dpiv[j] = dd;
                double lr[4], uc[4], yc[4];
                lds4(rb + r0, lr);
                lds4(rb + c0, uc);
                lds4(rb + 64 + c0, yc);
#pragma unroll
                for (int i = 0; i < 4; ++i) lr[i] = (r0 + i > j) ? lr[i] : 0.0;   // g_jr, r > j
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    uc[k] = (c0 + k > j) ? uc[k] * ip2 : 0.0;
                    yc[k] *= ip2;
                }
                // the wavefront's columns are 16 wv .. 16 wv + 15: G's trailing
                // columns are those > j, the nonzero columns of row j of R^{-T}
                // those <= j
                if (16 * wv + 15 > j) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int k = 0; k < 4; ++k) e[i][k] = fma(-lr[i], uc[k], e[i][k]);
                }
                if (16 * wv <= j) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int k = 0; k < 4; ++k) y[i][k] = fma(-lr[i], yc[k], y[i][k]);
                }
                // row j + 1 for the next step: row (jj + 1) % 4 of the block
                // of rows 4 ((j + 1) / 4)
                const int jn = j + 1, in = (jj + 1) & 3;
                if (jn < B && (jn & ~3) == r0) {
                    double *nb = buf + ((jj + 1) & 1) * 128;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        nb[c0 + k] = e[in][k];
                        nb[64 + c0 + k] = y[in][k];
                    }
                }
            }
        }
    }
    __syncthreads();
    double ir[4];   // 1 / r_jj of the thread's rows
#pragma unroll
    for (int i = 0; i < 4; ++i) ir[i] = (r0 + i < B) ? 1.0 / sqrt(dpiv[r0 + i]) : 1.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = r0 + i, c = c0 + k;
            M[r * 65 + c] = (r <= c) ? e[i][k] * ir[i] : 0.0;
            X[c * 65 + r] = (c <= r) ? y[i][k] * ir[i] : 0.0;   // R^{-1} = (R^{-T})^T
        }
    __syncthreads();
    return true;
}

// LU factorization M - S = L U without pivoting, S = diag(s_i) with
// s_i = -sign of the pivot met at step i (so |u_ii| >= 1), together with
// L^{-1} and U^{-1}, in one pass of B steps.  L^{-1}: forward elimination of
// [M - S | I] ends at [U | L^{-1}].  The working matrix keeps the eliminated
// column j unscaled (L's column is it divided by u_jj, at the end) and the
// diagonal at the pivot u_jj + s_j.  U^{-1} by columns: column c is
// (e_c - X[:, :c] U[:c, c]) / u_cc, its sum accumulated one row of U at a time;
// the contribution of column j - 1 is added at step j, when its owners have
// published it.  On return M holds L (strictly below the diagonal) and U (on
// and above it), Xu = U^{-1} and Yl = L^{-1} (zeros outside their triangles),
// sgn[i] = s_i.  Rows and columns B..63 of M must be zero.  The caller
// synchronizes after writing M; buf holds 1024 doubles, 16-byte aligned (four sets of the
// pivot row of [M | I], the pivot column and the last column of U^{-1}; set
// j % 4 is read at step j and written at step j - 1).  Steps run in groups
// of four as in chol_inv64.
__device__ __forceinline__ void lu_signed_inv64(double *M, double *Xu, double *Yl, int B, double *sgn, double *buf)
{
    const int r0 = 4 * (threadIdx.x & 15), c0 = 4 * (threadIdx.x >> 4);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double e[4][4], y[4][4], x[4][4], ic[4];   // ic: 1 / u_jj of the thread's columns
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        ic[i] = 1.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            e[i][k] = M[(r0 + i) * 65 + c0 + k];
            y[i][k] = (r0 + i == c0 + k) ? 1.0 : 0.0;
            x[i][k] = 0.0;
        }
    }
    // set layout: [0, 64) pivot row, [64, 128) its row of L^{-1}, [128, 192)
    // pivot column, [192, 256) the previous column of U^{-1}
    if (r0 == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            buf[c0 + k] = e[0][k];
            buf[64 + c0 + k] = y[0][k];
        }
    }
    if (c0 == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) buf[128 + r0 + i] = e[i][0];
    }
    for (int jb = 0; jb < B; jb += 4) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int j = jb + jj;
            if (j < B) {   // uniform
                __syncthreads();
                const double *cur = buf + jj * 256, *prv = buf + ((jj + 3) & 3) * 256;
                const double d = cur[j];
                const double s = (d >= 0.0) ? -1.0 : 1.0, piv = d - s, ip = recip(piv);   // |piv| >= 1
                if (threadIdx.x == 0) sgn[j] = s;
                double lr[4], ur[4], yr[4], xr[4], up[4];
                lds4(cur + 128 + r0, lr);
                lds4(cur + 192 + r0, xr);
                lds4(cur + c0, ur);
                lds4(cur + 64 + c0, yr);
                lds4(prv + c0, up);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    lr[i] = (r0 + i > j) ? lr[i] * ip : 0.0;   // L[r][j], r > j
                    xr[i] = (j > 0) ? xr[i] : 0.0;             // column j - 1 of U^{-1}
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    ur[k] = (c0 + k > j) ? ur[k] : 0.0;
                    up[k] = (j > 0 && c0 + k >= j) ? up[k] : 0.0;  // U[j-1][c], c > j - 1
                }
                // the wavefront's columns are 16 wv .. 16 wv + 15: the trailing
                // columns are those > j, the nonzero columns of row j of L^{-1}
                // those <= j, the open columns of U^{-1} those >= j
                if (16 * wv + 15 > j) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int k = 0; k < 4; ++k) e[i][k] = fma(-lr[i], ur[k], e[i][k]);
                }
                if (16 * wv <= j) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int k = 0; k < 4; ++k) y[i][k] = fma(-lr[i], yr[k], y[i][k]);
                }
                if (16 * wv + 15 >= j) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int k = 0; k < 4; ++k) x[i][k] = fma(xr[i], up[k], x[i][k]);
                }
                if (jb == c0) {   // column j of U^{-1}, and 1 / u_jj
                    ic[jj] = ip;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = r0 + i;
                        x[i][jj] = (r <= j) ? (((r == j) ? 1.0 : 0.0) - x[i][jj]) * ip : 0.0;
                    }
                }
                double *nb = buf + ((jj + 1) & 3) * 256;
                const int jn = j + 1, in = (jj + 1) & 3;
                if (jn < B && (jn & ~3) == r0) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        nb[c0 + k] = e[in][k];
                        nb[64 + c0 + k] = y[in][k];
                    }
                }
                if (jn < B && (jn & ~3) == c0) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) nb[128 + r0 + i] = e[i][in];
                }
                if (jb == c0) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) nb[192 + r0 + i] = x[i][jj];
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = r0 + i, c = c0 + k;
            const double sr = (r < B) ? sgn[r] : 0.0;
            M[r * 65 + c] = (r > c) ? e[i][k] * ic[k] : ((r == c) ? e[i][k] - sr : e[i][k]);
            Xu[r * 65 + c] = (r <= c) ? x[i][k] : 0.0;
            Yl[r * 65 + c] = (r >= c) ? y[i][k] : 0.0;
        }
    __syncthreads();
}

// C = op(A) B for 64 x 64 matrices in LDS (row r at r * 65) on the FP64
// MFMA: wavefront w computes the 32 x 32 quadrant (w / 2, w % 2); op(A) = A,
// or A^T with TA.  C must not overlap A or B; the caller synchronizes before
// (operands written) and after (C read by other wavefronts).
template <bool TA>
__device__ __forceinline__ void mm64(const double *A, const double *B, double *C)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm0 = (w >> 1) * 32, wn0 = (w & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    d4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k4 = 0; k4 < 64; k4 += 4) {
        const int k = k4 + lk;
        double a[2], bb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row = wm0 + 16 * i + lr;
            a[i] = TA ? A[k * 65 + row] : A[row * 65 + k];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) bb[j] = B[k * 65 + wn0 + 16 * j + lr];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma_16x16x4(a[i], bb[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                C[(wm0 + 16 * i + mfma_row<double>(lane, r)) * 65 + wn0 + 16 * j + lr] = acc[i][j][r];
}

}  // namespace
