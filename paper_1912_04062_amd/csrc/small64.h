// Dense 64 x 64 building blocks for kernels of one 256-thread workgroup
// (Cholesky QR of panels, Cholesky-QR of eigenvector blocks).  Matrices live
// in LDS (row r at r * 65); thread (tx, ty) = (tid % 64, tid / 64) owns row
// tx, columns ty + 4q (q = 0..15) and is the only writer of those elements
// (owner computes: no branches around the LDS accesses, no write races).
#pragma once
#include "common.h"

namespace {

// X = R^{-1} for R upper triangular (B x B), rows of X from the bottom:
// X[i][c] = (delta_ic - sum_{i < u <= c} R[i][u] X[u][c]) / R[i][i].  X
// starts at zero and row i is written at step i, so at that step X[u][c] is
// zero for u <= i and for u > c: the sum runs over all u with no masks.
// The strict lower triangle of R is read (multiplied by zeros): it must hold
// finite values.
__device__ __forceinline__ void tri_inv_upper(const double *R, double *X, int B, double (*part)[64], double *rinv)
{
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    if (tid < 64) rinv[tid] = (tid < B) ? 1.0 / R[tid * 65 + tid] : 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) X[tx * 65 + ty + 4 * q] = 0.0;
    __syncthreads();
    for (int i = B - 1; i >= 0; --i) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int q = 0; q < 16; q += 2) {
            const int u = ty + 4 * q;
            s0 = fma(R[i * 65 + u], X[u * 65 + tx], s0);
            s1 = fma(R[i * 65 + u + 4], X[(u + 4) * 65 + tx], s1);
        }
        part[ty][tx] = s0 + s1;
        __syncthreads();
        if (ty == 0 && tx < B && i <= tx)
            X[i * 65 + tx] = (((i == tx) ? 1.0 : 0.0) - (part[0][tx] + part[1][tx] + part[2][tx] + part[3][tx])) * rinv[i];
        __syncthreads();
    }
}

// Cholesky M = R^T R of the symmetric positive B x B matrix M in place (64
// steps, right-looking, both triangles updated): step j scales row j by
// 1/r_jj and subtracts R[j][r] R[j][c] from every element (r, c) with r > j.
// R ends in the upper triangle, the strict lower triangle tends to zero
// (finite).  Returns false when a pivot leaves (lo, hi); with clamp a pivot
// <= 0 is replaced by 1e-300 and the factorization never fails.  Rows and
// columns B..63 must be zero.
__device__ __forceinline__ bool cholesky64(double *M, int B, bool clamp, double lo, double hi, int *bad)
{
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    for (int j = 0; j < B; ++j) {
        const double d = M[j * 65 + j];
        if (!clamp && !(d > lo && d < hi)) {   // uniform: every thread reads the same d
            if (tid == 0) *bad = 1;
            return false;
        }
        const double ip = 1.0 / sqrt((clamp && !(d > 0.0)) ? 1e-300 : d);
        const double lr = (tx > j) ? M[j * 65 + tx] * ip : 0.0;   // R[j][tx] for rows below j
        const double a = (tx == j) ? ip : 1.0;                      // row j: scaled by 1/r_jj
        double rc[16], old[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            rc[q] = M[j * 65 + ty + 4 * q];
            old[q] = M[tx * 65 + ty + 4 * q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) M[tx * 65 + ty + 4 * q] = fma(-lr, rc[q] * ip, old[q] * a);
        __syncthreads();
    }
    return true;
}

// LU factorization M - S = L U without pivoting, S = diag(s_i) with
// s_i = -sign of the pivot met at step i (so |u_ii| >= 1); s_i goes to
// sgn[i].  L (unit lower) ends below the diagonal, U on and above it.  Rows
// and columns B..63 must be zero.
__device__ __forceinline__ void lu_signed64(double *M, int B, double *sgn)
{
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    for (int j = 0; j < B; ++j) {
        const double d = M[j * 65 + j];
        const double si = (d >= 0.0) ? -1.0 : 1.0, piv = d - si, ip = 1.0 / piv;
        // rows below j: multiplier l = M[r][j] / u_jj; column j receives l
        // itself (old - l (u_jj - 1) = l), columns right of j the update, the
        // columns left of j (earlier multipliers) nothing
        const double lr = (tx > j) ? M[tx * 65 + j] * ip : 0.0;
        double rc[16], old[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = ty + 4 * q;
            const double u = M[j * 65 + c];
            rc[q] = (c > j) ? u : ((c == j) ? piv - 1.0 : 0.0);
            old[q] = M[tx * 65 + c];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) M[tx * 65 + ty + 4 * q] = fma(-lr, rc[q], old[q]);
        if (tid == 0) sgn[j] = si;
        __syncthreads();
    }
    // row j was left at the pivot d = u_jj + s_j
    for (int q = 0; q < 16; ++q) {
        const int c = ty + 4 * q;
        if (c == tx && c < B) M[c * 65 + c] -= sgn[c];
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
