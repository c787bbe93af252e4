// Dense 64 x 64 building blocks for kernels of one 256-thread workgroup
// (Cholesky QR of panels, Cholesky-QR of eigenvector blocks).  Matrices live
// in LDS (row r at r * 65); thread (tx, ty) = (tid % 64, tid / 64) owns row
// tx, columns ty + 4q (q = 0..15) and is the only writer of those elements
// (owner computes: no branches around the LDS accesses, no write races).
#pragma once
#include "common.h"

namespace {

// X = R^{-1} for R upper triangular (B x B), rows of X from the bottom:
// X[i][c] = (delta_ic - sum_{i < u <= c} R[i][u] X[u][c]) / R[i][i].
__device__ __forceinline__ void tri_inv_upper(const double *R, double *X, int B, double (*part)[64], double *rinv)
{
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    if (tid < 64) rinv[tid] = (tid < B) ? 1.0 / R[tid * 65 + tid] : 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) X[tx * 65 + ty + 4 * q] = 0.0;
    __syncthreads();
    for (int i = B - 1; i >= 0; --i) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int u = ty + 4 * q;
            const double a = R[i * 65 + u], x = X[u * 65 + tx];
            s += (u > i && u <= tx && u < B) ? a * x : 0.0;
        }
        part[ty][tx] = s;
        __syncthreads();
        if (ty == 0 && tx < B && i <= tx)
            X[i * 65 + tx] = (((i == tx) ? 1.0 : 0.0) - (part[0][tx] + part[1][tx] + part[2][tx] + part[3][tx])) * rinv[i];
        __syncthreads();
    }
}

// Right-looking elimination of the B x B matrix M in place (64 steps).
// Cholesky (chol = true): M = R^T R, R upper in the upper triangle; returns
// false when a pivot leaves (lo, hi), or, with clamp, replaces a pivot
// <= 0 by 1e-300 and never fails.  LU (chol = false): M - S = L U with
// s_i = -sign(pivot) chosen at step i (sgn[i]); L unit lower below the
// diagonal, U on and above it (|u_ii| >= 1, no pivoting).
__device__ __forceinline__ bool eliminate(double *M, int B, bool chol, bool clamp, double lo, double hi, double *sgn,
                                          int *bad)
{
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    for (int j = 0; j < B; ++j) {
        const double d = M[j * 65 + j];
        double piv, si = 0.0;
        if (chol) {
            if (!clamp && !(d > lo && d < hi)) {   // uniform: every thread reads the same d
                if (tid == 0) *bad = 1;
                return false;
            }
            piv = sqrt((clamp && !(d > 0.0)) ? 1e-300 : d);
        } else {
            si = (d >= 0.0) ? -1.0 : 1.0;
            piv = d - si;
        }
        const double ip = 1.0 / piv;
        // Cholesky: row j of R is M[j][c] / r_jj and row r is updated with
        // R[j][r] R[j][c]; LU: multipliers l_r = M[r][j] / u_jj, row j of U
        // unchanged
        const double lr = (chol ? M[j * 65 + tx] : M[tx * 65 + j]) * ip;
        double rc[16], old[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = ty + 4 * q;
            rc[q] = M[j * 65 + c] * (chol ? ip : 1.0);
            old[q] = M[tx * 65 + c];
        }
        __syncthreads();
        const bool live = tx < B;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = ty + 4 * q;
            double v = old[q];
            if (chol) {
                if (tx == j) v = (c == j) ? piv : ((c > j) ? rc[q] : v);
                else if (tx > j && c >= tx && c < B) v = old[q] - lr * rc[q];
            } else {
                if (tx == j && c == j) v = piv;
                else if (tx > j && c == j) v = lr;
                else if (tx > j && c > j && c < B) v = old[q] - lr * rc[q];
            }
            M[tx * 65 + c] = live ? v : old[q];
        }
        if (!chol && tid == 0) sgn[j] = si;
        __syncthreads();
    }
    return true;
}

}  // namespace
