// One-stage skew tridiagonalization (Section 2.3.1: the ELPA1 route, the one
// the paper's GPU variant offloads), blocked by panels of b columns with the
// trailing update deferred to one skew rank-2b update per panel.
//
// Column c of panel p (columns c0 .. c0 + b - 1), r = c + 1, m = n - r:
//   k_os_col     the current column a = A(r:, c) + V W(c, :)^T - W V(c, :)^T
//                (the panel's deferred update restricted to it; k_os_w of the
//                previous column has left all of it but the previous
//                reflector's term in column jj of V), its Householder
//                reflector (v, tau, beta; alpha_c = -beta) and v into column
//                jj of the panel's V;
//   k_os_symv    y = A_stored(r:, r:) v over tiles of the stored lower
//                triangle: A_ij = L_ij (i > j), A_ji = -L_ij, so a tile adds
//                L v_J to y_I and -L^T v_I to y_J (two partial vectors per
//                tile); the diagonal tiles also form partial dot products
//                V(:, k)^T v and W(:, k)^T v for the earlier columns k;
//   k_os_dots    those dot products summed (one workgroup, fixed order) and
//                the compact-WY column T(:jj, jj) = -tau T V^T v, T(jj, jj) = tau;
//   k_os_w       w = tau (y + V (W^T v) - W (V^T v)) into column jj of W:
//                A + v w^T - w v^T is the two-sided update H A H of the skew
//                matrix (v^T A v = 0); with the same loads of V and W it forms
//                the next column's deferred update except the term of w(r),
//                which only its first workgroup knows.
// After the panel, the stored trailing matrix gets A += V W^T - W V^T (the
// lower tiles of the stage-1 SYR2K kernel).  V (unit lower trapezoidal, rows
// c0 + 1 .. n - 1) and T are kept per panel for the back-transformation.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int OT = 64;        // SYMV tile

// one workgroup of 1024 threads
constexpr int CT = 1024;
__global__ __launch_bounds__(CT) void k_os_col(const double *__restrict__ A, int lda, int n, int c0, int jj,
                                               double *__restrict__ V, double *__restrict__ W, int ldv,
                                               double *__restrict__ tau, double *__restrict__ alpha)
{
    __shared__ double red[CT / 64];
    __shared__ double bsc[2];
    const int c = c0 + jj, r = c + 1, m = n - r;
    const int off = r - (c0 + 1);            // row r in the panel arrays (rows c0+1 ..)
    const int tid = threadIdx.x;
    double *col = V + (size_t)jj * ldv + off;
    // jj > 0: column jj of V holds A(r:, c) plus the deferred terms of the
    // reflectors k < jj - 1 (and -W(:, jj-1) V(c, jj-1), V(c, jj-1) = 1); the
    // term V(:, jj-1) W(c, jj-1) is added here
    const double wc = jj > 0 ? W[(size_t)(jj - 1) * ldv + off - 1] : 0.0;
    const double *vp = V + (size_t)(jj - 1) * ldv + off;
    double sq = 0.0;
    for (int i = tid; i < m; i += CT) {
        const double a = jj > 0 ? fma(vp[i], wc, col[i]) : A[(size_t)c * lda + r + i];
        col[i] = a;                          // the reflector overwrites it below
        if (i > 0) sq = fma(a, a, sq);
    }
    // rows above the reflector's first row hold zeros in V and W
    for (int i = tid; i < off; i += CT) {
        V[(size_t)jj * ldv + i] = 0.0;
        W[(size_t)jj * ldv + i] = 0.0;
    }
    sq = wave_sum(sq);
    if ((tid & 63) == 0) red[tid >> 6] = sq;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int q = 0; q < CT / 64; ++q) s += red[q];
        const double x0 = col[0];
        double t = 0.0, beta = x0, scale = 0.0;
        if (s != 0.0) {
            const double nrm = sqrt(x0 * x0 + s);
            beta = (x0 >= 0.0) ? -nrm : nrm;
            t = (beta - x0) / beta;
            scale = 1.0 / (x0 - beta);
        }
        bsc[0] = scale;
        tau[jj] = t;
        alpha[c] = -beta;                    // super-diagonal: A_trd[c, c+1] = -A_trd[c+1, c]
    }
    __syncthreads();
    const double scale = bsc[0];
    for (int i = tid; i < m; i += CT) col[i] = (i == 0) ? 1.0 : col[i] * scale;
}

// Lower tiles (I >= J) of the stored trailing block A(r:, r:) (m x m), in
// vertical strips of up to ss tiles of one column block J (strip s holds the
// row blocks I in [nt - (s+1) ss, nt - s ss) with I >= J), one strip per
// workgroup so that a workgroup streams up to ss x 32 KB (ss from
// strip_len: long strips for large blocks, single tiles for small ones,
// where the strip's tiles would run one after another): tile (I, J) writes
// Prow(I, J) = L_IJ v_J (64), and the strip writes Pcol(J, s) = sum over its
// tiles of L_IJ^T v_I (64; accumulated in registers, reduced across the lanes
// once per strip).  Diagonal tiles use the strict lower part only and write
// the partial dot products Pd[I] = (V(:, k)^T v, W(:, k)^T v) (k < jj) over
// their 64 rows.
constexpr int SS = 8;     // longest strip

__host__ __device__ __forceinline__ int strip_len(int nt) { return nt >= 16 * SS ? SS : (nt >= 16 ? nt / 16 : 1); }

__device__ __forceinline__ int strips(int nt) { return (nt + strip_len(nt) - 1) / strip_len(nt); }

// workgroup t -> strip s, column block J: strip s spans the column blocks
// J < nt - s ss
__device__ __forceinline__ void strip_of(int t, int nt, int ss, int &s, int &J)
{
    s = 0;
    while (t >= nt - s * ss) {
        t -= nt - s * ss;
        ++s;
    }
    J = t;
}

__global__ __launch_bounds__(256) void k_os_symv(const double *__restrict__ A, int lda, int r, int m,
                                                 const double *__restrict__ v, const double *__restrict__ V,
                                                 const double *__restrict__ W, int ldv, int off, int jj,
                                                 double *__restrict__ Prow, double *__restrict__ Pcol,
                                                 double *__restrict__ Pd)
{
    __shared__ double vI[OT], vJ[OT], part[4][OT];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int nt = (m + OT - 1) / OT, ss = strip_len(nt);
    int s, J;
    strip_of(blockIdx.x, nt, ss, s, J);
    const int Ib = max(J, nt - (s + 1) * ss), Ie = nt - s * ss;
    const int j0 = J * OT;
    if (tid < OT) vJ[tid] = (j0 + tid < m) ? v[j0 + tid] : 0.0;
    const double *Ab = A + (size_t)r * lda + r;
    double cs[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) cs[q] = 0.0;
    for (int I = Ib; I < Ie; ++I) {
        const int i0 = I * OT, i = i0 + tx;
        if (tid < OT) vI[tid] = (i0 + tid < m) ? v[i0 + tid] : 0.0;
        __syncthreads();
        const double vi = vI[tx];
        double rs = 0.0;
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
            const int jl = ty + 4 * q, j = j0 + jl;
            const bool in = i < m && j < m && (I != J || tx > jl);
            const double x = in ? Ab[(size_t)j * lda + i] : 0.0;
            rs = fma(x, vJ[jl], rs);
            cs[q] = fma(x, vi, cs[q]);
        }
        part[ty][tx] = rs;
        __syncthreads();
        if (ty == 0)
            Prow[(size_t)(I * (I + 1) / 2 + J) * OT + tx] = part[0][tx] + part[1][tx] + part[2][tx] + part[3][tx];
        if (I == J) {
            // partial dots over rows i0 .. i0 + 63 of the trailing block: wave w
            // takes k = w, w + 4, ... (V) and the same for W, all loads first
            double a[16], b[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int k = ty + 4 * u;
                const bool ok = k < jj && i < m;
                a[u] = ok ? V[(size_t)k * ldv + off + i] : 0.0;
                b[u] = ok ? W[(size_t)k * ldv + off + i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int k = ty + 4 * u;
                if (k >= jj) break;
                const double sa = wave_sum(a[u] * vi), sb = wave_sum(b[u] * vi);
                if (tx == 0) {
                    Pd[(size_t)I * 128 + k] = sa;
                    Pd[(size_t)I * 128 + 64 + k] = sb;
                }
            }
        }
        __syncthreads();                     // vI and part are rewritten by the next tile
    }
    double *pc = Pcol + ((size_t)J * strips(nt) + s) * OT;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const double c = wave_sum(cs[q]);
        if (tx == 0) pc[ty + 4 * q] = c;
    }
}

// D[0..jj) = V^T v, D[64..64+jj) = W^T v summed over the nt row blocks (wave
// q takes the blocks I = q mod 4, four at a time; the four wave sums are added
// in order); T(:jj, jj) = -tau T(:jj, :jj) V^T v, T(jj, jj) = tau (T
// column-major, ldt = 64; T(:jj, :jj) is staged in LDS first).
__global__ __launch_bounds__(256) void k_os_dots(const double *__restrict__ Pd, int nt, int jj,
                                                 const double *__restrict__ tau, double *__restrict__ D,
                                                 double *__restrict__ T)
{
    __shared__ double Ts[64 * 64];
    __shared__ double pa[4][64], pb[4][64], dv[64];
    const int tid = threadIdx.x, k = tid & 63, q = tid >> 6;
    for (int e = tid; e < jj * 64; e += 256) Ts[e] = T[e];
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
    if (k < jj) {
        int I = q;
        for (; I + 4 < nt; I += 8) {
            a0 += Pd[(size_t)I * 128 + k];
            b0 += Pd[(size_t)I * 128 + 64 + k];
            a1 += Pd[(size_t)(I + 4) * 128 + k];
            b1 += Pd[(size_t)(I + 4) * 128 + 64 + k];
        }
        if (I < nt) {
            a0 += Pd[(size_t)I * 128 + k];
            b0 += Pd[(size_t)I * 128 + 64 + k];
        }
    }
    pa[q][k] = a0 + a1;
    pb[q][k] = b0 + b1;
    __syncthreads();
    if (q == 0) {
        const double a = ((pa[0][k] + pa[1][k]) + pa[2][k]) + pa[3][k];
        const double b = ((pb[0][k] + pb[1][k]) + pb[2][k]) + pb[3][k];
        D[k] = a;
        D[64 + k] = b;
        dv[k] = a;
    }
    __syncthreads();
    if (q == 0) {
        const double t = tau[jj];
        if (k < jj) {
            double s = 0.0;
            for (int u = k; u < jj; ++u) s = fma(Ts[u * 64 + k], dv[u], s);   // T upper
            T[(size_t)jj * 64 + k] = -t * s;
        } else {
            T[(size_t)jj * 64 + k] = (k == jj) ? t : 0.0;
        }
    }
}

// w for rows i0 .. i0 + 63 of the trailing block: y = sum of the tile
// partials (Prow of tiles (I, J <= I), minus Pcol of the strips of column
// block I), then
// w = tau (y + V (W^T v) - W (V^T v)) into column jj of W.  With next set, the
// next column (c + 1 = r) below its diagonal gets A(r+i, r) + sum over k < jj of
// (V(i, k) W(r, k) - W(i, k) V(r, k)) - w(i) into column jj + 1 of V: all of
// its deferred update but V(:, jj) w(r).  Wave q takes the tiles and the
// columns k = q mod 4; the four wave sums are added in order.
__global__ __launch_bounds__(256) void k_os_w(const double *__restrict__ A, int lda, int r, int m, int nt,
                                              const double *__restrict__ Prow, const double *__restrict__ Pcol,
                                              const double *__restrict__ D, double *__restrict__ V,
                                              double *__restrict__ W, int ldv, int off, int jj,
                                              const double *__restrict__ tau, int next)
{
    __shared__ double py[4][OT], pn[4][OT];
    const int I = blockIdx.x, tx = threadIdx.x & 63, q = threadIdx.x >> 6, i = I * OT + tx;
    const bool in = i < m;
    const bool nx = next && i > 0 && in;
    double y0 = 0.0, y1 = 0.0, a = 0.0;
    const double *pr = Prow + (size_t)(I * (I + 1) / 2) * OT + tx;
    for (int J = q; J <= I; J += 8) {
        y0 += pr[(size_t)J * OT];
        if (J + 4 <= I) y1 += pr[(size_t)(J + 4) * OT];
    }
    // the strips of column block I: s < ceil((nt - I) / ss)
    const int ss = strip_len(nt);
    const double *pc = Pcol + (size_t)I * strips(nt) * OT + tx;
    for (int s = q; s * ss < nt - I; s += 4) y0 -= pc[(size_t)s * OT];
    if (in)
        for (int k = q; k < jj; k += 4) {
            const double vik = V[(size_t)k * ldv + off + i], wik = W[(size_t)k * ldv + off + i];
            y0 += vik * D[64 + k] - wik * D[k];
            if (nx) a += vik * W[(size_t)k * ldv + off] - wik * V[(size_t)k * ldv + off];
        }
    py[q][tx] = y0 + y1;
    pn[q][tx] = a;
    __syncthreads();
    if (q != 0 || !in) return;
    const double y = ((py[0][tx] + py[1][tx]) + py[2][tx]) + py[3][tx];
    const double w = tau[jj] * y;
    W[(size_t)jj * ldv + off + i] = w;
    if (nx) {
        const double an = ((pn[0][tx] + pn[1][tx]) + pn[2][tx]) + pn[3][tx];
        V[(size_t)(jj + 1) * ldv + off + i] = A[(size_t)r * lda + r + i] + an - w;
    }
}

}  // namespace

namespace skew {

size_t onestage_scratch_doubles(int n)
{
    const size_t nt = (size_t)(n + OT - 1) / OT;
    return (nt * (nt + 1) / 2) * OT + nt * nt * OT + nt * 128 + 128;     // Pcol: up to nt strips per block
}

// Reduce the panel of columns c0 .. c0 + nb - 1 (nb <= 64) of the skew matrix
// whose strict lower triangle is in A (lda), then update the trailing block.
// V, W: (n - c0 - 1) x 64 (ldv = n - c0 - 1); tau[64]; T: 64 x 64; alpha: the
// super-diagonal; scratch: onestage_scratch_doubles(n).
void launch_onestage_panel(double *A, int lda, int n, int c0, int nb, double *V, double *W, int ldv, double *tau,
                           double *T, double *alpha, double *scratch, hipStream_t st)
{
    const size_t ntm = (size_t)(n + OT - 1) / OT;
    double *Prow = scratch, *Pcol = Prow + (ntm * (ntm + 1) / 2) * OT;
    double *Pd = Pcol + ntm * ntm * OT;
    double *D = Pd + ntm * 128;
    for (int jj = 0; jj < nb; ++jj) {
        const int c = c0 + jj, r = c + 1, m = n - r, off = r - (c0 + 1);
        hipLaunchKernelGGL(k_os_col, dim3(1), dim3(CT), 0, st, (const double *)A, lda, n, c0, jj, V, W, ldv, tau,
                           alpha);
        const int nt = (int)cdiv(m, OT);
        const int ss = strip_len(nt);
        int nwg = 0;                                     // strips: nt - s ss column blocks each
        for (int s = 0; s * ss < nt; ++s) nwg += nt - s * ss;
        hipLaunchKernelGGL(k_os_symv, dim3(nwg), dim3(256), 0, st, (const double *)A, lda, r, m,
                           (const double *)(V + (size_t)jj * ldv + off), (const double *)V, (const double *)W, ldv,
                           off, jj, Prow, Pcol, Pd);
        hipLaunchKernelGGL(k_os_dots, dim3(1), dim3(256), 0, st, (const double *)Pd, nt, jj, (const double *)tau, D, T);
        hipLaunchKernelGGL(k_os_w, dim3(nt), dim3(256), 0, st, (const double *)A, lda, r, m, nt, (const double *)Prow,
                           (const double *)Pcol, (const double *)D, V, W, ldv, off, jj, (const double *)tau,
                           (int)(jj + 1 < nb));
    }
    // trailing update of the columns after the panel: rows and columns from c0 + nb
    const int r0 = c0 + nb, m0 = n - r0;
    if (m0 > 1) launch_syr2k_ld<double>(A, lda, r0, m0, nb, V + (r0 - (c0 + 1)), W + (r0 - (c0 + 1)), ldv, st);
}

}  // namespace skew
