// Iterative refinement of the eigenpairs for the precision form.
//
// The eigenvectors z_k = x_k + i y_k of the +i lambda_k (lambda_k > 0) satisfy
// A x = -lambda y, A y = lambda x, so the real basis X = sqrt(2) [x_1 y_1 x_2
// y_2 ...] (plus the real null vector first when n is odd) is orthogonal and
// block-diagonalizes A:  X^T A X = D = blockdiag(lambda_k J), J = [[0,1],[-1,0]]
// (a 1x1 zero block for the null vector).  One refinement sweep (Newton step
// in the style of Ogita and Aishima's refinement for symmetric eigenproblems,
// here in real-Schur block form):
//   P = A X;  S = X^T P (skew);  G = X^T X,  R = I - G (symmetric)
//   lambda_p from the diagonal blocks:  lambda_p = s12 (1 + (r11 + r22)/2)
//   E_pp = R_pp / 2;  for p != q the 2x2 Sylvester equation
//      D_p E_pq - E_pq D_q = -S_pq - R_pq D_q
//   (E_pq = R_pq / 2 where lambda_p and lambda_q are closer than the cluster
//   threshold);  X <- X + X E.
// With D_p = a J, D_q = c J, write M = J C for the right-hand side C; the
// part of E commuting with J is -M_c/(a - c) and the anti-commuting part is
// -M_a/(a + c), with M_c = (M - J M J)/2 and M_a = (M + J M J)/2.
// P, S and G are FP64 (FP64 MFMA, from the original FP64 A); the update X E
// runs on FP32 MFMA since E is small.
#include "common.h"
#include "gemm.h"
#include "kernels.h"

namespace {

// Column layout of X: block p occupies columns blk_col(p) .. + blk_size(p)-1.
__device__ __forceinline__ int blk_of_col(int c, int odd) { return odd ? (c + 1) >> 1 : c >> 1; }
__device__ __forceinline__ int blk_col(int p, int odd) { return odd ? (p == 0 ? 0 : 2 * p - 1) : 2 * p; }
__device__ __forceinline__ int blk_size(int p, int odd) { return (odd && p == 0) ? 1 : 2; }

// X (n x ncx, double) from Z = [Re | Im] (n x 2 nev, type T)
template <typename T>
__global__ void k_build_x(const T *__restrict__ Z, int ldz, int n, int nev, int odd, double *__restrict__ X)
{
    const int c = blockIdx.y;                 // column of X
    const int p = blk_of_col(c, odd);
    const bool zero_blk = odd && p == 0;
    const int within = c - blk_col(p, odd);
    const T *src = Z + (size_t)(within == 0 ? p : nev + p) * ldz;
    const double s = zero_blk ? 1.0 : 1.4142135623730951;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        X[(size_t)c * n + i] = s * (double)src[i];
}

// X -> Z_re, Z_im (double, user leading dimensions)
__global__ void k_split_x(const double *__restrict__ X, int n, int nev, int odd, double *__restrict__ Zr, int ldr,
                          double *__restrict__ Zi, int ldi)
{
    const int p = blockIdx.y;
    const int c0 = blk_col(p, odd);
    const bool zero_blk = odd && p == 0;
    const double s = zero_blk ? 1.0 : 0.7071067811865476;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        Zr[(size_t)p * ldr + i] = s * X[(size_t)c0 * n + i];
        Zi[(size_t)p * ldi + i] = zero_blk ? 0.0 : s * X[(size_t)(c0 + 1) * n + i];
    }
}

// P = A X with A skew, read from its strict lower triangle (lda), FP64.
template <int TM, int TN>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_skew_mm(const double *__restrict__ A, int lda, int n,
                                                 const double *__restrict__ X, int ncx, double *__restrict__ P)
{
    extern __shared__ char smraw[];
    double *smem = (double *)smraw;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    auto f_low = [=](int i, int k) -> double { return (i < n && k < n) ? A[(size_t)k * lda + i] : 0.0; };
    auto f_up = [=](int i, int k) -> double { return (i < n && k < n) ? -A[(size_t)i * lda + k] : 0.0; };
    auto f_mix = [=](int i, int k) -> double {
        if (i >= n || k >= n || i == k) return 0.0;
        return (i > k) ? A[(size_t)k * lda + i] : -A[(size_t)i * lda + k];
    };
    auto f_x = [=](int j, int k) -> double { return (j < ncx && k < n) ? X[(size_t)j * n + k] : 0.0; };
    gemm::Acc<double, TM, TN> acc;
    acc.zero();
    gemm::skew_kloop<double, TM, TN>(f_low, f_up, f_mix, f_x, m0, n0, 0, n, smem, acc);
    gemm::epilogue<double, TM, TN>(acc, smem, [=](int i, int j, double v) {
        if (m0 + i < n && n0 + j < ncx) P[(size_t)(n0 + j) * n + m0 + i] = v;
    });
}

// Lower tiles (I >= J) of S = X^T P and G = X^T X (both ncx x ncx, FP64).
template <int TT>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_xtp_xtx(const double *__restrict__ X, const double *__restrict__ P, int n,
                                                 int ncx, double *__restrict__ S, double *__restrict__ G)
{
    extern __shared__ char smraw[];
    double *smem = (double *)smraw;
    int t = blockIdx.x;
    int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int J = t - I * (I + 1) / 2;
    const int m0 = I * TT, n0 = J * TT;
    auto fa = [=](int i, int k) -> double { return (i < ncx && k < n) ? X[(size_t)i * n + k] : 0.0; };
    auto fp = [=](int j, int k) -> double { return (j < ncx && k < n) ? P[(size_t)j * n + k] : 0.0; };
    auto fx = [=](int j, int k) -> double { return (j < ncx && k < n) ? X[(size_t)j * n + k] : 0.0; };
    gemm::Acc<double, TT, TT> a1, a2;
    a1.zero();
    a2.zero();
    double *As = smem, *Bs = smem + gemm::TK * (TT + 1), *Cs = Bs + gemm::TK * (TT + 1);
    gemm::Frag<double, TT> ra, rb, rc;
    gemm::gload<double, TT, true>(ra, fa, m0, 0);
    gemm::gload<double, TT, true>(rb, fp, n0, 0);
    gemm::gload<double, TT, true>(rc, fx, n0, 0);
    for (int k0 = 0; k0 < n; k0 += gemm::TK) {
        gemm::lstore<double, TT, true>(As, ra);
        gemm::lstore<double, TT, true>(Bs, rb);
        gemm::lstore<double, TT, true>(Cs, rc);
        __syncthreads();
        if (k0 + gemm::TK < n) {
            gemm::gload<double, TT, true>(ra, fa, m0, k0 + gemm::TK);
            gemm::gload<double, TT, true>(rb, fp, n0, k0 + gemm::TK);
            gemm::gload<double, TT, true>(rc, fx, n0, k0 + gemm::TK);
        }
        gemm::mma_chunk<double, TT, TT>(As, Bs, a1);
        gemm::mma_chunk<double, TT, TT>(As, Cs, a2);
        __syncthreads();
    }
    gemm::epilogue<double, TT, TT>(a1, smem, [=](int i, int j, double v) {
        if (m0 + i < ncx && n0 + j < ncx) S[(size_t)(n0 + j) * ncx + m0 + i] = v;
    });
    gemm::epilogue<double, TT, TT>(a2, smem, [=](int i, int j, double v) {
        if (m0 + i < ncx && n0 + j < ncx) G[(size_t)(n0 + j) * ncx + m0 + i] = v;
    });
}

__device__ __forceinline__ void atomic_max_pos(double *addr, double v)
{
    // v >= 0: the bit patterns of non-negative doubles order like the values
    atomicMax((unsigned long long *)addr, (unsigned long long)__double_as_longlong(v));
}

// lambda_p per block and the convergence measures: stat[0] = max |R_ij|,
// stat[1] = max |S_ij| over off-diagonal blocks (i > j), stat[2] = max lambda.
__global__ void k_lambda(const double *__restrict__ S, const double *__restrict__ G, int ncx, int nblk, int odd,
                         double *__restrict__ lam, double *__restrict__ stat)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= nblk) return;
    const int c = blk_col(p, odd);
    double l = 0.0;
    if (blk_size(p, odd) == 2) {
        const double s12 = -S[(size_t)c * ncx + c + 1];        // S[c][c+1] = -S[c+1][c]
        const double r11 = 1.0 - G[(size_t)c * ncx + c];
        const double r22 = 1.0 - G[(size_t)(c + 1) * ncx + c + 1];
        l = s12 * (1.0 + 0.5 * (r11 + r22));
    }
    lam[p] = l;
    atomic_max_pos(&stat[2], fabs(l));
}

// Columns j = blockIdx.x, blockIdx.x + gridDim.x, ... (rows i >= j); one
// atomic per workgroup after a reduction in LDS.
__global__ __launch_bounds__(256) void k_stats(const double *__restrict__ S, const double *__restrict__ G, int ncx,
                                               int odd, double *__restrict__ stat)
{
    __shared__ double red[2][4];
    double mr = 0.0, ms = 0.0;
    for (int j = blockIdx.x; j < ncx; j += gridDim.x) {
        const int pj = blk_of_col(j, odd);
        for (int i = j + threadIdx.x; i < ncx; i += 256) {
            const double r = (i == j ? 1.0 : 0.0) - G[(size_t)j * ncx + i];
            mr = fmax(mr, fabs(r));
            if (blk_of_col(i, odd) != pj) ms = fmax(ms, fabs(S[(size_t)j * ncx + i]));
        }
    }
    mr = wave_max(mr);
    ms = wave_max(ms);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = mr;
        red[1][threadIdx.x >> 6] = ms;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomic_max_pos(&stat[0], fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3])));
        atomic_max_pos(&stat[1], fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3])));
    }
}

// E (ncx x ncx, type TE): one thread per block pair (p, q).
template <typename TE>
__global__ void k_eform(const double *__restrict__ S, const double *__restrict__ G, int ncx, int nblk, int odd,
                        const double *__restrict__ lam, double omega, TE *__restrict__ E, unsigned *nclust,
                        double *emax)
{
    const int p = blockIdx.x * 16 + threadIdx.x % 16;
    const int q = blockIdx.y * 16 + threadIdx.x / 16;
    double macc = 0.0;      // largest accepted off-diagonal correction of this thread
    if (p < nblk && q < nblk) {
        const int cp = blk_col(p, odd), sp = blk_size(p, odd);
        const int cq = blk_col(q, odd), sq = blk_size(q, odd);
        // S(i, j) and R(i, j) for any i, j from the lower triangles
        auto Sv = [&](int i, int j) -> double {
            if (i == j) return 0.0;
            return i > j ? S[(size_t)j * ncx + i] : -S[(size_t)i * ncx + j];
        };
        auto Rv = [&](int i, int j) -> double {
            double g = i >= j ? G[(size_t)j * ncx + i] : G[(size_t)i * ncx + j];
            return (i == j ? 1.0 : 0.0) - g;
        };
        double e[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        if (p == q) {
            for (int a = 0; a < sp; ++a)
                for (int b = 0; b < sq; ++b) e[a][b] = 0.5 * Rv(cp + a, cq + b);
        } else {
            const double a = lam[p], c = lam[q];
            double C[2][2];
            // C = -S_pq - R_pq D_q,  D_q = c J (J = [[0,1],[-1,0]]):  (R J)[i][0] = -R[i][1], (R J)[i][1] = R[i][0]
            for (int i = 0; i < sp; ++i)
                for (int j = 0; j < sq; ++j) {
                    double rj = 0.0;
                    if (sq == 2) rj = (j == 0) ? -Rv(cp + i, cq + 1) : Rv(cp + i, cq + 0);
                    C[i][j] = -Sv(cp + i, cq + j) - c * rj;
                }
            if (fabs(a - c) <= omega) {
                for (int i = 0; i < sp; ++i)
                    for (int j = 0; j < sq; ++j) e[i][j] = 0.5 * Rv(cp + i, cq + j);
            } else if (sp == 2 && sq == 2) {
                // M = J C
                const double M00 = C[1][0], M01 = C[1][1], M10 = -C[0][0], M11 = -C[0][1];
                // J M J = [[-M11, M10], [M01, -M00]]
                const double c00 = 0.5 * (M00 + M11), c01 = 0.5 * (M01 - M10);
                const double a00 = 0.5 * (M00 - M11), a01 = 0.5 * (M01 + M10);
                // commuting part [[c00, c01], [-c01, c00]], anti part [[a00, a01], [a01, -a00]]
                const double ic = -1.0 / (a - c), ia = -1.0 / (a + c);
                e[0][0] = ic * c00 + ia * a00;
                e[0][1] = ic * c01 + ia * a01;
                e[1][0] = -ic * c01 + ia * a01;
                e[1][1] = ic * c00 - ia * a00;
            } else if (sp == 1 && sq == 2) {
                // -c E J = C  ->  E = C J / c :  (C J)[0][0] = -C[0][1], (C J)[0][1] = C[0][0]
                e[0][0] = -C[0][1] / c;
                e[0][1] = C[0][0] / c;
            } else if (sp == 2 && sq == 1) {
                // a J E = C  ->  E = -J C / a :  (J C)[0][0] = C[1][0], (J C)[1][0] = -C[0][0]
                e[0][0] = -C[1][0] / a;
                e[1][0] = C[0][0] / a;
            }
        }
        // a Newton step is only valid for small corrections: a pair whose solution
        // is not small is near-degenerate at this accuracy; it keeps E = R/2 and is
        // counted (the caller then solves the problem in FP64 instead)
        if (p != q) {
            double mx = 0.0;
            for (int i = 0; i < sp; ++i)
                for (int j = 0; j < sq; ++j) mx = fmax(mx, fabs(e[i][j]));
            if (!(mx <= 0.25)) {
                for (int i = 0; i < sp; ++i)
                    for (int j = 0; j < sq; ++j) e[i][j] = 0.5 * Rv(cp + i, cq + j);
                atomicAdd(nclust, 1u);
            } else {
                macc = mx;
            }
        }
        for (int i = 0; i < sp; ++i)
            for (int j = 0; j < sq; ++j) E[(size_t)(cq + j) * ncx + cp + i] = (TE)e[i][j];
    }
    // the largest correction bounds what the step leaves behind (about the
    // current error times it); one atomic per workgroup
    __shared__ double red[4];
    macc = wave_max(macc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = macc;
    __syncthreads();
    if (threadIdx.x == 0) atomic_max_pos(emax, fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}

// Xn = X + X E  (ncx x ncx E), the product on the MFMA of type T.
template <typename T, typename TE, int TM, int TN>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_xe(const double *__restrict__ X, const TE *__restrict__ E, int n, int ncx,
                                            double *__restrict__ Xn)
{
    extern __shared__ char smraw[];
    T *smem = (T *)smraw;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    auto fa = [=](int i, int k) -> T { return (i < n && k < ncx) ? (T)X[(size_t)k * n + i] : T(0); };
    auto fb = [=](int j, int k) -> T { return (j < ncx && k < ncx) ? (T)E[(size_t)j * ncx + k] : T(0); };
    gemm::Acc<T, TM, TN> acc;
    acc.zero();
    gemm::kloop<T, TM, TN, false, true>(fa, fb, m0, n0, 0, ncx, smem, acc);
    // the old values come from X (double) and the result goes to Xn
    gemm::epilogue_rmw<T, TM, TN>(
        acc, smem,
        // unconditional load at a clamped address: values outside are never stored
        [=](int i, int j) -> double { return X[(size_t)min(n0 + j, ncx - 1) * n + min(m0 + i, n - 1)]; },
        [=](int i, int j, double old, T v) {
            const int gi = m0 + i, gj = n0 + j;
            if (gi < n && gj < ncx) Xn[(size_t)gj * n + gi] = old + (double)v;
        });
}

}  // namespace

namespace skew {

template <typename T>
void launch_build_x(const T *Z, int ldz, int n, int nev, int odd, double *X, hipStream_t st)
{
    const int ncx = odd ? 2 * nev - 1 : 2 * nev;
    hipLaunchKernelGGL(k_build_x<T>, dim3(cdiv(n, 256) > 8 ? 8 : cdiv(n, 256), ncx), dim3(256), 0, st, Z, ldz, n,
                       nev, odd, X);
}

void launch_split_x(const double *X, int n, int nev, int odd, double *Zr, int ldr, double *Zi, int ldi,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_split_x, dim3(cdiv(n, 256) > 8 ? 8 : cdiv(n, 256), nev), dim3(256), 0, st, X, n, nev, odd, Zr,
                       ldr, Zi, ldi);
}

void launch_refine_products(const double *A, int lda, int n, const double *X, int ncx, double *P, double *S,
                            double *G, hipStream_t st)
{
    dim3 g1(cdiv(n, 128), cdiv(ncx, 128));
    hipLaunchKernelGGL((k_skew_mm<128, 128>), g1, dim3(256), (gemm::smem_bytes<double, 128, 128>()), st, A, lda, n,
                       X, ncx, P);
    const int TT = 64;
    unsigned nt = cdiv(ncx, TT);
    size_t shm = sizeof(double) * 3 * gemm::TK * (TT + 1);
    if (shm < gemm::smem_bytes<double, 64, 64>()) shm = gemm::smem_bytes<double, 64, 64>();
    hipLaunchKernelGGL((k_xtp_xtx<64>), dim3(nt * (nt + 1) / 2), dim3(256), shm, st, X, (const double *)P, n, ncx, S,
                       G);
}

void launch_refine_eigs(const double *S, const double *G, int ncx, int nblk, int odd, double *lam, double *stat,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_lambda, dim3(cdiv(nblk, 256)), dim3(256), 0, st, S, G, ncx, nblk, odd, lam, stat);
    hipLaunchKernelGGL(k_stats, dim3(ncx < 1024 ? (ncx > 0 ? ncx : 1) : 1024), dim3(256), 0, st, S, G, ncx, odd, stat);
}

void launch_refine_update(const double *S, const double *G, int n, int ncx, int nblk, int odd, const double *lam,
                          double omega, float *E, const double *X, double *Xn, unsigned *nclust, double *emax,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_eform<float>, dim3(cdiv(nblk, 16), cdiv(nblk, 16)), dim3(256), 0, st, S, G, ncx, nblk, odd,
                       lam, omega, E, nclust, emax);
    dim3 g(cdiv(n, 128), cdiv(ncx, 128));
    hipLaunchKernelGGL((k_xe<float, float, 128, 128>), g, dim3(256), (gemm::smem_bytes<float, 128, 128>()), st, X,
                       (const float *)E, n, ncx, Xn);
}

template void launch_build_x<double>(const double *, int, int, int, int, double *, hipStream_t);
template void launch_build_x<float>(const float *, int, int, int, int, double *, hipStream_t);

}  // namespace skew
