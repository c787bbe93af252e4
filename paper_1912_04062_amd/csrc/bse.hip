// The Bethe-Salpeter route around the skew-symmetric solver (Section 3, the
// four steps of the BSEPACK method):
//   1. M = [[Re(A+B), Im(A-B)], [-Im(A+B), Re(A-B)]] (Eq. SymmetricM: M = JH
//      with H the real Hamiltonian of Theorem 2), n = 2m, lower triangle;
//   2. Cholesky M = L L^T, blocked by 64: the diagonal block in one workgroup
//      (k_chol_diag, which also keeps R^{-1} of its block, R = L_jj^T), the
//      panel below by L_pj = M_pj R^{-1} (k_panel_solve, in place), the
//      trailing lower tiles by M -= L_pj L_pj^T (k_syrk_lower, MFMA);
//   3. K = L^T J L, J = [[0, I], [-I, 0]], lower tiles (k_ltjl, MFMA); its
//      eigenpairs come from the skew-symmetric solver;
//   4. back-transformation: W = L^{-T} Z by blocks from the bottom (split-K
//      W_j-partials L_{>j,j}^T W_{>j}, then k_trsm_block W_j = R_j^{-1} (Z_j -
//      sum)), and x = sqrt(lambda) Q W with Q = [[I, -iI], [I, iI]] / sqrt(2)
//      of Theorem 2 (k_bse_x): H_BS x = lambda x with x^H S x = 1.
#include "common.h"
#include "gemm.h"
#include "kernels.h"
#include "small64.h"

namespace {

constexpr int NB = 64;

// Step 1: the lower triangle of M (n x n, ldm) from the real and imaginary
// planes of A (Hermitian) and B (complex symmetric), m x m each.
__global__ void k_bse_build_m(const double *__restrict__ Ar, const double *__restrict__ Ai, int lda,
                              const double *__restrict__ Br, const double *__restrict__ Bi, int ldb, int m,
                              double *__restrict__ M, int ldm, unsigned *flags)
{
    const int j = blockIdx.y;                // column of M
    const int n = 2 * m;
    bool bad = false;
    for (int i = j + blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        double v;
        if (j < m) {
            const size_t a = (size_t)j * lda + (i < m ? i : i - m), bb = (size_t)j * ldb + (i < m ? i : i - m);
            v = (i < m) ? Ar[a] + Br[bb] : -(Ai[a] + Bi[bb]);     // Re(A+B) ; -Im(A+B)
        } else {
            const size_t a = (size_t)(j - m) * lda + (i - m), bb = (size_t)(j - m) * ldb + (i - m);
            v = Ar[a] - Br[bb];                                   // Re(A-B)
        }
        if (!__builtin_isfinite(v)) bad = true;
        M[(size_t)j * ldm + i] = v;
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, 1u);
}

// Step 2, diagonal block j0 (nb <= 64): M_jj = R^T R (R = L_jj^T) from its
// lower triangle; L_jj goes back into the lower triangle of M, R^{-1} to Rinv
// (64 x 64, column-major).  A pivot that is not positive sets bit 4 of *flags
// (M not positive definite) and the block is left as it is.
__global__ __launch_bounds__(256) void k_chol_diag(double *__restrict__ M, int ldm, int j0, int nb,
                                                   double *__restrict__ Rinv, unsigned *flags)
{
    __shared__ double G[64 * 65], X[64 * 65];
    __shared__ __attribute__((aligned(16))) double buf[320];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    if (*flags & 4u) return;                  // an earlier block already failed
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int c = ty + 4 * q;
        double v = 0.0;
        if (tx < nb && c < nb) {
            const int r0 = max(tx, c), c0 = min(tx, c);
            v = M[(size_t)(j0 + c0) * ldm + j0 + r0];
        }
        G[tx * 65 + c] = v;
    }
    __syncthreads();
    if (!chol_inv64(G, X, nb, false, 0.0, 1.7976931348623157e308, buf)) {
        if (tid == 0) atomicOr(flags, 4u);
        return;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int c = ty + 4 * q;
        if (tx < nb && c < nb && tx >= c) M[(size_t)(j0 + c) * ldm + j0 + tx] = G[c * 65 + tx];   // L = R^T
        Rinv[(size_t)c * NB + tx] = (tx <= c && c < nb) ? X[tx * 65 + c] : 0.0;
    }
}

// Step 2, panel: M[r0:r0+mr, j0:j0+nb] <- M[...] R^{-1} in place (each
// workgroup owns TM whole rows of the panel and reads them before writing).
template <int TM>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_panel_solve(double *__restrict__ M, int ldm, int r0, int mr,
                                                               int j0, int nb, const double *__restrict__ Rinv,
                                                               const unsigned *__restrict__ flags)
{
    extern __shared__ char smraw[];
    double *smem = (double *)smraw;
    if (*flags & 4u) return;
    const int m0 = blockIdx.x * TM;
    auto fa = [=](int i, int k) -> double {
        return (i < mr && k < nb) ? M[(size_t)(j0 + k) * ldm + r0 + i] : 0.0;
    };
    auto fb = [=](int c, int k) -> double { return (c < nb && k < nb) ? Rinv[(size_t)c * NB + k] : 0.0; };
    gemm::Acc<double, TM, 64> acc;
    acc.zero();
    gemm::kloop<double, TM, 64, false, true>(fa, fb, m0, 0, 0, NB, smem, acc);
    gemm::epilogue<double, TM, 64>(acc, smem, [=](int i, int c, double v) {
        if (m0 + i < mr && c < nb) M[(size_t)(j0 + c) * ldm + r0 + m0 + i] = v;
    });
}

// Step 2, trailing update: lower tiles (I >= J) of M[r0:, r0:] -= P P^T with
// P = M[r0:r0+mr, j0:j0+nb] (the panel just solved).
template <int TT>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_syrk_lower(double *__restrict__ M, int ldm, int r0, int mr,
                                                              int j0, int nb, const unsigned *__restrict__ flags)
{
    extern __shared__ char smraw[];
    double *smem = (double *)smraw;
    if (*flags & 4u) return;
    int I, J;
    tri_index(blockIdx.x, I, J);
    const int m0 = I * TT, n0 = J * TT;
    auto fp = [=](int i, int k) -> double {
        return (i < mr && k < nb) ? M[(size_t)(j0 + k) * ldm + r0 + i] : 0.0;
    };
    gemm::Acc<double, TT, TT> acc;
    acc.zero();
    gemm::kloop<double, TT, TT, false, false>(fp, fp, m0, n0, 0, NB, smem, acc);
    gemm::epilogue_rmw<double, TT, TT>(
        acc, smem,
        [=](int i, int j) -> double {
            return M[(size_t)(r0 + min(n0 + j, mr - 1)) * ldm + r0 + min(m0 + i, mr - 1)];
        },
        [=](int i, int j, double old, double v) {
            const int gi = m0 + i, gj = n0 + j;
            if (gi < mr && gj <= gi) M[(size_t)(r0 + gj) * ldm + r0 + gi] = old - v;
        });
}

// Step 3: lower tiles of K = L^T (J L): K_ij = sum_{k >= i} L_ki (JL)_kj with
// (JL)_kj = L_{k+m, j} (k < m), -L_{k-m, j} (k >= m); L lower (ldl).
template <int TT>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_ltjl(const double *__restrict__ L, int ldl, int m,
                                                        double *__restrict__ K, int ldk)
{
    extern __shared__ char smraw[];
    double *smem = (double *)smraw;
    const int n = 2 * m;
    int I, J;
    tri_index(blockIdx.x, I, J);
    const int m0 = I * TT, n0 = J * TT;
    // A(i, k) = L[k, i], zero above the diagonal of L; consecutive k contiguous
    auto fa = [=](int i, int k) -> double {
        return (i < n && k < n && k >= i) ? L[(size_t)i * ldl + k] : 0.0;
    };
    auto fb = [=](int j, int k) -> double {
        if (j >= n || k >= n) return 0.0;
        const int r = (k < m) ? k + m : k - m;
        const double x = (r >= j) ? L[(size_t)j * ldl + r] : 0.0;
        return (k < m) ? x : -x;
    };
    gemm::Acc<double, TT, TT> acc;
    acc.zero();
    gemm::kloop<double, TT, TT, true, true>(fa, fb, m0, n0, m0, n, smem, acc);
    gemm::epilogue<double, TT, TT>(acc, smem, [=](int i, int j, double v) {
        const int gi = m0 + i, gj = n0 + j;
        if (gi < n && gj < n && gj <= gi) K[(size_t)gj * ldk + gi] = v;
    });
}

// Step 4, block j0 of W = L^{-T} Z (Z = [Re | Im], n x ncols, in place):
// W_j = R_j^{-1} (Z_j - sum_s Wp[s]), Wp = partials of L_{>j,j}^T W_{>j}
// (nb x ncols each).  One workgroup of 64 threads per column.
__global__ __launch_bounds__(64) void k_trsm_block(double *__restrict__ Z, int ldz, int j0, int nb,
                                                   const double *__restrict__ Rinv, const double *__restrict__ Wp,
                                                   int S, int ncols)
{
    __shared__ double y[64];
    const int c = blockIdx.x, t = threadIdx.x;
    double v = 0.0;
    if (t < nb) {
        v = Z[(size_t)c * ldz + j0 + t];
        for (int s = 0; s < S; ++s) v -= Wp[((size_t)s * ncols + c) * nb + t];
    }
    y[t] = v;
    __syncthreads();
    if (t < nb) {
        double r = 0.0;
        for (int k = t; k < nb; ++k) r = fma(Rinv[(size_t)k * NB + t], y[k], r);   // R^{-1} upper
        Z[(size_t)c * ldz + j0 + t] = r;
    }
}

// Step 4, x = sqrt(lambda) Q W: W = Wr + i Wi (2m x nev, columns of Z = [Wr |
// Wi]); x_top = (w_top - i w_bot) s, x_bot = (w_top + i w_bot) s with
// s = sqrt(lambda / 2).
__global__ void k_bse_x(const double *__restrict__ Z, int ldz, int m, int nev, const double *__restrict__ lam,
                        double *__restrict__ Xr, double *__restrict__ Xi, int ldx)
{
    const int k = blockIdx.y;
    const double s = sqrt(0.5 * fmax(lam[k], 0.0));
    const double *wr = Z + (size_t)k * ldz, *wi = Z + (size_t)(nev + k) * ldz;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
        const double tr = wr[i], ti = wi[i], br = wr[m + i], bi = wi[m + i];
        Xr[(size_t)k * ldx + i] = s * (tr + bi);
        Xi[(size_t)k * ldx + i] = s * (ti - br);
        Xr[(size_t)k * ldx + m + i] = s * (tr - bi);
        Xi[(size_t)k * ldx + m + i] = s * (ti + br);
    }
}

}  // namespace

namespace skew {

void launch_bse_build_m(const double *Ar, const double *Ai, int lda, const double *Br, const double *Bi, int ldb,
                        int m, double *M, int ldm, unsigned *flags, hipStream_t st)
{
    const int n = 2 * m;
    if (n <= 0) return;
    dim3 grid(cdiv(n, 256) > 16 ? 16 : cdiv(n, 256), n);
    hipLaunchKernelGGL(k_bse_build_m, grid, dim3(256), 0, st, Ar, Ai, lda, Br, Bi, ldb, m, M, ldm, flags);
}

void launch_cholesky(double *M, int ldm, int n, double *Rinv_all, unsigned *flags, hipStream_t st)
{
    constexpr int TMP = 128, TT = 64;
    for (int j0 = 0; j0 < n; j0 += NB) {
        const int nb = min(NB, n - j0);
        double *Rinv = Rinv_all + (size_t)(j0 / NB) * NB * NB;
        hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, st, M, ldm, j0, nb, Rinv, flags);
        const int r0 = j0 + nb, mr = n - r0;
        if (mr <= 0) continue;
        hipLaunchKernelGGL((k_panel_solve<TMP>), dim3(cdiv(mr, TMP)), dim3(256), (gemm::smem_bytes<double, TMP, 64>()),
                           st, M, ldm, r0, mr, j0, nb, (const double *)Rinv, (const unsigned *)flags);
        const unsigned nt = cdiv(mr, TT);
        hipLaunchKernelGGL((k_syrk_lower<TT>), dim3(nt * (nt + 1) / 2), dim3(256), (gemm::smem_bytes<double, TT, TT>()),
                           st, M, ldm, r0, mr, j0, nb, (const unsigned *)flags);
    }
}

void launch_ltjl(const double *L, int ldl, int m, double *K, int ldk, hipStream_t st)
{
    constexpr int TT = 64;
    const int n = 2 * m;
    if (n <= 0) return;
    const unsigned nt = cdiv(n, TT);
    hipLaunchKernelGGL((k_ltjl<TT>), dim3(nt * (nt + 1) / 2), dim3(256), (gemm::smem_bytes<double, TT, TT>()), st, L,
                       ldl, m, K, ldk);
}

void launch_trsm_lt(const double *L, int ldl, int n, const double *Rinv_all, double *Z, int ldz, int ncols,
                    double *Wp, hipStream_t st)
{
    const int nblk = (int)cdiv(n, NB);
    for (int b = nblk - 1; b >= 0; --b) {
        const int j0 = b * NB, nb = min(NB, n - j0), r0 = j0 + nb, rest = n - r0;
        int S = 0;
        if (rest > 0)
            S = launch_gemm_tn_part<double>(L + (size_t)j0 * ldl + r0, ldl, Z + r0, ldz, nb, ncols, rest, Wp, st);
        hipLaunchKernelGGL(k_trsm_block, dim3(ncols), dim3(64), 0, st, Z, ldz, j0, nb,
                           Rinv_all + (size_t)b * NB * NB, (const double *)Wp, S, ncols);
    }
}

void launch_bse_x(const double *Z, int ldz, int m, int nev, const double *lam, double *Xr, double *Xi, int ldx,
                  hipStream_t st)
{
    if (m <= 0 || nev <= 0) return;
    hipLaunchKernelGGL(k_bse_x, dim3(cdiv(m, 256) > 8 ? 8 : cdiv(m, 256), nev), dim3(256), 0, st, Z, ldz, m, nev,
                       lam, Xr, Xi, ldx);
}

}  // namespace skew
