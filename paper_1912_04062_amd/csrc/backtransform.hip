// Back-transformations (Algorithm 1, steps 3 and 4, in the two-stage form of
// Section 2.1) and the generic products they and the orthogonalization use.
//
//   k_dscale     step 3: Q <- D Q_diag with D = diag(i^k): row k of the real
//                part is +q_k (k = 0 mod 4), -q_k (k = 2 mod 4), 0 otherwise;
//                of the imaginary part +q_k (k = 1 mod 4), -q_k (k = 3 mod 4).
//                Real and imaginary parts are kept side by side, Z = [Re Im].
//   k_bt2_tfac   compact-WY factor T of each group of nb2 consecutive
//                bulge-chasing reflectors at the same step (their vectors form
//                a parallelogram: column i occupies rows i..i+b-1).
//   k_bt2_apply  stage-2 back-transformation  Z <- Q_trd Z: groups applied as
//                Z <- (I - V T V^T) Z, sweep-blocks in descending order and,
//                inside a sweep-block, steps in ascending order (reflectors of
//                one sweep act on disjoint rows; the only overlapping pairs
//                keep their order).  One workgroup per slab of NC columns;
//                the MFMA loops skip the zero triangles of the parallelogram.
//   k_gemm_tn_part / k_gemm_nn   split-K  A^T B  and  C (+)= alpha A B, used
//                by the stage-1 back-transformation Z <- (I - V T V^T) Z and
//                by the block Gram-Schmidt of the eigenvector basis.
#include "common.h"
#include "gemm.h"
#include "kernels.h"

namespace {

template <typename T>
__global__ void k_dscale(const double *__restrict__ Q, int ldq, int n, int nev, T *__restrict__ Z, int ldz)
{
    const int c = blockIdx.y;                     // 0 .. 2 nev - 1
    const bool im = c >= nev;
    const int k = im ? c - nev : c;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double q = Q[(size_t)k * ldq + i];
        const int r = i & 3;
        double z;
        if (!im) z = (r == 0) ? q : ((r == 2) ? -q : 0.0);
        else z = (r == 1) ? q : ((r == 3) ? -q : 0.0);
        Z[(size_t)c * ldz + i] = (T)z;
    }
}

// One workgroup per group; nb2 <= 64, b <= 64.
template <typename T>
__global__ __launch_bounds__(256) void k_bt2_tfac(const double *__restrict__ V2, const double *__restrict__ tau2,
                                                  int b, int nb2, T *__restrict__ T2, T *__restrict__ V2t)
{
    __shared__ double Vs[64 * 65];       // Vs[r][i]
    __shared__ double Gm[64 * 65];       // Gram (upper)
    __shared__ double Tm[64 * 65];
    __shared__ double tv[64];
    const size_t g = blockIdx.x;
    const int tid = threadIdx.x;
    const double *Vg = V2 + g * (size_t)b * nb2;
    for (int e = tid; e < b * nb2; e += 256) {
        int r = e % b, i = e / b;
        Vs[r * 65 + i] = Vg[e];
        if (V2t) V2t[g * (size_t)b * nb2 + e] = (T)Vg[e];
    }
    if (tid < nb2) tv[tid] = tau2[g * nb2 + tid];
    for (int e = tid; e < 64 * 65; e += 256) Tm[e] = 0.0;
    __syncthreads();
    // Gram: v_i . v_j (i < j), overlap rows j..i+b-1 (absolute), r = row - i
    for (int e = tid; e < nb2 * nb2; e += 256) {
        int i = e % nb2, j = e / nb2;
        if (i < j) {
            int d = j - i;
            double s = 0.0;
            for (int r = d; r < b; ++r) s += Vs[r * 65 + i] * Vs[(r - d) * 65 + j];
            Gm[i * 65 + j] = s;
        }
    }
    __syncthreads();
    for (int j = 0; j < nb2; ++j) {
        if (tid < j) {
            double s = 0.0;
            for (int u = tid; u < j; ++u) s += Tm[tid * 65 + u] * Gm[u * 65 + j];
            Tm[tid * 65 + j] = -tv[j] * s;
        }
        if (tid == j) Tm[j * 65 + j] = tv[j];
        __syncthreads();
    }
    T *To = T2 + g * (size_t)nb2 * nb2;
    for (int e = tid; e < nb2 * nb2; e += 256) {
        int i = e % nb2, j = e / nb2;
        To[e] = (T)Tm[i * 65 + j];       // column-major
    }
}

// Stage-2 application.  Z is n x ncols (column-major, ldz).  A workgroup owns
// NCT = 64 columns, processed as two halves of 32 that share the group's V and
// T staged in LDS.  LDS: Zs[128][33], Vs[b][nb2] and Ts[nb2][nb2] (ld 65),
// W1/W2 [64][33].
template <typename T>
__global__ __launch_bounds__(256) void k_bt2_apply(T *__restrict__ Z, int ldz, int n, int ncols, int b, int nb2,
                                                   const T *__restrict__ V2, const T *__restrict__ T2,
                                                   const int *__restrict__ goff, int nsig)
{
    constexpr int NC = 32, NCT = 64, LDZ = NC + 1, LDV = 65;
    __shared__ T Zs[128 * LDZ];
    __shared__ T Vs[64 * LDV];
    __shared__ T Ts[64 * LDV];
    __shared__ T W1[64 * LDZ];
    __shared__ T W2[64 * LDZ];
    typedef typename acc4<T>::type A4;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int Lmax = b + nb2 - 1;

    for (int sg = nsig - 1; sg >= 0; --sg) {
        const int g0 = goff[sg], g1 = goff[sg + 1];
        for (int g = g0; g < g1; ++g) {
            const int k = g - g0;
            const int base = sg * nb2 + 1 + k * b;
            if (base >= n) break;
            const int L = min(Lmax, n - base);
            const T *Vg = V2 + (size_t)g * b * nb2;
            const T *Tg = T2 + (size_t)g * nb2 * nb2;
            __syncthreads();
            for (int e = tid; e < b * nb2; e += 256) {
                int r = e % b, i = e / b;
                Vs[r * LDV + i] = Vg[e];
            }
            for (int e = tid; e < nb2 * nb2; e += 256) {
                int i = e % nb2, u = e / nb2;
                Ts[u * LDV + i] = Tg[e];          // Ts[u][i] = T[i][u]
            }
            for (int half = 0; half < NCT / NC; ++half) {
                const int col0 = blockIdx.x * NCT + half * NC;
                const int ncl = min(NC, ncols - col0);
                if (ncl <= 0) break;
                for (int e = tid; e < 128 * NC; e += 256) {
                    int r = e % 128, c = e / 128;
                    Zs[r * LDZ + c] = (r < L && c < ncl) ? Z[(size_t)(col0 + c) * ldz + base + r] : T(0);
                }
                __syncthreads();
                // W1 = Vpar^T Zs   (nb2 x NC); wave wv -> rows i in [16wv, 16wv+16)
                if (16 * wv < nb2) {
                    A4 acc0 = (A4)(T(0)), acc1 = (A4)(T(0));
                    const int i = 16 * wv + lr;
                    const int rbeg = 16 * wv, rend = min(16 * wv + 16 + b - 1, 128);
                    for (int r4 = rbeg; r4 < rend; r4 += 4) {
                        const int r = r4 + lk;
                        const int d = r - i;
                        T a = (i < nb2 && d >= 0 && d < b) ? Vs[d * LDV + i] : T(0);
                        T b0 = Zs[r * LDZ + lr], b1 = Zs[r * LDZ + 16 + lr];
                        acc0 = mfma_16x16x4(a, b0, acc0);
                        acc1 = mfma_16x16x4(a, b1, acc1);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        int row = 16 * wv + mfma_row<T>(lane, q);
                        W1[row * LDZ + lr] = acc0[q];
                        W1[row * LDZ + 16 + lr] = acc1[q];
                    }
                }
                __syncthreads();
                // W2 = T W1 (T upper triangular)
                if (16 * wv < nb2) {
                    A4 acc0 = (A4)(T(0)), acc1 = (A4)(T(0));
                    const int i = 16 * wv + lr;
                    for (int u4 = 16 * wv; u4 < nb2; u4 += 4) {
                        const int u = u4 + lk;
                        T a = (i < nb2 && u < nb2) ? Ts[u * LDV + i] : T(0);
                        T b0 = (u < nb2) ? W1[u * LDZ + lr] : T(0);
                        T b1 = (u < nb2) ? W1[u * LDZ + 16 + lr] : T(0);
                        acc0 = mfma_16x16x4(a, b0, acc0);
                        acc1 = mfma_16x16x4(a, b1, acc1);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        int row = 16 * wv + mfma_row<T>(lane, q);
                        W2[row * LDZ + lr] = acc0[q];
                        W2[row * LDZ + 16 + lr] = acc1[q];
                    }
                }
                __syncthreads();
                // Zs -= Vpar W2 ; row tiles mt = wv, wv+4 (128 rows = 8 tiles)
                for (int mt = wv; mt < 8; mt += 4) {
                    if (16 * mt >= L) continue;
                    A4 acc0 = (A4)(T(0)), acc1 = (A4)(T(0));
                    const int r = 16 * mt + lr;
                    int ibeg = max(0, 16 * mt - b + 1) & ~3;
                    int iend = min(nb2, 16 * mt + 16);
                    for (int i4 = ibeg; i4 < iend; i4 += 4) {
                        const int i = i4 + lk;
                        const int d = r - i;
                        T a = (i < nb2 && d >= 0 && d < b) ? Vs[d * LDV + i] : T(0);
                        T b0 = (i < nb2) ? W2[i * LDZ + lr] : T(0);
                        T b1 = (i < nb2) ? W2[i * LDZ + 16 + lr] : T(0);
                        acc0 = mfma_16x16x4(a, b0, acc0);
                        acc1 = mfma_16x16x4(a, b1, acc1);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        int row = 16 * mt + mfma_row<T>(lane, q);
                        Zs[row * LDZ + lr] -= acc0[q];
                        Zs[row * LDZ + 16 + lr] -= acc1[q];
                    }
                }
                __syncthreads();
                for (int e = tid; e < 128 * NC; e += 256) {
                    int r = e % 128, c = e / 128;
                    if (r < L && c < ncl) Z[(size_t)(col0 + c) * ldz + base + r] = Zs[r * LDZ + c];
                }
                __syncthreads();
            }
        }
    }
}

// Cpart[s] = A[kb:ke, 0:M]^T B[kb:ke, 0:N]   (A: K x M, B: K x N, column-major)
template <typename T, int TM, int TN>
__global__ __launch_bounds__(256) void k_gemm_tn_part(const T *__restrict__ A, int lda, const T *__restrict__ B,
                                                      int ldb, int M, int N, int K, int kchunk,
                                                      double *__restrict__ Cpart)
{
    extern __shared__ char smraw[];
    T *smem = (T *)smraw;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN, s = blockIdx.z;
    const int kb = s * kchunk, ke = min(K, kb + kchunk);
    auto fa = [=](int i, int k) -> T { return (i < M && k < ke) ? A[(size_t)i * lda + k] : T(0); };
    auto fb = [=](int j, int k) -> T { return (j < N && k < ke) ? B[(size_t)j * ldb + k] : T(0); };
    gemm::Acc<T, TM, TN> acc;
    acc.zero();
    gemm::kloop<T, TM, TN, true, true>(fa, fb, m0, n0, kb, ke, smem, acc);
    double *C = Cpart + (size_t)s * M * N;
    gemm::epilogue<T, TM, TN>(acc, smem, [=](int i, int j, T v) {
        if (m0 + i < M && n0 + j < N) C[(size_t)(n0 + j) * M + m0 + i] = (double)v;
    });
}

// C = beta*C + alpha * A (M x K, column-major) * Bsum, Bsum = sum_s Bpart[s]
// (K x N, column-major ld K, S parts, double).
template <typename T, int TM, int TN>
__global__ __launch_bounds__(256) void k_gemm_nn(const T *__restrict__ A, int lda, const double *__restrict__ Bpart,
                                                 int S, int M, int N, int K, T *__restrict__ C, int ldc,
                                                 double alpha, int beta)
{
    extern __shared__ char smraw[];
    T *smem = (T *)smraw;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const size_t pst = (size_t)K * N;
    auto fa = [=](int i, int k) -> T { return (i < M && k < K) ? A[(size_t)k * lda + i] : T(0); };
    auto fb = [=](int j, int k) -> T {
        if (j >= N || k >= K) return T(0);
        double s = 0.0;
        for (int p = 0; p < S; ++p) s += Bpart[p * pst + (size_t)j * K + k];
        return (T)s;
    };
    gemm::Acc<T, TM, TN> acc;
    acc.zero();
    gemm::kloop<T, TM, TN, false, true>(fa, fb, m0, n0, 0, K, smem, acc);
    gemm::epilogue_rmw<T, TM, TN>(
        acc, smem,
        [=](int i, int j) -> T {
            const int gi = m0 + i, gj = n0 + j;
            return (beta && gi < M && gj < N) ? C[(size_t)gj * ldc + gi] : T(0);
        },
        [=](int i, int j, T old, T v) {
            const int gi = m0 + i, gj = n0 + j;
            if (gi < M && gj < N) C[(size_t)gj * ldc + gi] = (T)((double)old + alpha * (double)v);
        });
}

// out = S0 * sum_s Cpart[s]  (S0: M x M column-major, M <= 64) or, with
// S0 == nullptr, out = sum_s Cpart[s].  One workgroup per column.
__global__ __launch_bounds__(256) void k_reduce_left(const double *__restrict__ S0, const double *__restrict__ Cpart,
                                                     int S, int M, int N, double *__restrict__ out)
{
    extern __shared__ double cs[];        // M (+ M*M when S0)
    const size_t pst = (size_t)M * N;
    const int j = blockIdx.x;
    for (int u = threadIdx.x; u < M; u += 256) {
        double c = 0.0;
        for (int p = 0; p < S; ++p) c += Cpart[p * pst + (size_t)j * M + u];
        cs[u] = c;
    }
    if (!S0) {
        for (int u = threadIdx.x; u < M; u += 256) out[(size_t)j * M + u] = cs[u];
        return;
    }
    double *Ss = cs + M;
    for (int e = threadIdx.x; e < M * M; e += 256) Ss[e] = S0[e];
    __syncthreads();
    for (int i = threadIdx.x; i < M; i += 256) {
        double s = 0.0;
        for (int u = 0; u < M; ++u) s += Ss[(size_t)u * M + i] * cs[u];
        out[(size_t)j * M + i] = s;
    }
}

template <typename T>
__global__ void k_copy_cols(const T *__restrict__ src, int lds, T *__restrict__ dst, int ldd, int m, int ncol)
{
    const int c = blockIdx.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256)
        dst[(size_t)c * ldd + i] = src[(size_t)c * lds + i];
}

template <typename T>
__global__ void k_to_double(const T *__restrict__ src, int lds, double *__restrict__ dst, int ldd, int m)
{
    const int c = blockIdx.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256)
        dst[(size_t)c * ldd + i] = (double)src[(size_t)c * lds + i];
}

}  // namespace

namespace skew {

template <typename T>
void launch_dscale(const double *Q, int ldq, int n, int nev, T *Z, int ldz, hipStream_t st)
{
    if (nev <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_dscale<T>, dim3(cdiv(n, 256) > 8 ? 8 : cdiv(n, 256), 2 * nev), dim3(256), 0, st, Q, ldq,
                       n, nev, Z, ldz);
}

template <typename T>
void launch_bt2(T *Z, int ldz, int n, int ncols, int b, int nb2, const double *V2, const double *tau2, T *T2,
                T *V2t, const int *goff_dev, int nsig, int ngroups, hipStream_t st)
{
    if (ngroups <= 0 || ncols <= 0) return;
    hipLaunchKernelGGL(k_bt2_tfac<T>, dim3(ngroups), dim3(256), 0, st, V2, tau2, b, nb2, T2, V2t);
    const T *Vuse = V2t ? (const T *)V2t : (const T *)(const void *)V2;
    hipLaunchKernelGGL(k_bt2_apply<T>, dim3(cdiv(ncols, 64)), dim3(256), 0, st, Z, ldz, n, ncols, b, nb2, Vuse,
                       (const T *)T2, goff_dev, nsig);
}

int tn_splits(int K, int tiles)
{
    int S = (int)cdiv(512, tiles > 0 ? tiles : 1);
    int maxS = (int)cdiv(K, 512);
    if (S > maxS) S = maxS;
    if (S > 32) S = 32;
    if (S < 1) S = 1;
    return S;
}

template <typename T>
int launch_gemm_tn_part(const T *A, int lda, const T *B, int ldb, int M, int N, int K, double *Cpart, hipStream_t st)
{
    // returns the number of partial products written
    const int TM = 64, TN = 64;
    unsigned tiles = cdiv(M, TM) * cdiv(N, TN);
    int S = tn_splits(K, (int)tiles);
    int kc = (int)(cdiv(cdiv(K, S), 16) * 16);
    S = (int)cdiv(K, kc);
    dim3 grid(cdiv(M, TM), cdiv(N, TN), S);
    hipLaunchKernelGGL((k_gemm_tn_part<T, 64, 64>), grid, dim3(256), (gemm::smem_bytes<T, 64, 64>()), st, A, lda, B,
                       ldb, M, N, K, kc, Cpart);
    return S;
}

template <typename T>
void launch_gemm_nn(const T *A, int lda, const double *Bpart, int S, int M, int N, int K, T *C, int ldc,
                    double alpha, int beta, hipStream_t st)
{
    if (M <= 0 || N <= 0) return;
    if ((size_t)M * N >= (size_t)8192 * 256) {
        dim3 grid(cdiv(M, 128), cdiv(N, 128));
        hipLaunchKernelGGL((k_gemm_nn<T, 128, 128>), grid, dim3(256), (gemm::smem_bytes<T, 128, 128>()), st, A, lda,
                           Bpart, S, M, N, K, C, ldc, alpha, beta);
    } else {
        dim3 grid(cdiv(M, 64), cdiv(N, 64));
        hipLaunchKernelGGL((k_gemm_nn<T, 64, 64>), grid, dim3(256), (gemm::smem_bytes<T, 64, 64>()), st, A, lda, Bpart,
                           S, M, N, K, C, ldc, alpha, beta);
    }
}

void launch_reduce_left(const double *S0, const double *Cpart, int S, int M, int N, double *out, hipStream_t st)
{
    if (M <= 0 || N <= 0) return;
    size_t shm = sizeof(double) * ((size_t)M + (S0 ? (size_t)M * M : 0));
    hipLaunchKernelGGL(k_reduce_left, dim3(N), dim3(256), shm, st, S0, Cpart, S, M, N, out);
}

template <typename T>
void launch_copy_cols(const T *src, int lds, T *dst, int ldd, int m, int ncol, hipStream_t st)
{
    if (m <= 0 || ncol <= 0) return;
    hipLaunchKernelGGL(k_copy_cols<T>, dim3(cdiv(m, 256) > 8 ? 8 : cdiv(m, 256), ncol), dim3(256), 0, st, src, lds,
                       dst, ldd, m, ncol);
}

template <typename T>
void launch_to_double(const T *src, int lds, double *dst, int ldd, int m, int ncol, hipStream_t st)
{
    if (m <= 0 || ncol <= 0) return;
    hipLaunchKernelGGL(k_to_double<T>, dim3(cdiv(m, 256) > 8 ? 8 : cdiv(m, 256), ncol), dim3(256), 0, st, src, lds,
                       dst, ldd, m);
}

template void launch_dscale<double>(const double *, int, int, int, double *, int, hipStream_t);
template void launch_dscale<float>(const double *, int, int, int, float *, int, hipStream_t);
template void launch_bt2<double>(double *, int, int, int, int, int, const double *, const double *, double *,
                                 double *, const int *, int, int, hipStream_t);
template void launch_bt2<float>(float *, int, int, int, int, int, const double *, const double *, float *, float *,
                                const int *, int, int, hipStream_t);
template int launch_gemm_tn_part<double>(const double *, int, const double *, int, int, int, int, double *,
                                         hipStream_t);
template int launch_gemm_tn_part<float>(const float *, int, const float *, int, int, int, int, double *,
                                        hipStream_t);
template void launch_gemm_nn<double>(const double *, int, const double *, int, int, int, int, double *, int, double,
                                     int, hipStream_t);
template void launch_gemm_nn<float>(const float *, int, const double *, int, int, int, int, float *, int, double,
                                    int, hipStream_t);
template void launch_copy_cols<double>(const double *, int, double *, int, int, int, hipStream_t);
template void launch_copy_cols<float>(const float *, int, float *, int, int, int, hipStream_t);
template void launch_to_double<double>(const double *, int, double *, int, int, int, hipStream_t);
template void launch_to_double<float>(const float *, int, double *, int, int, int, hipStream_t);

}  // namespace skew
