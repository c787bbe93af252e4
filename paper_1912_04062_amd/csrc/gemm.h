// MFMA tile engine for the dense stages (skew SYMM, skew SYR2K, block-
// reflector applications, refinement products).
//
// A workgroup of 256 threads (4 wavefronts of 64, arranged 2 x 2) computes a
// TM x TN tile of  sum_k A(i, k) * B(k, j)  with the 16x16x4 MFMA of the
// element type.  Operands are staged through LDS in K-chunks of 16 in a
// k-major layout  L[k][x]  (x = row of A or column of B), padded by one
// element so that both the transposing and the direct fills are free of bank
// conflicts.  Each operand is described by a fetch functor  f(x, k)  that
// returns the (possibly transformed, e.g. negated or implicitly unit-diagonal)
// element and 0 outside the operand; the template flag KC says whether
// consecutive k are contiguous in memory (then 16 lanes read 16 consecutive
// k of one x), otherwise consecutive x are (64 lanes read 64 consecutive x).
#pragma once
#include "common.h"

namespace gemm {

constexpr int TK = 16;
constexpr int NT = 256;

template <int TX> __device__ constexpr int lds_ld() { return TX + 1; }

// Fill L[kk][x] (kk < 16, x < TX) with f(x0 + x, k0 + kk).
template <typename T, int TX, bool KC, class F>
__device__ __forceinline__ void fill(T *L, const F &f, int x0, int k0)
{
    constexpr int LD = lds_ld<TX>();
    constexpr int PER = TX * TK / NT;
    const int t = threadIdx.x;
    if constexpr (KC) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            int e = t + p * NT;
            int kk = e & (TK - 1), x = e >> 4;
            L[kk * LD + x] = f(x0 + x, k0 + kk);
        }
    } else {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            int e = t + p * NT;
            int x = e % TX, kk = e / TX;
            L[kk * LD + x] = f(x0 + x, k0 + kk);
        }
    }
}

// Accumulators of one wavefront: (TM/32) x (TN/32) tiles of 16 x 16.
template <typename T, int TM, int TN>
struct Acc {
    typename acc4<T>::type v[TM / 32][TN / 32];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int i = 0; i < TM / 32; ++i)
#pragma unroll
            for (int j = 0; j < TN / 32; ++j) v[i][j] = (typename acc4<T>::type)(T(0));
    }
};

// One K-chunk of MFMAs from the LDS tiles As[16][TM+1], Bs[16][TN+1].
template <typename T, int TM, int TN>
__device__ __forceinline__ void mma_chunk(const T *As, const T *Bs, Acc<T, TM, TN> &acc)
{
    constexpr int LDA = lds_ld<TM>(), LDB = lds_ld<TN>();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm0 = (w >> 1) * (TM / 2), wn0 = (w & 1) * (TN / 2);
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int k4 = 0; k4 < TK; k4 += 4) {
        T a[TM / 32], b[TN / 32];
#pragma unroll
        for (int i = 0; i < TM / 32; ++i) a[i] = As[(k4 + lk) * LDA + wm0 + i * 16 + lr];
#pragma unroll
        for (int j = 0; j < TN / 32; ++j) b[j] = Bs[(k4 + lk) * LDB + wn0 + j * 16 + lr];
#pragma unroll
        for (int i = 0; i < TM / 32; ++i)
#pragma unroll
            for (int j = 0; j < TN / 32; ++j) acc.v[i][j] = mfma_16x16x4(a[i], b[j], acc.v[i][j]);
    }
}

// Visit the tile's results: epi(row, col, value) with row/col relative to the
// tile origin.  The tile is staged through LDS (smem, 32 columns at a time) so
// that consecutive threads visit consecutive rows: column-major destinations
// are then written with coalesced accesses.  Must be called by all threads.
template <typename T, int TM, int TN, class E>
__device__ __forceinline__ void epilogue(const Acc<T, TM, TN> &acc, T *smem, const E &epi)
{
    constexpr int LDC = TM + 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm0 = (w >> 1) * (TM / 2), wn0 = (w & 1) * (TN / 2);
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < TN / 32; ++cb) {
        // columns [32 cb, 32 cb + 32): held by the waves with wn0 <= 32 cb < wn0 + TN/2
#pragma unroll
        for (int i = 0; i < TM / 32; ++i)
#pragma unroll
            for (int j = 0; j < TN / 32; ++j) {
                const int c0 = wn0 + j * 16;
                if (c0 >= 32 * cb && c0 < 32 * cb + 32)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        smem[(c0 - 32 * cb + (lane & 15)) * LDC + wm0 + i * 16 + mfma_row<T>(lane, r)] =
                            acc.v[i][j][r];
            }
        __syncthreads();
        for (int e = threadIdx.x; e < TM * 32; e += NT) {
            const int r = e % TM, c = e / TM;
            epi(r, 32 * cb + c, smem[c * LDC + r]);
        }
        __syncthreads();
    }
}

// Full K loop: acc += sum_{k in [kb, ke)} A(m0 + i, k) B(k, n0 + j).
// smem must hold 16*(TM+1) + 16*(TN+1) elements.
template <typename T, int TM, int TN, bool AKC, bool BKC, class FA, class FB>
__device__ __forceinline__ void kloop(const FA &fa, const FB &fb, int m0, int n0, int kb, int ke,
                                      T *smem, Acc<T, TM, TN> &acc)
{
    T *As = smem;
    T *Bs = smem + TK * lds_ld<TM>();
    for (int k0 = kb; k0 < ke; k0 += TK) {
        fill<T, TM, AKC>(As, fa, m0, k0);
        fill<T, TN, BKC>(Bs, fb, n0, k0);
        __syncthreads();
        mma_chunk<T, TM, TN>(As, Bs, acc);
        __syncthreads();
    }
}

template <typename T, int TM, int TN> __host__ __device__ constexpr size_t smem_bytes()
{
    size_t ops = (size_t)(TK * (TM + 1) + TK * (TN + 1));
    size_t epi = (size_t)32 * (TM + 1);
    return sizeof(T) * (ops > epi ? ops : epi);
}

}  // namespace gemm
