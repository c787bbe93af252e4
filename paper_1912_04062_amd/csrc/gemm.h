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

// Register cap for kernels built on the engine: two wavefronts per SIMD, so
// that one wave's LDS and global traffic overlaps the other's MFMAs.
#define GEMM_OCC2 __attribute__((amdgpu_waves_per_eu(2, 8)))

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

// Global -> registers half of a fill (the chunk's elements owned by this
// thread), and registers -> LDS half.  Splitting the two lets the K loop keep
// the next chunk's global loads in flight while the MFMAs of the current one
// run.
template <typename T, int TX> struct Frag {
    T v[TX * TK / NT];
};

template <typename T, int TX, bool KC, class F>
__device__ __forceinline__ void gload(Frag<T, TX> &r, const F &f, int x0, int k0)
{
    constexpr int PER = TX * TK / NT;
    const int t = threadIdx.x;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int e = t + p * NT;
        if constexpr (KC) r.v[p] = f(x0 + (e >> 4), k0 + (e & (TK - 1)));
        else r.v[p] = f(x0 + e % TX, k0 + e / TX);
    }
}

template <typename T, int TX, bool KC>
__device__ __forceinline__ void lstore(T *L, const Frag<T, TX> &r)
{
    constexpr int LD = lds_ld<TX>();
    constexpr int PER = TX * TK / NT;
    const int t = threadIdx.x;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int e = t + p * NT;
        if constexpr (KC) L[(e & (TK - 1)) * LD + (e >> 4)] = r.v[p];
        else L[(e / TX) * LD + e % TX] = r.v[p];
    }
}

// Full K loop: acc += sum_{k in [kb, ke)} A(m0 + i, k) B(k, n0 + j), with the
// next K-chunk prefetched into registers during the current chunk's MFMAs.
// smem must hold 16*(TM+1) + 16*(TN+1) elements.
template <typename T, int TM, int TN, bool AKC, bool BKC, class FA, class FB>
__device__ __forceinline__ void kloop(const FA &fa, const FB &fb, int m0, int n0, int kb, int ke,
                                      T *smem, Acc<T, TM, TN> &acc)
{
    T *As = smem;
    T *Bs = smem + TK * lds_ld<TM>();
    if (kb >= ke) return;
    Frag<T, TM> ra;
    Frag<T, TN> rb;
    gload<T, TM, AKC>(ra, fa, m0, kb);
    gload<T, TN, BKC>(rb, fb, n0, kb);
    for (int k0 = kb; k0 < ke; k0 += TK) {
        lstore<T, TM, AKC>(As, ra);
        lstore<T, TN, BKC>(Bs, rb);
        __syncthreads();
        if (k0 + TK < ke) {
            gload<T, TM, AKC>(ra, fa, m0, k0 + TK);
            gload<T, TN, BKC>(rb, fb, n0, k0 + TK);
        }
        mma_chunk<T, TM, TN>(As, Bs, acc);
        __syncthreads();
    }
}

// The same K loop with the operand chunks alternating between two LDS
// buffers: chunk i + 1 is stored into the other buffer after the MFMAs of
// chunk i, and one workgroup barrier per chunk separates the two (a buffer is
// rewritten only after every wave has passed the barrier that ends the chunk
// that read it).  It needs smem_bytes_db<T, TM, TN>() bytes, which costs
// occupancy where LDS limits it; kernels whose registers already limit them
// to two workgroups per CU gain from the saved barrier.
template <typename T, int TM, int TN, bool AKC, bool BKC, class FA, class FB>
__device__ __forceinline__ void kloop_db(const FA &fa, const FB &fb, int m0, int n0, int kb, int ke,
                                         T *smem, Acc<T, TM, TN> &acc)
{
    constexpr int HALF = TK * lds_ld<TM>() + TK * lds_ld<TN>();
    if (kb >= ke) return;
    Frag<T, TM> ra;
    Frag<T, TN> rb;
    gload<T, TM, AKC>(ra, fa, m0, kb);
    gload<T, TN, BKC>(rb, fb, n0, kb);
    lstore<T, TM, AKC>(smem, ra);
    lstore<T, TN, BKC>(smem + TK * lds_ld<TM>(), rb);
    __syncthreads();
    int q = 0;
    for (int k0 = kb; k0 < ke; k0 += TK) {
        T *As = smem + q * HALF;
        const bool more = k0 + TK < ke;
        if (more) {
            gload<T, TM, AKC>(ra, fa, m0, k0 + TK);
            gload<T, TN, BKC>(rb, fb, n0, k0 + TK);
        }
        mma_chunk<T, TM, TN>(As, As + TK * lds_ld<TM>(), acc);
        if (more) {
            T *An = smem + (q ^ 1) * HALF;
            lstore<T, TM, AKC>(An, ra);
            lstore<T, TN, BKC>(An + TK * lds_ld<TM>(), rb);
        }
        __syncthreads();
        q ^= 1;
    }
}

// K loop whose A operand is a skew matrix read from its strict lower
// triangle: chunks left of the tile's rows come from the lower triangle
// (x-contiguous), chunks right of them from the transposed lower triangle
// (k-contiguous, negated), the diagonal chunks element by element.
template <typename T, int TM, int TN, class FL, class FU, class FM, class FB>
__device__ __forceinline__ void skew_kloop(const FL &f_low, const FU &f_up, const FM &f_mix, const FB &fb, int m0,
                                           int n0, int kb, int ke, T *smem, Acc<T, TM, TN> &acc)
{
    T *As = smem;
    T *Bs = smem + TK * lds_ld<TM>();
    if (kb >= ke) return;
    auto mode_of = [&](int k0) { return (k0 + TK <= m0) ? 0 : ((k0 >= m0 + TM) ? 1 : 2); };
    auto load_a = [&](Frag<T, TM> &r, int mode, int k0) {
        if (mode == 0) gload<T, TM, false>(r, f_low, m0, k0);
        else if (mode == 1) gload<T, TM, true>(r, f_up, m0, k0);
        else gload<T, TM, false>(r, f_mix, m0, k0);
    };
    Frag<T, TM> ra;
    Frag<T, TN> rb;
    int mode = mode_of(kb);
    load_a(ra, mode, kb);
    gload<T, TN, true>(rb, fb, n0, kb);
    for (int k0 = kb; k0 < ke; k0 += TK) {
        if (mode == 1) lstore<T, TM, true>(As, ra);
        else lstore<T, TM, false>(As, ra);
        lstore<T, TN, true>(Bs, rb);
        __syncthreads();
        if (k0 + TK < ke) {
            mode = mode_of(k0 + TK);
            load_a(ra, mode, k0 + TK);
            gload<T, TN, true>(rb, fb, n0, k0 + TK);
        }
        mma_chunk<T, TM, TN>(As, Bs, acc);
        __syncthreads();
    }
}

// Read-modify-write epilogue: ld(row, col) returns the destination's current
// value (0 outside), st(row, col, old, acc) stores the combination.  All loads
// of a column block are issued before its stores.
template <typename T, int TM, int TN, class LD, class ST>
__device__ __forceinline__ void epilogue_rmw(const Acc<T, TM, TN> &acc, T *smem, const LD &ld, const ST &st)
{
    constexpr int LDC = TM + 1;
    constexpr int EPT = TM * 32 / NT;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm0 = (w >> 1) * (TM / 2), wn0 = (w & 1) * (TN / 2);
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < TN / 32; ++cb) {
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
        decltype(ld(0, 0)) old[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = threadIdx.x + q * NT;
            old[q] = ld(e % TM, 32 * cb + e / TM);
        }
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = threadIdx.x + q * NT;
            const int r = e % TM, c = e / TM;
            st(r, 32 * cb + c, old[q], smem[c * LDC + r]);
        }
        __syncthreads();
    }
}

template <typename T, int TM, int TN> __host__ __device__ constexpr size_t smem_bytes()
{
    size_t ops = (size_t)(TK * (TM + 1) + TK * (TN + 1));
    size_t epi = (size_t)32 * (TM + 1);
    return sizeof(T) * (ops > epi ? ops : epi);
}

template <typename T, int TM, int TN> __host__ __device__ constexpr size_t smem_bytes_db()
{
    size_t ops = (size_t)2 * (TK * (TM + 1) + TK * (TN + 1));
    size_t epi = (size_t)32 * (TM + 1);
    return sizeof(T) * (ops > epi ? ops : epi);
}

}  // namespace gemm
