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
#include "small64.h"
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
                                                  int b, int nb2, T *__restrict__ T2, T *__restrict__ V2t,
                                                  int rowmajor)
{
    __shared__ double Vs[64 * 65];       // Vs[r][i]; T after the Gram matrix is formed
    __shared__ double Gm[64 * 65];       // Gram (strict upper; zero elsewhere)
    __shared__ double tv[64], part[4][64];
    double *Tm = Vs;                     // 67 KB of LDS: two workgroups per CU
    const size_t g = blockIdx.x;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const double *Vg = V2 + g * (size_t)b * nb2;
    for (int e = tid; e < b * nb2; e += 256) {
        int r = e % b, i = e / b;
        Vs[r * 65 + i] = Vg[e];
        if (V2t) V2t[g * (size_t)b * nb2 + e] = (T)Vg[e];
    }
    if (tid < 64) tv[tid] = (tid < nb2) ? tau2[g * nb2 + tid] : 0.0;
    __syncthreads();
    // Gram: v_i . v_j (i < j), overlap rows j..i+b-1 (absolute), r = row - i
    for (int e = tid; e < 64 * 64; e += 256) {
        int i = e % 64, j = e / 64;
        double s = 0.0;
        if (i < j && j < nb2) {
            int d = j - i;
            for (int r = d; r < b; ++r) s += Vs[r * 65 + i] * Vs[(r - d) * 65 + j];
        }
        Gm[i * 65 + j] = s;
    }
    __syncthreads();
    for (int e = tid; e < 64 * 65; e += 256) Tm[e] = 0.0;
    __syncthreads();
    // T[i][j] = -tau_j sum_{i <= u < j} T[i][u] G[u][j], T[j][j] = tau_j.  T
    // starts at zero and column u is written at step u, so the sum runs over
    // all u (G is zero on and below the diagonal); the four wavefronts take
    // a quarter of the u each.
    for (int j = 0; j < nb2; ++j) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int q = 0; q < 16; q += 2) {
            const int u = ty + 4 * q;
            s0 = fma(Tm[tx * 65 + u], Gm[u * 65 + j], s0);
            s1 = fma(Tm[tx * 65 + u + 4], Gm[(u + 4) * 65 + j], s1);
        }
        part[ty][tx] = s0 + s1;
        __syncthreads();
        if (ty == 0 && tx <= j)
            Tm[tx * 65 + j] = (tx == j) ? tv[j] : -tv[j] * (part[0][tx] + part[1][tx] + part[2][tx] + part[3][tx]);
        __syncthreads();
    }
    T *To = T2 + g * (size_t)nb2 * nb2;
    for (int e = tid; e < nb2 * nb2; e += 256) {
        int i = e % nb2, j = e / nb2;
        To[e] = rowmajor ? (T)Tm[j * 65 + i] : (T)Tm[i * 65 + j];   // row- or column-major
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

// ---------------------------------------------------------------------------
// Stage-2 application, FP64, b = nb2 = 64: register-resident sliding window.
//
// Row block x = rows [1 + 64x, 1 + 64(x+1)).  Group (s, k) (sweep-block s,
// step k) acts on row blocks t = s + k and t + 1.  Required order: (s, k)
// before (s, k+1), and (s+1, k') before (s, k) when they share rows.  With two
// sweep-blocks s_hi, s_hi - 1 per pass, the schedule tau(s, k) = k + (s_hi - s)
// satisfies both, and the groups of one tau are row-disjoint; at time tau the
// active row blocks are s_hi + tau - 2 .. s_hi + tau + 1, a window of 4 blocks
// that slides down by one block per tau.  Z is therefore read and written once
// per pass of two sweep-blocks.
//
// A workgroup owns 64 columns; each wavefront keeps its 16-column strip of the
// 256-row window in registers, in the FP64 MFMA result layout (row
// 16q + l/16 + 4r of tile q, column l%16), which is also the B-operand layout
// of k-step 4r of the tile, so Z, W1 = V^T Z and W2 = T W1 never leave
// registers.  The window's slots are kept in positional order (slot j = row
// block s_hi + tau - 2 + j) by rotating registers when it slides, so group
// (s_hi, tau) always uses slots 2, 3 and group (s_hi - 1, tau - 1) slots 0, 1.
// Each wavefront owns its columns for the whole kernel, so Z moves directly
// between global memory and registers (the block entering the window is
// loaded one step ahead).  V and T (64 x 64 each, compact as in memory) are
// double-buffered in LDS and filled by 16-byte global-to-LDS loads one group
// ahead; one barrier per group.
namespace bt2p {

constexpr int B = 64;
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void gbl_void;

struct Win {
    d4 z[4][4];      // [slot][row tile]
};

// Group cursor: pass sh (sweep-blocks sh and sh - 1), time tau, w = 0 for
// group (sh, tau) and w = 1 for group (sh - 1, tau - 1).  sh < 0: done.
struct Cur {
    int sh, tau, w;
};

__device__ __forceinline__ int ngr(const int *goff, int sg) { return goff[sg + 1] - goff[sg]; }

__device__ __forceinline__ int taumax(const int *goff, int sh)
{
    int t = ngr(goff, sh) - 1;
    if (sh >= 1) t = max(t, ngr(goff, sh - 1));
    return t;
}

__device__ __forceinline__ bool cvalid(const Cur &c, const int *goff)
{
    if (c.w == 0) return c.tau < ngr(goff, c.sh);
    return c.sh >= 1 && c.tau >= 1 && c.tau - 1 < ngr(goff, c.sh - 1);
}

__device__ __forceinline__ void advance(Cur &c, const int *goff)
{
    while (c.sh >= 0) {
        if (c.w == 0) {
            c.w = 1;
        } else {
            c.w = 0;
            if (++c.tau > taumax(goff, c.sh)) {
                c.sh -= 2;
                c.tau = 0;
                if (c.sh < 0) return;
            }
        }
        if (cvalid(c, goff)) return;
    }
}

__device__ __forceinline__ size_t gid(const Cur &c, const int *goff)
{
    return (c.w == 0) ? (size_t)goff[c.sh] + c.tau : (size_t)goff[c.sh - 1] + c.tau - 1;
}

// LDS image of a group: V (b x nb2 column-major) and T (row-major), each
// moved as 32 chunks of 1 KB (two columns of V, two rows of T) that are
// padded apart (PV, PT doubles) so that the MFMA operand reads spread over
// the banks.  V[d][i] is at chunk i/2, offset 64 (i%2) + d; T[i][u] at chunk
// i/2, offset 64 (i%2) + u.
constexpr int PV = 6, PT = 4;
constexpr int CV = 128 + PV, CT = 128 + PT;     // chunk strides
constexpr int BUF = 32 * CV + 32 * CT;          // one buffer (V then T)

// Part i (0..7) of the move of group g's V then T into Vl / Tl: wave w moves
// chunks 16w + 2i and 16w + 2i + 1 (0..31 of V, then 0..31 of T), 16 bytes
// per lane.  The eight parts are issued between the MFMAs of the preceding
// group's first phase.
__device__ __forceinline__ void prefetch_part(const double *__restrict__ V2, const double *__restrict__ T2, size_t g,
                                              double *Vl, double *Tl, int i)
{
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double *src = (wv < 2) ? V2 + g * (B * B) : T2 + g * (B * B);
    double *dst = (wv < 2) ? Vl : Tl;
    const int cs = (wv < 2) ? CV : CT;
    const int c0 = (wv & 1) * 16;
#pragma unroll
    for (int j = 2 * i; j < 2 * i + 2; ++j)
        __builtin_amdgcn_global_load_lds((gbl_void *)(src + (size_t)(c0 + j) * 128 + 2 * lane),
                                         (lds_void *)(dst + (c0 + j) * cs), 16, 0, 0);
}

__device__ __forceinline__ void prefetch(const double *__restrict__ V2, const double *__restrict__ T2, size_t g,
                                         double *Vl, double *Tl)
{
#pragma unroll
    for (int i = 0; i < 8; ++i) prefetch_part(V2, T2, g, Vl, Tl, i);
}

__device__ __forceinline__ bool blk_ok(int x, int n) { return x >= 0 && 1 + 64 * x < n; }

// Row block x (64 rows from 1 + 64x) of this wavefront's 16 columns, in the
// MFMA result layout.  Every load is issued unconditionally, clamped to a
// valid address, and nothing waits for it until the block is used: rows past
// n and columns past ncols hold copies of valid (finite) entries, which only
// ever meet zero reflector entries and are never stored.
__device__ __forceinline__ void load_block(d4 (&zb)[4], const double *__restrict__ Z, int ldz, int n, int col0,
                                           int ncl, int x)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (!blk_ok(x, n)) {
#pragma unroll
        for (int q = 0; q < 4; ++q) zb[q] = (d4){0.0, 0.0, 0.0, 0.0};
        return;
    }
    const int c = 16 * wv + (lane & 15);
    const int r0 = 1 + 64 * x;
    const double *zc = Z + (size_t)(col0 + (c < ncl ? c : 0)) * ldz;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int r = r0 + 16 * q + (lane >> 4) + 4 * rr;
            zb[q][rr] = zc[r < n ? r : n - 1];
        }
}

__device__ __forceinline__ void store_block(const d4 (&zb)[4], double *__restrict__ Z, int ldz, int n, int col0,
                                            int ncl, int x)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = 16 * wv + (lane & 15);
    if (!blk_ok(x, n) || c >= ncl) return;
    const int r0 = 1 + 64 * x;
    double *zc = Z + (size_t)(col0 + c) * ldz;
    if (r0 + 63 < n) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) zc[r0 + 16 * q + (lane >> 4) + 4 * rr] = zb[q][rr];
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int r = r0 + 16 * q + (lane >> 4) + 4 * rr;
                if (r < n) zc[r] = zb[q][rr];
            }
    }
}

// Z[slots S0, S1] <- (I - Vp T Vp^T) Z[slots S0, S1]; Vp is the 128 x 64
// parallelogram Vp[r][i] = V[r - i][i] (0 <= r - i < 64), V and T in the
// padded LDS image above.
//
// Every LDS operand address is a per-lane base plus a compile-time offset,
// and the parallelogram test is a compare of a per-lane constant with a
// compile-time bound; the per-lane constants are re-derived at each call so
// that the compiler does not keep hundreds of hoisted addresses and masks
// alive across the group loop.  Each phase runs its k-steps outermost so that
// MFMAs of independent output tiles follow each other, and loads the LDS
// operands of a chunk of k-steps before the chunk's MFMAs.
// hook1(i) runs before the i-th chunk of the first phase's k-steps (i = 0..7),
// pinned there so that its memory instructions issue between MFMAs.
template <int S0, int S1, class H1>
__device__ __forceinline__ void apply(Win &w, const double *Vl, const double *Tl, const H1 &hook1)
{
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const int lr = lane & 15, lk = lane >> 4;
    // W1 = Vp^T Zg: element (i = 16mt + lr, r = 4ks + lk) at chunk 8mt + lr/2, offset
    // 64 (lr % 2) + lk - lr + 4ks - 16mt; inside when 0 <= lk - lr + 4ks - 16mt < 64
    const double *vb1 = Vl + (lr >> 1) * CV + (lr & 1) * 64 + lk - lr;
    const int dw = lk - lr;
    __builtin_assume(dw >= -15 && dw <= 3);     // the tiles whose k-steps lie inside need no test
    d4 w1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) w1[mt] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 32; kc += 4) {
        __builtin_amdgcn_sched_barrier(0);
        hook1(kc >> 2);
        __builtin_amdgcn_sched_barrier(0);
        double a[4][4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int ks = kc + kk;
                if (ks >= 4 * mt && ks < 4 * mt + 20) {
                    const double x = vb1[8 * mt * CV + 4 * ks - 16 * mt];
                    const int d = dw + 4 * ks - 16 * mt;
                    a[kk][mt] = ((unsigned)d < (unsigned)B) ? x : 0.0;
                } else {
                    a[kk][mt] = 0.0;
                }
            }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int ks = kc + kk;
            const double bz = (ks < 16) ? w.z[S0][ks >> 2][ks & 3] : w.z[S1][(ks >> 2) & 3][ks & 3];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                if (ks >= 4 * mt && ks < 4 * mt + 20) w1[mt] = mfma_16x16x4(a[kk][mt], bz, w1[mt]);
        }
    }
    // W2 = T W1 (T upper triangular): T[16mt + lr][4ks + lk] at chunk 8mt + lr/2,
    // offset 64 (lr % 2) + lk + 4ks
    const double *tb = Tl + (lr >> 1) * CT + (lr & 1) * 64 + lk;
    d4 w2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) w2[mt] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 16; kc += 4) {
        double a[4][4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int ks = kc + kk;
                a[kk][mt] = (ks >= 4 * mt) ? tb[8 * mt * CT + 4 * ks] : 0.0;
            }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int ks = kc + kk;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                if (ks >= 4 * mt) w2[mt] = mfma_16x16x4(a[kk][mt], w1[ks >> 2][ks & 3], w2[mt]);
        }
    }
    // Zg -= Vp W2: element (r = 16rt + lr, i = 4ks + lk) at chunk 2ks + lk/2, offset
    // 64 (lk % 2) + lr - lk + 16rt - 4ks; inside when 0 <= lr - lk + 16rt - 4ks < 64
    const double *vb3 = Vl + (lk >> 1) * CV + (lk & 1) * 64 + lr - lk;
    const int dz = lr - lk;
    __builtin_assume(dz >= -3 && dz <= 15);
#pragma unroll
    for (int kc = 0; kc < 16; kc += 2) {
        double a[2][8];
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
            for (int rt = 0; rt < 8; ++rt) {
                const int ks = kc + kk, i4 = 4 * ks;
                if (!(i4 + 3 < 16 * rt - B + 1 || i4 >= 16 * rt + 16)) {
                    const double x = vb3[2 * ks * CV + 16 * rt - 4 * ks];
                    const int d = dz + 16 * rt - 4 * ks;
                    a[kk][rt] = ((unsigned)d < (unsigned)B) ? -x : 0.0;
                } else {
                    a[kk][rt] = 0.0;
                }
            }
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int ks = kc + kk, i4 = 4 * ks;
            const double bw = w2[ks >> 2][ks & 3];
#pragma unroll
            for (int rt = 0; rt < 8; ++rt) {
                if (i4 + 3 < 16 * rt - B + 1 || i4 >= 16 * rt + 16) continue;
                if (rt < 4) w.z[S0][rt] = mfma_16x16x4(a[kk][rt], bw, w.z[S0][rt]);
                else w.z[S1][rt - 4] = mfma_16x16x4(a[kk][rt], bw, w.z[S1][rt - 4]);
            }
        }
    }
}

}  // namespace bt2p

__global__ __launch_bounds__(256) void k_bt2_win(double *__restrict__ Z, int ldz, int n, int ncols,
                                                const double *__restrict__ V2, const double *__restrict__ T2,
                                                const int *__restrict__ goff, int nsig)
{
    using namespace bt2p;
    extern __shared__ double lds[];
    // buffer q: V image, then T image
    auto Vl = [&](int q) -> double * { return lds + q * BUF; };
    auto Tl = [&](int q) -> double * { return lds + q * BUF + 32 * CV; };
    const int col0 = blockIdx.x * 64;
    const int ncl = min(64, ncols - col0);
    if (nsig <= 0) return;
    Cur c{nsig - 1, 0, 0};
    if (!cvalid(c, goff)) advance(c, goff);
    if (c.sh < 0) return;
    prefetch(V2, T2, gid(c, goff), Vl(0), Tl(0));
    Cur nx = c;
    advance(nx, goff);
    Win w;
    d4 nxt[4];                                     // the block that enters the window next
    int cur_sh = c.sh, cur_tau = 0, buf = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) load_block(w.z[j], Z, ldz, n, col0, ncl, cur_sh - 2 + j);
    load_block(nxt, Z, ldz, n, col0, ncl, cur_sh + 2);
    wait_vmem();
    __syncthreads();
    while (c.sh >= 0) {
        if (c.sh != cur_sh) {                      // next pass: flush the window, load the new one
#pragma unroll
            for (int j = 0; j < 4; ++j) store_block(w.z[j], Z, ldz, n, col0, ncl, cur_sh + cur_tau - 2 + j);
            cur_sh = c.sh;
            cur_tau = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) load_block(w.z[j], Z, ldz, n, col0, ncl, cur_sh - 2 + j);
            load_block(nxt, Z, ldz, n, col0, ncl, cur_sh + 2);
        }
        while (cur_tau < c.tau) {                  // slide down one block
            store_block(w.z[0], Z, ldz, n, col0, ncl, cur_sh + cur_tau - 2);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                w.z[0][q] = w.z[1][q];
                w.z[1][q] = w.z[2][q];
                w.z[2][q] = w.z[3][q];
                w.z[3][q] = nxt[q];
            }
            ++cur_tau;
            load_block(nxt, Z, ldz, n, col0, ncl, cur_sh + cur_tau + 2);
        }
        // the next group's V and T move into the other buffer during this
        // group's first phase (the last group re-fetches itself: harmless)
        const size_t gn = gid(nx.sh >= 0 ? nx : c, goff);
        double *vn = Vl(buf ^ 1), *tn = Tl(buf ^ 1);
        auto pf = [&](int i) { prefetch_part(V2, T2, gn, vn, tn, i); };
        if (c.w == 0) apply<2, 3>(w, Vl(buf), Tl(buf), pf);
        else apply<0, 1>(w, Vl(buf), Tl(buf), pf);
        wait_vmem();
        __syncthreads();
        buf ^= 1;
        c = nx;
        advance(nx, goff);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) store_block(w.z[j], Z, ldz, n, col0, ncl, cur_sh + cur_tau - 2 + j);
}

// ---------------------------------------------------------------------------
// Stage-1 back-transformation of one compact-WY block of KK reflectors (one
// panel, or two consecutive panels merged: V = [V_j, V_{j+1} shifted down by
// b rows], T = [[T_j, T12], [0, T_{j+1}]]):  Z[r0:, :] -= V (T (V^T Z[r0:, :])).
// Three launches with many workgroups each (two per CU: the register budget
// is capped so that two waves share every SIMD):
//   k_bt1_w   Wp[s] = V^T Z over the s-th chunk of rows (split K)
//   k_bt1_t   W2 = T * sum_s Wp[s]
//   k_bt1_z   Z -= V W2 on 64 x 128 tiles (taller tiles measured slower).

// Element (row, k) of the (merged) V of a block: column k < b1 comes from V1
// (m rows), k >= b1 from V2 (m2 rows, starting b1 rows lower); 0 elsewhere.
template <typename T>
struct MergedV {
    const T *V1;
    const T *V2;
    int b1, m, m2;
    __device__ __forceinline__ T operator()(int row, int k) const
    {
        if (row >= m) return T(0);
        if (k < b1) return V1[(size_t)k * m + row];
        if (!V2) return T(0);
        const int r2 = row - b1;
        return (r2 >= 0 && r2 < m2) ? V2[(size_t)(k - b1) * m2 + r2] : T(0);
    }
};

template <typename T, int KK>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_bt1_w(
    const T *__restrict__ Z, int ldz, int ncols, MergedV<T> V, int kchunk, double *__restrict__ Wp)
{
    constexpr int TN = 128;
    extern __shared__ char smraw[];
    T *smem = (T *)smraw;
    const int n0 = blockIdx.x * TN, s = blockIdx.y;
    const int kb = s * kchunk, ke = min(V.m, kb + kchunk);
    auto fa = [=](int l, int row) -> T { return (l < KK && row < ke) ? V(row, l) : T(0); };
    // fetch functors take absolute indices (the engine adds the tile origin)
    auto fb = [=](int j, int row) -> T { return (row < ke && j < ncols) ? Z[(size_t)j * ldz + row] : T(0); };
    gemm::Acc<T, KK, TN> acc;
    acc.zero();
    gemm::kloop_db<T, KK, TN, true, true>(fa, fb, 0, n0, kb, ke, smem, acc);
    double *W = Wp + (size_t)s * KK * ncols;
    gemm::epilogue<T, KK, TN>(acc, smem, [=](int i, int j, T v) {
        if (n0 + j < ncols) W[(size_t)(n0 + j) * KK + i] = (double)v;
    });
}

template <typename T, int KK>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_bt1_t(
    const double *__restrict__ Tm, const double *__restrict__ Wp, int S, int ncols, T *__restrict__ W2)
{
    constexpr int TN = 64;
    extern __shared__ char smraw[];
    T *smem = (T *)smraw;
    const int n0 = blockIdx.x * TN;
    const size_t pst = (size_t)KK * ncols;
    auto fa = [=](int i, int k) -> T { return (T)Tm[(size_t)k * KK + i]; };
    auto fb = [=](int j, int k) -> T {
        if (j >= ncols) return T(0);
        double sum = 0.0;
        for (int p = 0; p < S; ++p) sum += Wp[p * pst + (size_t)j * KK + k];
        return (T)sum;
    };
    gemm::Acc<T, KK, TN> acc;
    acc.zero();
    gemm::kloop<T, KK, TN, false, true>(fa, fb, 0, n0, 0, KK, smem, acc);
    gemm::epilogue<T, KK, TN>(acc, smem, [=](int i, int j, T v) {
        if (n0 + j < ncols) W2[(size_t)(n0 + j) * KK + i] = v;
    });
}

template <typename T, int KK>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_bt1_z(
    T *__restrict__ Z, int ldz, int ncols, MergedV<T> V, const T *__restrict__ W2)
{
    constexpr int TM = 64, TN = 128;
    extern __shared__ char smraw[];
    T *smem = (T *)smraw;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    auto fa = [=](int row, int k) -> T { return V(row, k); };
    auto fb = [=](int j, int k) -> T { return (j < ncols) ? W2[(size_t)j * KK + k] : T(0); };
    gemm::Acc<T, TM, TN> acc;
    acc.zero();
    gemm::kloop<T, TM, TN, false, true>(fa, fb, m0, n0, 0, KK, smem, acc);
    gemm::epilogue_rmw<T, TM, TN>(
        acc, smem,
        // unconditional load at a clamped address: values outside are never
        // stored, and a test here would become a branch around every load
        [=](int i, int j) -> T { return Z[(size_t)min(n0 + j, ncols - 1) * ldz + min(m0 + i, V.m - 1)]; },
        [=](int i, int j, T old, T v) {
            const int gi = m0 + i, gj = n0 + j;
            if (gi < V.m && gj < ncols) Z[(size_t)gj * ldz + gi] = old - v;
        });
}

// Merged T of two consecutive panels: Tm = [[T1, -T1 G T2], [0, T2]] with
// G = sum of the partial products V1(b:, :)^T V2 (b x b each, b <= 64).
__global__ __launch_bounds__(256) void k_merge_t(const double *__restrict__ T1, const double *__restrict__ T2,
                                                 const double *__restrict__ Gp, int S, int b,
                                                 double *__restrict__ Tm)
{
    __shared__ double G[64 * 65], M1[64 * 65], A1[64 * 65], A2[64 * 65];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6, K = 2 * b;
    auto off = [=](int i, int j) -> int { return (i < b && j < b) ? j * b + i : -1; };
    {
        double acc[16], t1[16], t2[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int o = off(tx, ty + 4 * q);
            const bool up = o >= 0 && tx <= ty + 4 * q;       // T1, T2 upper, zero elsewhere
            t1[q] = up ? T1[o] : 0.0;
            t2[q] = up ? T2[o] : 0.0;
        }
        sum_partials_2d(Gp, S, (size_t)b * b, off, acc);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = ty + 4 * q;
            G[tx * 65 + j] = acc[q];                 // G[u][v]
            A1[tx * 65 + j] = t1[q];                 // T1[i][u]
            A2[tx * 65 + j] = t2[q];                 // T2[w][v]
        }
    }
    __syncthreads();
    mm64<false>(G, A2, M1);                          // M1 = G T2
    __syncthreads();
    mm64<false>(A1, M1, G);                          // T1 M1 (into G); T12 = -T1 M1
    __syncthreads();
    for (int j = ty; j < K; j += 4)
        for (int i = tx; i < K; i += 64) {
            double val = 0.0;
            if (i < b && j < b) val = A1[i * 65 + j];
            else if (i >= b && j >= b) val = A2[(i - b) * 65 + (j - b)];
            else if (i < b) val = -G[i * 65 + (j - b)];
            Tm[(size_t)j * K + i] = val;
        }
}

// Cpart[s] = A[kb:ke, 0:M]^T B[kb:ke, 0:N]   (A: K x M, B: K x N, column-major)
// TL: the element type in memory (float operands can be multiplied and
// summed in FP64 with T = double: the FP32 form's panel Gram matrices)
template <typename T, int TM, int TN, typename TL = T>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_gemm_tn_part(const TL *__restrict__ A, int lda,
                                                      const TL *__restrict__ B, int ldb, int M, int N, int K,
                                                      int kchunk, double *__restrict__ Cpart)
{
    extern __shared__ char smraw[];
    T *smem = (T *)smraw;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN, s = blockIdx.z;
    const int kb = s * kchunk, ke = min(K, kb + kchunk);
    auto fa = [=](int i, int k) -> T { return (i < M && k < ke) ? (T)A[(size_t)i * lda + k] : T(0); };
    auto fb = [=](int j, int k) -> T { return (j < N && k < ke) ? (T)B[(size_t)j * ldb + k] : T(0); };
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
__global__ __launch_bounds__(256) GEMM_OCC2 void k_gemm_nn(const T *__restrict__ A, int lda, const double *__restrict__ Bpart,
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
    if (beta) {
        gemm::epilogue_rmw<T, TM, TN>(
            acc, smem,
            // unconditional load at a clamped address (see k_bt1_z)
            [=](int i, int j) -> T { return C[(size_t)min(n0 + j, N - 1) * ldc + min(m0 + i, M - 1)]; },
            [=](int i, int j, T old, T v) {
                const int gi = m0 + i, gj = n0 + j;
                if (gi < M && gj < N) C[(size_t)gj * ldc + gi] = (T)((double)old + alpha * (double)v);
            });
    } else {
        // C's old value is not needed: no read round trip
        gemm::epilogue<T, TM, TN>(acc, smem, [=](int i, int j, T v) {
            const int gi = m0 + i, gj = n0 + j;
            if (gi < M && gj < N) C[(size_t)gj * ldc + gi] = (T)(alpha * (double)v);
        });
    }
}

// out = S0 * sum_s Cpart[s]  (S0: M x M column-major, M <= 64) or, with
// S0 == nullptr, out = sum_s Cpart[s].  One workgroup per column.
__global__ __launch_bounds__(256) void k_reduce_left(const double *__restrict__ S0, const double *__restrict__ Cpart,
                                                     int S, int M, int N, double *__restrict__ out)
{
    extern __shared__ double cs[];        // M (+ M*M when S0)
    const size_t pst = (size_t)M * N;
    const int j = blockIdx.x;
    for (int u0 = 0; u0 < M; u0 += 1024) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int p = 0; p < S; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int u = u0 + threadIdx.x + 256 * q;
                if (u < M) acc[q] += Cpart[p * pst + (size_t)j * M + u];
            }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int u = u0 + threadIdx.x + 256 * q;
            if (u < M) {
                if (S0) cs[u] = acc[q];
                else out[(size_t)j * M + u] = acc[q];   // plain sum: no LDS needed (any M)
            }
        }
    }
    if (!S0) return;
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

__global__ void k_to_float(const double *__restrict__ src, int lds, float *__restrict__ dst, int ldd, int m)
{
    const int c = blockIdx.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256)
        dst[(size_t)c * ldd + i] = (float)src[(size_t)c * lds + i];
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
                T *V2t, const int *goff_dev, int nsig, int ngroups, int phases, hipStream_t st)
{
    if (ngroups <= 0 || ncols <= 0) return;
    const bool win = sizeof(T) == sizeof(double) && b == 64 && nb2 == 64;   // window kernel: T row-major
    if (phases & 1)
        hipLaunchKernelGGL(k_bt2_tfac<T>, dim3(ngroups), dim3(256), 0, st, V2, tau2, b, nb2, T2, V2t, win ? 1 : 0);
    if (!(phases & 2)) return;
    const T *Vuse = V2t ? (const T *)V2t : (const T *)(const void *)V2;
    if (win) {
        const size_t shm = sizeof(double) * 2 * bt2p::BUF;
        static bool attr = false;
        if (!attr) {
            (void)hipFuncSetAttribute((const void *)k_bt2_win, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
            attr = true;
        }
        hipLaunchKernelGGL(k_bt2_win, dim3(cdiv(ncols, 64)), dim3(256), shm, st, (double *)(void *)Z, ldz, n, ncols,
                           V2, (const double *)(const void *)T2, goff_dev, nsig);
    } else {
        hipLaunchKernelGGL(k_bt2_apply<T>, dim3(cdiv(ncols, 64)), dim3(256), 0, st, Z, ldz, n, ncols, b, nb2, Vuse,
                           (const T *)T2, goff_dev, nsig);
    }
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

int launch_gemm_tn_part_f64(const float *A, int lda, const float *B, int ldb, int M, int N, int K, double *Cpart,
                            hipStream_t st, int S_req)
{
    const int TM = 64, TN = 64;
    unsigned tiles = cdiv(M, TM) * cdiv(N, TN);
    int S = S_req > 0 ? S_req : tn_splits(K, (int)tiles);
    int kc = (int)(cdiv(cdiv(K, S), 16) * 16);
    S = (int)cdiv(K, kc);
    dim3 grid(cdiv(M, TM), cdiv(N, TN), S);
    hipLaunchKernelGGL((k_gemm_tn_part<double, 64, 64, float>), grid, dim3(256), (gemm::smem_bytes<double, 64, 64>()),
                       st, A, lda, B, ldb, M, N, K, kc, Cpart);
    return S;
}

template <typename T>
int launch_gemm_tn_part(const T *A, int lda, const T *B, int ldb, int M, int N, int K, double *Cpart, hipStream_t st,
                        int S_req)
{
    // returns the number of partial products written
    const int TM = 64, TN = 64;
    unsigned tiles = cdiv(M, TM) * cdiv(N, TN);
    int S = S_req > 0 ? S_req : tn_splits(K, (int)tiles);
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
    } else if ((size_t)cdiv(M, 64) * cdiv(N, 64) >= 512) {
        dim3 grid(cdiv(M, 64), cdiv(N, 64));
        hipLaunchKernelGGL((k_gemm_nn<T, 64, 64>), grid, dim3(256), (gemm::smem_bytes<T, 64, 64>()), st, A, lda, Bpart,
                           S, M, N, K, C, ldc, alpha, beta);
    } else {
        // thin products (n x 64 blocks): 32-row tiles, two workgroups per CU
        dim3 grid(cdiv(M, 32), cdiv(N, 64));
        hipLaunchKernelGGL((k_gemm_nn<T, 32, 64>), grid, dim3(256), (gemm::smem_bytes<T, 32, 64>()), st, A, lda, Bpart,
                           S, M, N, K, C, ldc, alpha, beta);
    }
}

void launch_reduce_left(const double *S0, const double *Cpart, int S, int M, int N, double *out, hipStream_t st)
{
    if (M <= 0 || N <= 0) return;
    size_t shm = S0 ? sizeof(double) * ((size_t)M + (size_t)M * M) : 0;
    hipLaunchKernelGGL(k_reduce_left, dim3(N), dim3(256), shm, st, S0, Cpart, S, M, N, out);
}

// Whole-spectrum output: columns c < off get the conjugate of column n-1-c
// (the eigenvector of -lambda is conj(z) of +lambda), lambda[c] = -lambda[n-1-c].
__global__ void k_mirror(double *__restrict__ Zr, int ldr, double *__restrict__ Zi, int ldi,
                         double *__restrict__ lam, int n, int off)
{
    const int c = blockIdx.y, src = n - 1 - c;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        Zr[(size_t)c * ldr + i] = Zr[(size_t)src * ldr + i];
        Zi[(size_t)c * ldi + i] = -Zi[(size_t)src * ldi + i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) lam[c] = -lam[src];
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

void launch_to_float(const double *src, int lds, float *dst, int ldd, int m, int ncol, hipStream_t st)
{
    if (m <= 0 || ncol <= 0) return;
    hipLaunchKernelGGL(k_to_float, dim3(cdiv(m, 256) > 8 ? 8 : cdiv(m, 256), ncol), dim3(256), 0, st, src, lds, dst,
                       ldd, m);
}

// Split of the row range of k_bt1_w: about two workgroups per CU, chunks of
// at least 512 rows.
int bt1_splits(int m, int ncols)
{
    const int tiles = (int)cdiv(ncols, 128);
    int S = (int)cdiv(512, tiles > 0 ? tiles : 1);
    const int maxS = (int)cdiv(m, 512);
    if (S > maxS) S = maxS;
    if (S > bt1_max_splits()) S = bt1_max_splits();
    if (S < 1) S = 1;
    return S;
}

template <typename T, int KK>
static void bt1_block(T *Z, int ldz, int m, int ncols, MergedV<T> V, const double *Tm, double *Wp, T *W2,
                      hipStream_t st)
{
    int S = bt1_splits(m, ncols);
    const int kc = (int)(cdiv(cdiv(m, S), 16) * 16);
    S = (int)cdiv(m, kc);
    constexpr size_t shw = gemm::smem_bytes_db<T, KK, 128>();
    if constexpr (shw > 65536) {   // dynamic LDS above 64 KB needs the kernel attribute
        static bool attr = false;
        if (!attr) {
            (void)hipFuncSetAttribute((const void *)k_bt1_w<T, KK>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shw);
            attr = true;
        }
    }
    hipLaunchKernelGGL((k_bt1_w<T, KK>), dim3(cdiv(ncols, 128), S), dim3(256), shw, st,
                       (const T *)Z, ldz, ncols, V, kc, Wp);
    hipLaunchKernelGGL((k_bt1_t<T, KK>), dim3(cdiv(ncols, 64)), dim3(256), (gemm::smem_bytes<T, KK, 64>()), st, Tm,
                       (const double *)Wp, S, ncols, W2);
    hipLaunchKernelGGL((k_bt1_z<T, KK>), dim3(cdiv(m, 64), cdiv(ncols, 128)), dim3(256),
                       (gemm::smem_bytes<T, 64, 128>()), st, Z, ldz, ncols, V, (const T *)W2);
}

template <typename T>
void launch_bt1_block(T *Z, int ldz, int r0, int m, int ncols, const T *V1, int b1, const T *V2, int m2,
                      const double *Tm, int KK, double *Wp, T *W2, hipStream_t st)
{
    if (m <= 0 || ncols <= 0) return;
    MergedV<T> V{V1, V2, b1, m, m2};
    if (KK == 128) bt1_block<T, 128>(Z + r0, ldz, m, ncols, V, Tm, Wp, W2, st);
    else if (KK == 64) bt1_block<T, 64>(Z + r0, ldz, m, ncols, V, Tm, Wp, W2, st);
    else bt1_block<T, 32>(Z + r0, ldz, m, ncols, V, Tm, Wp, W2, st);
}

void launch_merge_t(const double *T1, const double *T2, const double *Gp, int S, int b, double *Tm, hipStream_t st)
{
    hipLaunchKernelGGL(k_merge_t, dim3(1), dim3(256), 0, st, T1, T2, Gp, S, b, Tm);
}

template void launch_bt1_block<double>(double *, int, int, int, int, const double *, int, const double *, int,
                                       const double *, int, double *, double *, hipStream_t);
template void launch_bt1_block<float>(float *, int, int, int, int, const float *, int, const float *, int,
                                      const double *, int, double *, float *, hipStream_t);
template void launch_dscale<double>(const double *, int, int, int, double *, int, hipStream_t);
template void launch_dscale<float>(const double *, int, int, int, float *, int, hipStream_t);
template void launch_bt2<double>(double *, int, int, int, int, int, const double *, const double *, double *,
                                 double *, const int *, int, int, int, hipStream_t);
template void launch_bt2<float>(float *, int, int, int, int, int, const double *, const double *, float *, float *,
                                const int *, int, int, int, hipStream_t);
template int launch_gemm_tn_part<double>(const double *, int, const double *, int, int, int, int, double *,
                                         hipStream_t, int);
template int launch_gemm_tn_part<float>(const float *, int, const float *, int, int, int, int, double *,
                                        hipStream_t, int);
template void launch_gemm_nn<double>(const double *, int, const double *, int, int, int, int, double *, int, double,
                                     int, hipStream_t);
template void launch_gemm_nn<float>(const float *, int, const double *, int, int, int, int, float *, int, double,
                                    int, hipStream_t);
void launch_mirror(double *Zr, int ldr, double *Zi, int ldi, double *lam, int n, int off, hipStream_t st)
{
    if (off <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_mirror, dim3(cdiv(n, 256) > 8 ? 8 : cdiv(n, 256), off), dim3(256), 0, st, Zr, ldr, Zi, ldi,
                       lam, n, off);
}

template void launch_copy_cols<double>(const double *, int, double *, int, int, int, hipStream_t);
template void launch_copy_cols<float>(const float *, int, float *, int, int, int, hipStream_t);
template void launch_to_double<double>(const double *, int, double *, int, int, int, hipStream_t);
template void launch_to_double<float>(const float *, int, double *, int, int, int, hipStream_t);

}  // namespace skew
