// Full-to-band reduction of a skew-symmetric matrix (Section 2.3.2: blocked
// Householder reduction with the compact WY form Q = I - V T V^T, and the
// skew two-sided update A <- Q^T A Q = A + V W^T - W V^T).
//
// For a panel with reflectors V (m x b) and T (b x b), with A the trailing
// skew block:  Y = A V T,  X = T^T V^T Y (b x b, skew),  W = Y - V X / 2, and
// then  A <- A + V W^T - W V^T.  (Derivation: V^T A = -(A V)^T for skew A, so
// the update of the paper's Eq. for ELPA2, A + [V U2][U1 V]^T, has U2 = -U1
// = -W.)  Only the strict lower triangle of A is stored and updated.
//
// Kernels:
//   k_ingest      copy the strict lower triangle of A into the work matrix,
//                 flagging non-finite entries
//   k_panel_qr    Householder QR of one panel (grid barriers; its few workgroups
//                 are resident together),
//                 rows resident in LDS, FP64 norms and dot products; also
//                 accumulates T column by column
//   k_skew_symm   Y0 = A V (split-K partials), A read from the lower triangle
//                 in both orientations
//   k_ysum        Y0 = sum of the split-K partials
//   k_gram        partial V^T Y0
//   k_small       X = T^T (V^T Y0) T and the 2b x b matrix [T; -X/2]
//   k_wform       W = [Y0 V] [T; -X/2]
//   k_skew_syr2k  lower tiles A += [V W][W -V]^T
//   k_band_extract  lower band storage of the result
#include "common.h"
#include "gemm.h"
#include "kernels.h"
#include "small64.h"

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_ingest(const double *__restrict__ A, int lda, int n,
                                                T *__restrict__ W, int ldw, unsigned *flags)
{
    const int j = blockIdx.y;
    bool bad = false;
    for (int i = j + 1 + blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        double a = A[(size_t)j * lda + i];
        if (!__builtin_isfinite(a)) bad = true;
        W[(size_t)j * ldw + i] = (T)a;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) W[(size_t)j * ldw + j] = T(0);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&flags[0], 1u);
}

// ---------------------------------------------------------------------------
// Panel QR.  ROWS rows per workgroup, 256 threads; the workgroup's rows live
// in LDS as P[g][0..B) (double).  Column l:
//   partial sums  s_t = sum_{g>l} P[g][l] P[g][t] (t >= l; t = l gives the
//   squared norm below the diagonal) and z_t = sum_{g>=l} P[g][t] P[g][l-1]
//   (t < l-1; dot products of the previous reflector with the earlier ones,
//   for T), one grid barrier, then every workgroup reduces the partials in
//   the same order (bitwise-identical scalars everywhere) and updates its rows.
// Row l (l < B <= ROWS) always lives in workgroup 0, which broadcasts it.
constexpr int PQR_ROWS = 128;

template <typename T, int B>
__global__ __launch_bounds__(256) void k_panel_qr(T *__restrict__ W, int ldw, int c0, int r0, int m,
                                                  T *__restrict__ Vd, double *__restrict__ tau,
                                                  double *__restrict__ Tf, double *__restrict__ part,
                                                  unsigned *bar, unsigned bar_base, unsigned *err,
                                                  const unsigned *__restrict__ skip)
{
    extern __shared__ double sm[];
    double *P = sm;                        // [ROWS][B]
    double *Ts = sm + PQR_ROWS * B;        // [B][B] column-major (workgroup 0 only)
    __shared__ double red[256];
    __shared__ double tot[B], piv[B], ppiv[B], wv[B], vtmp[PQR_ROWS];
    __shared__ double sc[4];               // tau, beta, scale, previous tau
    constexpr int NP = 256 / B;            // parts
    constexpr int RP = PQR_ROWS / NP;      // rows per part
    const int tid = threadIdx.x, wg = blockIdx.x, G = gridDim.x;
    const int tcol = tid % B, tp = tid / B;
    const int gbase = wg * PQR_ROWS;
    const int L = m < B ? m : B;           // columns that get a reflector
    double *pbuf = part;                   // [2][G][B]
    double *pvbuf = part + 2 * (size_t)G * B;  // [2][B]
    if (skip && *skip == 0u) {
        // the Cholesky-QR path factored this panel: advance the barrier
        // counter as the L + 1 barriers of this launch would have
        if (tid == 0) __hip_atomic_fetch_add(bar, (unsigned)(L + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }

    for (int e = tid; e < PQR_ROWS * B; e += 256) {
        int g = e / B, t = e % B;
        int gg = gbase + g;
        P[e] = (gg < m) ? (double)W[(size_t)(c0 + t) * ldw + r0 + gg] : 0.0;
    }
    if (wg == 0)
        for (int e = tid; e < B * B; e += 256) Ts[e] = 0.0;
    __syncthreads();

    unsigned nbar = 0;
    for (int l = 0; l <= L; ++l) {
        // ---- partial sums
        double val = 0.0;
        const int lm1 = l - 1;
        for (int r = 0; r < RP; ++r) {
            int g = tp * RP + r, gg = gbase + g;
            if (gg >= m) break;
            if (l < L && tcol >= l && gg > l) val += P[g * B + l] * P[g * B + tcol];
            if (tcol < lm1 && gg >= l) val += P[g * B + tcol] * P[g * B + lm1];
        }
        red[tid] = val;
        __syncthreads();
        const int par = l & 1;
        if (tid < B) {
            double s = 0.0;
            for (int p = 0; p < NP; ++p) s += red[p * B + tid];
            st_coh(&pbuf[((size_t)par * G + wg) * B + tid], s);
            if (wg == 0) st_coh(&pvbuf[par * B + tid], (l < L) ? P[l * B + tid] : 0.0);
        }
        ++nbar;
        if (!grid_sync_coh(bar, bar_base + nbar * G, err)) return;
        {
            // all threads: thread (tcol, tp) sums the partials of workgroups
            // [tp*wc, (tp+1)*wc) with every load in flight at once, then the
            // NP sums of a column are added in tp order; the order is the same
            // in every workgroup (bitwise-identical scalars everywhere)
            const int wc = (G + NP - 1) / NP;
            const int wb = tp * wc, we = min(G, wb + wc);
            double s = 0.0;
            for (int w0 = wb; w0 < we; w0 += 32) {
                double t32[32];
#pragma unroll
                for (int q = 0; q < 32; ++q)
                    t32[q] = (w0 + q < we) ? ld_coh(&pbuf[((size_t)par * G + w0 + q) * B + tcol]) : 0.0;
#pragma unroll
                for (int q = 0; q < 32; ++q) s += t32[q];
            }
            if (tp == 0) piv[tcol] = ld_coh(&pvbuf[par * B + tcol]);
            red[tid] = s;
            __syncthreads();
            if (tid < B) {
                double a = 0.0;
                for (int p = 0; p < NP; ++p) a += red[p * B + tid];
                tot[tid] = a;
            }
        }
        __syncthreads();
        // ---- T column l-1: T[0:l-1, l-1] = -tau_{l-1} T[0:l-1, 0:l-1] z
        if (wg == 0 && l >= 1) {
            const double tprev = sc[3];
            if (tid < lm1) {
                double s = 0.0;
                for (int u = tid; u < lm1; ++u) s += Ts[u * B + tid] * (tot[u] + ppiv[u]);
                red[tid] = -tprev * s;
            }
            __syncthreads();
            if (tid < lm1) Ts[lm1 * B + tid] = red[tid];
            if (tid == 0) Ts[lm1 * B + lm1] = tprev;
            __syncthreads();
        }
        if (l == L) break;
        // ---- reflector of column l (every workgroup, same arithmetic)
        if (tid == 0) {
            double x0 = piv[l], ss = tot[l];
            double t = 0.0, beta = x0, scale = 0.0;
            if (ss != 0.0) {
                double nrm = sqrt(x0 * x0 + ss);
                beta = (x0 >= 0.0) ? -nrm : nrm;
                t = (beta - x0) / beta;
                scale = 1.0 / (x0 - beta);
            }
            sc[0] = t; sc[1] = beta; sc[2] = scale;
        }
        __syncthreads();
        const double t = sc[0], beta = sc[1], scale = sc[2];
        if (tid < B) wv[tid] = (tid > l) ? t * (piv[tid] + scale * tot[tid]) : 0.0;
        if (tid < PQR_ROWS) {
            int gg = gbase + tid;
            vtmp[tid] = (gg > l && gg < m) ? P[tid * B + l] * scale : (gg == l ? 1.0 : 0.0);
        }
        if (tid < B) ppiv[tid] = piv[tid];
        __syncthreads();
        for (int r = 0; r < RP; ++r) {
            int g = tp * RP + r, gg = gbase + g;
            if (gg >= m) break;
            if (gg < l) continue;
            if (tcol > l) P[g * B + tcol] -= vtmp[g] * wv[tcol];
            else if (tcol == l) P[g * B + l] = (gg == l) ? beta : vtmp[g];
        }
        if (tid == 0) {
            sc[3] = t;
            if (wg == 0) tau[l] = t;
        }
        __syncthreads();
    }
    // columns without a reflector
    if (wg == 0 && tid >= L && tid < B) tau[tid] = 0.0;
    // ---- write back: R and V into the panel, dense V, T
    for (int e = tid; e < PQR_ROWS * B; e += 256) {
        int g = e % PQR_ROWS, t = e / PQR_ROWS;
        int gg = gbase + g;
        if (gg < m) {
            double p = P[g * B + t];
            W[(size_t)(c0 + t) * ldw + r0 + gg] = (T)p;
            double v = (gg > t) ? p : ((gg == t && t < L) ? 1.0 : 0.0);
            Vd[(size_t)t * m + gg] = (T)v;
        }
    }
    if (wg == 0)
        for (int e = tid; e < B * B; e += 256) Tf[e] = Ts[e];
}

// ---------------------------------------------------------------------------
// Y0 partial (split s): rows [m0, m0+64) of  A_trail V  over k in [kb, ke).
template <typename T, int TN>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_skew_symm(const T *__restrict__ W, int ldw, int r0, int m,
                                                   const T *__restrict__ Vd, int B,
                                                   T *__restrict__ Ypart, int kchunk)
{
    constexpr int TM = 64;
    extern __shared__ char smraw[];
    T *smem = (T *)smraw;
    const int m0 = blockIdx.x * TM;
    const int s = blockIdx.y;
    const int kb = s * kchunk, ke = min(m, kb + kchunk);
    const T *A0 = W + (size_t)r0 * ldw + r0;
    // every fetch is one unconditional load at a clamped (valid, finite)
    // address scaled by 0 or +-1: a select here would become a branch around
    // the load, and the chunk's loads would no longer be in flight together
    const int mc = m - 1;
    auto f_low = [=](int i, int k) -> T {      // k < i
        const T x = A0[(size_t)min(k, mc) * ldw + min(i, mc)];
        return x * T((i < m && k < ke) ? 1 : 0);
    };
    auto f_up = [=](int i, int k) -> T {       // k > i: A(i,k) = -A(k,i)
        const T x = A0[(size_t)min(i, mc) * ldw + min(k, mc)];
        return x * T((i < m && k < ke) ? -1 : 0);
    };
    auto f_mix = [=](int i, int k) -> T {
        const int r = max(i, k), c = min(i, k);
        const T x = A0[(size_t)min(c, mc) * ldw + min(r, mc)];
        return x * T((i >= m || k >= ke || i == k) ? 0 : ((i > k) ? 1 : -1));
    };
    auto f_v = [=](int j, int k) -> T {
        const T x = Vd[(size_t)min(j, B - 1) * m + min(k, mc)];
        return x * T((j < B && k < ke) ? 1 : 0);
    };
    gemm::Acc<T, TM, TN> acc;
    acc.zero();
    gemm::skew_kloop<T, TM, TN>(f_low, f_up, f_mix, f_v, m0, 0, kb, ke, smem, acc);
    T *Y = Ypart + (size_t)s * m * B;
    gemm::epilogue<T, TM, TN>(acc, smem, [=](int i, int j, T v) {
        if (m0 + i < m && j < B) Y[(size_t)j * m + m0 + i] = v;
    });
}

template <typename T>
__global__ void k_ysum(const T *__restrict__ Ypart, int S, size_t len, T *__restrict__ Y0)
{
    for (size_t e = blockIdx.x * (size_t)256 + threadIdx.x; e < len; e += (size_t)gridDim.x * 256) {
        // the loads of eight partials are issued together; the sum runs over
        // p in order
        double s = 0.0;
        int p = 0;
        for (; p + 8 <= S; p += 8) {
            double t[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) t[q] = (double)Ypart[(size_t)(p + q) * len + e];
#pragma unroll
            for (int q = 0; q < 8; ++q) s += t[q];
        }
        for (; p < S; ++p) s += (double)Ypart[(size_t)p * len + e];
        Y0[e] = (T)s;
    }
}

// Partial V^T Y0 over row chunk blockIdx.x (rows [c*rc, (c+1)*rc)).
template <typename T, int TB>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_gram(const T *__restrict__ Vd, const T *__restrict__ Y0,
                                              int m, int B, int rc, double *__restrict__ Gp)
{
    extern __shared__ char smraw[];
    T *smem = (T *)smraw;
    const int kb = blockIdx.x * rc, ke = min(m, kb + rc);
    auto fa = [=](int l, int g) -> T { return (l < B && g < ke) ? Vd[(size_t)l * m + g] : T(0); };
    auto fb = [=](int j, int g) -> T { return (j < B && g < ke) ? Y0[(size_t)j * m + g] : T(0); };
    gemm::Acc<T, TB, TB> acc;
    acc.zero();
    gemm::kloop<T, TB, TB, true, true>(fa, fb, 0, 0, kb, ke, smem, acc);
    double *G = Gp + (size_t)blockIdx.x * B * B;
    gemm::epilogue<T, TB, TB>(acc, smem, [=](int i, int j, T v) {
        if (i < B && j < B) G[(size_t)j * B + i] = (double)v;
    });
}

// X = T^T G T with G = sum of the chunk partials; Tx = [T; -X/2] (2B x B).
template <typename T>
__global__ __launch_bounds__(256) void k_small(const double *__restrict__ Gp, int nchunk, int B,
                                               const double *__restrict__ Tf, T *__restrict__ Tx)
{
    __shared__ double G[64 * 65], Tm[64 * 65], M1[64 * 65];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    auto off = [=](int i, int j) -> int { return (i < B && j < B) ? j * B + i : -1; };
    {
        double acc[16], tf[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int o = off(tx, ty + 4 * q);
            tf[q] = (o >= 0 && tx <= ty + 4 * q) ? Tf[o] : 0.0;   // T upper, zero elsewhere
        }
        sum_partials_2d(Gp, nchunk, (size_t)B * B, off, acc);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            G[tx * 65 + ty + 4 * q] = acc[q];        // G[i][u]
            Tm[tx * 65 + ty + 4 * q] = tf[q];        // T[u][j]
        }
    }
    __syncthreads();
    mm64<false>(G, Tm, M1);                          // M1 = G T
    __syncthreads();
    mm64<true>(Tm, M1, G);                           // X = T^T M1 (into G)
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int j = ty + 4 * q;
        if (tx < B && j < B) {
            Tx[(size_t)j * 2 * B + tx] = (T)Tm[tx * 65 + j];
            Tx[(size_t)j * 2 * B + B + tx] = (T)(-0.5 * G[tx * 65 + j]);
        }
    }
}

// W = [Y0 V] Tx  (m x B)
template <typename T, int TN>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_wform(const T *__restrict__ Y0, const T *__restrict__ Vd,
                                               const T *__restrict__ Tx, int m, int B,
                                               T *__restrict__ Wd)
{
    constexpr int TM = 64;
    extern __shared__ char smraw[];
    T *smem = (T *)smraw;
    const int m0 = blockIdx.x * TM;
    auto fa = [=](int i, int k) -> T {
        if (i >= m || k >= 2 * B) return T(0);
        return k < B ? Y0[(size_t)k * m + i] : Vd[(size_t)(k - B) * m + i];
    };
    auto fb = [=](int j, int k) -> T { return (j < B && k < 2 * B) ? Tx[(size_t)j * 2 * B + k] : T(0); };
    gemm::Acc<T, TM, TN> acc;
    acc.zero();
    gemm::kloop<T, TM, TN, false, true>(fa, fb, m0, 0, 0, 2 * B, smem, acc);
    gemm::epilogue<T, TM, TN>(acc, smem, [=](int i, int j, T v) {
        if (m0 + i < m && j < B) Wd[(size_t)j * m + m0 + i] = v;
    });
}

// Lower tiles (I >= J) of the trailing block: A += V W^T - W V^T.
template <typename T, int TT>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_skew_syr2k(T *__restrict__ W, int ldw, int r0, int m,
                                                    const T *__restrict__ Vd, const T *__restrict__ Wd,
                                                    int B, int ldv)
{
    extern __shared__ char smraw[];
    T *smem = (T *)smraw;
    int I, J;
    tri_index(blockIdx.x, I, J);
    const int m0 = I * TT, n0 = J * TT;
    // unconditional loads at clamped rows scaled by 0 or +-1 (no branch
    // around the loads); k < 2B always
    auto fa = [=](int i, int k) -> T {
        const bool lo = k < B;
        const T x = (lo ? Vd : Wd)[(size_t)(lo ? k : k - B) * ldv + min(i, m - 1)];
        return x * T(i < m ? 1 : 0);
    };
    auto fb = [=](int j, int k) -> T {
        const bool lo = k < B;
        const T x = (lo ? Wd : Vd)[(size_t)(lo ? k : k - B) * ldv + min(j, m - 1)];
        return x * T(j < m ? (lo ? 1 : -1) : 0);
    };
    gemm::Acc<T, TT, TT> acc;
    acc.zero();
    gemm::kloop<T, TT, TT, false, false>(fa, fb, m0, n0, 0, 2 * B, smem, acc);
    T *A0 = W + (size_t)r0 * ldw + r0;
    const bool diag = (I == J);
    auto inside = [=](int i, int j) { return m0 + i < m && n0 + j < m && (!diag || i > j); };
    gemm::epilogue_rmw<T, TT, TT>(
        acc, smem,
        // unconditional load at a clamped address: values outside are never
        // stored, and a test here would become a branch around every load
        [=](int i, int j) -> T { return A0[(size_t)min(n0 + j, m - 1) * ldw + min(m0 + i, m - 1)]; },
        [=](int i, int j, T old, T v) {
            if (inside(i, j)) A0[(size_t)(n0 + j) * ldw + m0 + i] = old + v;
        });
}

template <typename T>
__global__ void k_band_extract(const T *__restrict__ W, int ldw, int n, int b,
                               double *__restrict__ ab, int ldab)
{
    const int j = blockIdx.x * blockDim.y + threadIdx.y;
    if (j >= n) return;
    for (int d = threadIdx.x; d < ldab; d += blockDim.x) {
        double v = 0.0;
        if (d >= 1 && d <= b && j + d < n) v = (double)W[(size_t)j * ldw + j + d];
        ab[(size_t)j * ldab + d] = v;
    }
}

// ---------------------------------------------------------------------------
// Panel factorization by Cholesky QR twice plus Householder reconstruction
// (FP64, panel P of m >= B rows, B <= 64):
//   G1 = P^T P = R1^T R1,  Q1 = P R1^{-1},  G2 = Q1^T Q1 = R2^T R2,
//   Q = Q1 R2^{-1},  R = R2 R1,
// then the compact-WY form of the same orthogonal factor: the LU
// factorization Q[0:B, :] - S = L U with the signs S = diag(s_i) chosen on the
// fly (s_i = -sign of the pivot, so that |u_ii| >= 1 and no pivoting is
// needed) gives V = [L; Q[B:, :] U^{-1}], T = -U S L^{-T} and R_h = S R, with
// (I - V T V^T)^T P = [R_h; 0].  A Cholesky pivot that signals a panel too
// ill-conditioned (or rank deficient) for two passes sets the flag, and the
// Householder panel kernel takes over.
//
// Small 64 x 64 kernels: thread (tx, ty) = (tid % 64, tid / 64) owns row tx
// and columns ty + 4q (q = 0..15).
// Scratch layout (cq, doubles): G, R1, R1inv, R2inv, R, Uinv (indices CQ_*),
// each 64 x 64 column-major.
using skew::CQ_G;
using skew::CQ_R1;
using skew::CQ_R1INV;
using skew::CQ_R2INV;
using skew::CQ_R;
using skew::CQ_UINV;

// G[e] = sum over np partials (each B*B, column-major), in order.
__global__ __launch_bounds__(256) void k_gram_reduce(const double *__restrict__ Gp, int np, int BB,
                                                     double *__restrict__ G)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= BB) return;
    double s = 0.0;
    for (int p0 = 0; p0 < np; p0 += 16) {
        double t[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int p = min(p0 + q, np - 1);
            t[q] = Gp[(size_t)p * BB + e];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (p0 + q < np) s += t[q];
    }
    G[e] = s;
}

// Cholesky factor R (upper, G = R^T R) and R^{-1} of the Gram matrix: the
// sum of the np partials Gp (each B x B, summed in order, as
// k_gram_reduce does), or cq[CQ_G] when Gp is null.  pass 1: R1, R1^{-1}; flag = 1 when a pivot falls below
// 1e-13 max_i G_ii (condition of the panel beyond what two passes restore).
// pass 2 (skipped when the flag is set): R2^{-1} and R = R2 R1.  There
// G2 = I + E; when max |E_ij| <= 1e-8 the factor is taken to first order,
// R2 = I + diag(E)/2 + strict upper(E), R2^{-1} = I - diag(E)/2 - strict
// upper(E), whose neglected terms are O(|E|^2) <= 1e-16; otherwise R2 is
// factored, and flag = 1 when a pivot leaves (0.5, 2).
__global__ __launch_bounds__(256) void k_chol_qr(int B, int pass, double *__restrict__ cq,
                                                 unsigned *__restrict__ flag, const double *__restrict__ Gp,
                                                 int np)
{
    __shared__ double M[64 * 65], X[64 * 65], R1s[64 * 65], part[4];
    __shared__ __attribute__((aligned(16))) double buf[320];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    if (pass == 2 && *flag) return;
    const size_t BB = 64 * 64;
    const double *G = cq + CQ_G * BB;
    const double *R1 = cq + CQ_R1 * BB;
    double emax = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int j = ty + 4 * q;
        const bool in = tx < B && j < B;
        double gv = 0.0;
        if (in) {
            if (Gp) {
                for (int p = 0; p < np; ++p) gv += Gp[(size_t)p * B * B + (size_t)j * B + tx];
            } else {
                gv = G[(size_t)j * B + tx];
            }
        }
        M[tx * 65 + j] = gv;
        if (pass == 2) {
            R1s[tx * 65 + j] = in ? R1[(size_t)j * B + tx] : 0.0;
            if (in) emax = fmax(emax, fabs(gv - ((tx == j) ? 1.0 : 0.0)));
        }
    }
    if (pass == 2) {
        const double wm = wave_max(emax);
        if (tx == 0) part[ty] = wm;
    }
    __syncthreads();
    bool first_order = false;
    if (pass == 2) first_order = fmax(fmax(part[0], part[1]), fmax(part[2], part[3])) <= 1e-8;
    if (first_order) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = ty + 4 * q;
            const double e = M[tx * 65 + c] - ((tx == c) ? 1.0 : 0.0);
            const double f = (tx == c) ? 0.5 * e : ((tx < c) ? e : 0.0);
            X[tx * 65 + c] = ((tx == c) ? 1.0 : 0.0) - f;                                 // R2^{-1}
            M[tx * 65 + c] = ((tx == c) ? 1.0 + 0.5 * e : ((tx < c) ? e : 0.0));         // R2
        }
        __syncthreads();
    } else {
        double dmax = 0.0;
#pragma unroll
        for (int i = 0; i < 64; ++i) dmax = fmax(dmax, (i < B) ? M[i * 65 + i] : 0.0);
        const double lo = (pass == 1) ? 1e-13 * dmax : 0.5, hi = (pass == 1) ? 2.0 * dmax : 2.0;
        if (!chol_inv64(M, X, B, false, lo, hi, buf)) {
            if (tid == 0) *flag = 1u;
            return;
        }
    }
    double *Ro = cq + ((pass == 1) ? CQ_R1 : CQ_R) * BB;
    double *Ri = cq + ((pass == 1) ? CQ_R1INV : CQ_R2INV) * BB;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int j = ty + 4 * q;
        if (tx < B && j < B) Ri[(size_t)j * B + tx] = X[tx * 65 + j];
    }
    if (pass == 2) {   // R = R2 R1 on the MFMA, into X once R2^{-1} is stored
        __syncthreads();
        mm64<false>(M, R1s, X);
        __syncthreads();
    }
    const double *Rs = (pass == 1) ? M : X;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int j = ty + 4 * q;
        if (tx < B && j < B) Ro[(size_t)j * B + tx] = (tx <= j) ? Rs[tx * 65 + j] : 0.0;
    }
    if (pass == 1 && tid == 0) *flag = 0u;
}

// Householder reconstruction from the orthonormal Q (in Vd, m x B, ld m):
// writes V's top block L into Vd, T into Tf (column-major), tau = diag(T),
// R_h = S R into the panel's top block of W (upper triangle), U^{-1} into
// cq[CQ_UINV].  Nothing is done when the flag is set.  One workgroup: the
// signed LU of the top block with L^{-1} and U^{-1} in one elimination pass,
// then T = -U S L^{-T} on the MFMA.  The input block is read into LDS before
// L overwrites it.
template <typename T>
__global__ __launch_bounds__(256) void k_hh_rebuild(T *__restrict__ Vd, int m, int B, T *__restrict__ Wp,
                                                    int ldw, double *__restrict__ cq, double *__restrict__ Tf,
                                                    double *__restrict__ tau, const unsigned *__restrict__ flag)
{
    __shared__ double M[64 * 65], Xu[64 * 65], Yl[64 * 65], sgn[64];
    __shared__ __attribute__((aligned(16))) double buf[1024];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    if (*flag) return;
    const size_t BB = 64 * 64;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int j = ty + 4 * q;
        M[tx * 65 + j] = (tx < B && j < B) ? (double)Vd[(size_t)j * m + tx] : 0.0;
    }
    __syncthreads();
    lu_signed_inv64(M, Xu, Yl, B, sgn, buf);
    const double *R = cq + CQ_R * BB;
    double *Ui = cq + CQ_UINV * BB;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int c = ty + 4 * q, r = tx;
        if (r < B && c < B) {
            Vd[(size_t)c * m + r] = (T)((r > c) ? M[r * 65 + c] : ((r == c) ? 1.0 : 0.0));
            Ui[(size_t)c * B + r] = Xu[r * 65 + c];
            if (r <= c) Wp[(size_t)c * ldw + r] = (T)(sgn[r] * R[(size_t)c * B + r]);
        }
    }
    __syncthreads();
    // U S into Xu, L^{-T} into M (each thread rewrites the elements it read)
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int c = ty + 4 * q, r = tx;
        Xu[r * 65 + c] = (r <= c && c < B) ? M[r * 65 + c] * sgn[c] : 0.0;   // sgn[c >= B] is not set
        M[r * 65 + c] = Yl[c * 65 + r];
    }
    __syncthreads();
    mm64<false>(Xu, M, Yl);   // Yl = U S L^{-T}
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int c = ty + 4 * q, r = tx;
        if (r < B && c < B) {
            Tf[(size_t)c * B + r] = (r <= c) ? -Yl[r * 65 + c] : 0.0;
            if (r == c) tau[r] = -Yl[r * 65 + r];
        }
    }
}



// 32-bit fill (clears control words and buffers; a kernel rather than a
// runtime memset so that the same sequence can be captured in a graph)
__global__ void k_fill32(unsigned *__restrict__ p, unsigned v, size_t nw)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < nw; i += (size_t)gridDim.x * 256) p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
namespace skew {

void launch_fill32(void *p, unsigned v, size_t nwords, hipStream_t st)
{
    if (nwords == 0) return;
    size_t g = (nwords + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill32, dim3((unsigned)g), dim3(256), 0, st, (unsigned *)p, v, nwords);
}

template <typename T>
void launch_ingest(const double *A, int lda, int n, T *W, int ldw, unsigned *flags, hipStream_t st)
{
    if (n <= 0) return;
    dim3 grid(cdiv(n, 256) > 16 ? 16 : cdiv(n, 256), n);
    hipLaunchKernelGGL(k_ingest<T>, grid, dim3(256), 0, st, A, lda, n, W, ldw, flags);
}

int panel_qr_groups(int m) { return (int)cdiv(m, PQR_ROWS); }
size_t panel_qr_part_doubles(int m, int B) { return 2 * (size_t)panel_qr_groups(m) * B + 2 * B; }

template <typename T, int B>
static hipError_t panel_qr_b(T *W, int ldw, int c0, int r0, int m, T *Vd, double *tau, double *Tf,
                             double *part, unsigned *bar, unsigned bar_base, unsigned *err,
                             const unsigned *skip, hipStream_t st)
{
    const int G = panel_qr_groups(m);
    size_t shm = sizeof(double) * ((size_t)PQR_ROWS * B + (size_t)B * B);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_panel_qr<T, B>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
        attr = true;
    }
    // an ordinary launch: at most m / 128 workgroups of one per CU, launched in
    // stream order after the panel's producers, so they are resident together;
    // the grid barriers are bounded all the same (code 1 in *err)
    hipLaunchKernelGGL((k_panel_qr<T, B>), dim3(G), dim3(256), shm, st, W, ldw, c0, r0, m, Vd, tau, Tf, part, bar,
                       bar_base, err, skip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_panel_qr(T *W, int ldw, int c0, int r0, int m, int B, T *Vd, double *tau, double *Tf,
                           double *part, unsigned *bar, unsigned bar_base, unsigned *err, const unsigned *skip,
                           hipStream_t st)
{
    switch (B) {
    case 8: return panel_qr_b<T, 8>(W, ldw, c0, r0, m, Vd, tau, Tf, part, bar, bar_base, err, skip, st);
    case 16: return panel_qr_b<T, 16>(W, ldw, c0, r0, m, Vd, tau, Tf, part, bar, bar_base, err, skip, st);
    case 32: return panel_qr_b<T, 32>(W, ldw, c0, r0, m, Vd, tau, Tf, part, bar, bar_base, err, skip, st);
    case 64: return panel_qr_b<T, 64>(W, ldw, c0, r0, m, Vd, tau, Tf, part, bar, bar_base, err, skip, st);
    default: return hipErrorInvalidValue;
    }
}

int symm_splits(int m)
{
    // about 16 workgroups per CU: the long K loops of few row tiles leave
    // the MFMA pipes idle otherwise
    int rows = (int)cdiv(m, 64);
    int S = (int)cdiv(4096, rows > 0 ? rows : 1);
    int maxS = (int)cdiv(m, 256);
    if (S > maxS) S = maxS;
    if (S > 16) S = 16;
    if (S < 1) S = 1;
    return S;
}
int symm_kchunk(int m, int S) { return (int)(cdiv(cdiv(m, S), 16) * 16); }
int gram_chunk_rows() { return 256; }

template <typename T>
void launch_stage1_w(T *W, int ldw, int r0, int m, int B, const T *Vd, const double *Tf, T *Ypart,
                     T *Y0, T *Wd, double *Gp, T *Tx, hipStream_t st)
{
    const int S = symm_splits(m);
    const int kc = symm_kchunk(m, S);
    const int S_eff = (int)cdiv(m, kc);
    dim3 g1(cdiv(m, 64), S_eff);
    if (B > 32) {
        hipLaunchKernelGGL((k_skew_symm<T, 64>), g1, dim3(256), (gemm::smem_bytes<T, 64, 64>()), st,
                           (const T *)W, ldw, r0, m, Vd, B, Ypart, kc);
    } else {
        hipLaunchKernelGGL((k_skew_symm<T, 32>), g1, dim3(256), (gemm::smem_bytes<T, 64, 32>()), st,
                           (const T *)W, ldw, r0, m, Vd, B, Ypart, kc);
    }
    size_t len = (size_t)m * B;
    hipLaunchKernelGGL(k_ysum<T>, dim3(cdiv(len, 256) > 2048 ? 2048 : cdiv(len, 256)), dim3(256), 0, st,
                       (const T *)Ypart, S_eff, len, Y0);
    const int rc = gram_chunk_rows();
    const int nch = (int)cdiv(m, rc);
    if (B > 32)
        hipLaunchKernelGGL((k_gram<T, 64>), dim3(nch), dim3(256), (gemm::smem_bytes<T, 64, 64>()), st,
                           (const T *)Vd, (const T *)Y0, m, B, rc, Gp);
    else
        hipLaunchKernelGGL((k_gram<T, 32>), dim3(nch), dim3(256), (gemm::smem_bytes<T, 32, 32>()), st,
                           (const T *)Vd, (const T *)Y0, m, B, rc, Gp);
    if (nch > 16) {
        // many partials: a parallel reduction first, into the spare block
        // after them (the buffer holds m / rc + 2 blocks)
        double *G1 = Gp + (size_t)nch * B * B;
        hipLaunchKernelGGL(k_gram_reduce, dim3(cdiv(B * B, 256)), dim3(256), 0, st, (const double *)Gp, nch, B * B,
                           G1);
        hipLaunchKernelGGL(k_small<T>, dim3(1), dim3(256), 0, st, (const double *)G1, 1, B, Tf, Tx);
    } else {
        hipLaunchKernelGGL(k_small<T>, dim3(1), dim3(256), 0, st, (const double *)Gp, nch, B, Tf, Tx);
    }
    if (B > 32)
        hipLaunchKernelGGL((k_wform<T, 64>), dim3(cdiv(m, 64)), dim3(256), (gemm::smem_bytes<T, 64, 64>()), st,
                           (const T *)Y0, Vd, (const T *)Tx, m, B, Wd);
    else
        hipLaunchKernelGGL((k_wform<T, 32>), dim3(cdiv(m, 64)), dim3(256), (gemm::smem_bytes<T, 64, 32>()), st,
                           (const T *)Y0, Vd, (const T *)Tx, m, B, Wd);
}

template <typename T>
void launch_syr2k_ld(T *W, int ldw, int r0, int m, int B, const T *Vd, const T *Wd, int ldv, hipStream_t st)
{
    const int TT = 64;
    unsigned nt = cdiv(m, TT);
    unsigned ntiles = nt * (nt + 1) / 2;
    hipLaunchKernelGGL((k_skew_syr2k<T, 64>), dim3(ntiles), dim3(256), (gemm::smem_bytes<T, 64, 64>()), st,
                       W, ldw, r0, m, Vd, (const T *)Wd, B, ldv);
}

template <typename T>
void launch_stage1_syr2k(T *W, int ldw, int r0, int m, int B, const T *Vd, const T *Wd, hipStream_t st)
{
    launch_syr2k_ld<T>(W, ldw, r0, m, B, Vd, Wd, m, st);
}

template <typename T>
void launch_band_extract(const T *W, int ldw, int n, int b, double *ab, int ldab, hipStream_t st)
{
    if (n <= 0) return;
    dim3 blk(64, 4);
    hipLaunchKernelGGL(k_band_extract<T>, dim3(cdiv(n, 4)), blk, 0, st, W, ldw, n, b, ab, ldab);
}

template void launch_ingest<double>(const double *, int, int, double *, int, unsigned *, hipStream_t);
template void launch_ingest<float>(const double *, int, int, float *, int, unsigned *, hipStream_t);
void launch_gram_reduce(const double *Gp, int np, int BB, double *G, hipStream_t st)
{
    hipLaunchKernelGGL(k_gram_reduce, dim3(cdiv(BB, 256)), dim3(256), 0, st, Gp, np, BB, G);
}
void launch_chol_qr(int B, int pass, double *cq, unsigned *flag, hipStream_t st, const double *Gp, int np)
{
    hipLaunchKernelGGL(k_chol_qr, dim3(1), dim3(256), 0, st, B, pass, cq, flag, Gp, np);
}
template <typename T>
void launch_hh_rebuild(T *Vd, int m, int B, T *Wp, int ldw, double *cq, double *Tf, double *tau,
                       const unsigned *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_hh_rebuild<T>, dim3(1), dim3(256), 0, st, Vd, m, B, Wp, ldw, cq, Tf, tau, flag);
}
template void launch_hh_rebuild<double>(double *, int, int, double *, int, double *, double *, double *,
                                        const unsigned *, hipStream_t);
template void launch_hh_rebuild<float>(float *, int, int, float *, int, double *, double *, double *,
                                       const unsigned *, hipStream_t);
size_t cholqr_scratch_doubles() { return (size_t)6 * 64 * 64; }

template hipError_t launch_panel_qr<double>(double *, int, int, int, int, int, double *, double *, double *,
                                            double *, unsigned *, unsigned, unsigned *, const unsigned *,
                                            hipStream_t);
template hipError_t launch_panel_qr<float>(float *, int, int, int, int, int, float *, double *, double *,
                                           double *, unsigned *, unsigned, unsigned *, const unsigned *,
                                           hipStream_t);
template void launch_stage1_w<double>(double *, int, int, int, int, const double *, const double *, double *,
                                      double *, double *, double *, double *, hipStream_t);
template void launch_stage1_w<float>(float *, int, int, int, int, const float *, const double *, float *,
                                     float *, float *, double *, float *, hipStream_t);
template void launch_stage1_syr2k<double>(double *, int, int, int, int, const double *, const double *,
                                          hipStream_t);
template void launch_syr2k_ld<double>(double *, int, int, int, int, const double *, const double *, int,
                                      hipStream_t);
template void launch_stage1_syr2k<float>(float *, int, int, int, int, const float *, const float *,
                                         hipStream_t);
template void launch_band_extract<double>(const double *, int, int, int, double *, int, hipStream_t);
template void launch_band_extract<float>(const float *, int, int, int, double *, int, hipStream_t);

}  // namespace skew
