// Complex Hermitian route: the eigenproblem of the Hermitian matrix H = iA
// solved with complex arithmetic, as a general complex Hermitian solver would
// (the comparison of the paper's introduction and Section 4.1, where the skew
// solver is weighed against complex ELPA on iA).  Nothing here uses the
// structure of iA: H is held as two planes (real and imaginary parts of its
// lower triangle), reduced to a real symmetric tridiagonal matrix by complex
// Householder reflectors blocked by panels of 64 columns (one stage), and the
// eigenvectors are back-transformed with the reflectors' complex compact-WY
// blocks.
//
// Reflector of column c (rows r = c + 1 ..): H_c = I - tau v v^H with v_0 = 1,
// H_c^H x = beta e_0 for the current column x, beta real (so the tridiagonal
// matrix is real: e_c = beta, d_c the current diagonal entry).  Applying H_c
// from both sides with y = H v: H <- H - v w^H - w v^H, w = tau y + alpha v,
// alpha = -|tau|^2 (v^H y) / 2 (v^H y is real).  Inside a panel the update is
// deferred: H_cur = H - V W^H - W V^H over the panel's earlier columns, so
// y = H_cur v = H v - V (W^H v) - W (V^H v).
//
//   k_h_col    the current column with its deferred update, d_c, the
//              reflector (tau complex, beta) and v into column jj of V;
//   k_h_hemv   H v over the stored lower triangle (H_ij = conj(H_ji), real
//              diagonal) in vertical strips of tiles: per tile the row
//              partial L v_J and the scalar 2 Re(v_I^H L v_J) (plus
//              sum d_i |v_i|^2 on diagonal tiles), per strip the column
//              partial sum of L^H v_I, on diagonal tiles the partial dot
//              products V^H v, W^H v;
//   k_h_dots   those sums (D1 = V^H v, D2 = W^H v), alpha from
//              v^H y_cur = v^H H v - 2 Re(D1^H D2), and the T column;
//   k_h_w      w = tau (y - V D2 - W D1) + alpha v, and the next column's
//              deferred update but its V(:, jj) conj(w(r)) term;
//   k_her2k    per panel the lower tiles of H -= V W^H + W V^H, the real and
//              the imaginary plane each as one real rank-4b product;
//   k_h_bt_t   the back-transformation's middle step (see launch_herm_bt).
#include "common.h"
#include "gemm.h"
#include "kernels.h"

namespace {

constexpr int OT = 64;   // tile
constexpr int SS = 8;    // longest strip of tiles
constexpr int CT = 1024; // threads of the column kernel

// strip length for nt x nt tiles: long strips for large blocks, single tiles
// for small ones (where a strip's tiles would run one after another)
__host__ __device__ __forceinline__ int strip_len(int nt) { return nt >= 16 * SS ? SS : (nt >= 16 ? nt / 16 : 1); }

__device__ __forceinline__ int nstrips(int nt) { return (nt + strip_len(nt) - 1) / strip_len(nt); }

// workgroup t -> strip s, column block J (strip s spans J < nt - s ss)
__device__ __forceinline__ void strip_of(int t, int nt, int ss, int &s, int &J)
{
    s = 0;
    while (t >= nt - s * ss) {
        t -= nt - s * ss;
        ++s;
    }
    J = t;
}

// V, W: planes of the panel (rows c0 + 1 ..., ldv); tau: [64] real parts then
// [64] imaginary parts.  For jj > 0 column jj of V holds, from the row above
// the reflector's first row (the diagonal entry) down, the current column
// but the term V(:, jj-1) conj(W(c, jj-1)).
__global__ __launch_bounds__(CT) void k_h_col(const double *__restrict__ Hr, const double *__restrict__ Hi, int lda,
                                              int n, int c0, int jj, double *__restrict__ Vr,
                                              double *__restrict__ Vi, double *__restrict__ Wr,
                                              double *__restrict__ Wi, int ldv, double *__restrict__ tau,
                                              double *__restrict__ d, double *__restrict__ e)
{
    __shared__ double red[CT / 64];
    __shared__ double bsc[2];
    const int c = c0 + jj, r = c + 1, m = n - r, off = jj;
    const int tid = threadIdx.x;
    double *cr = Vr + (size_t)jj * ldv + off, *ci = Vi + (size_t)jj * ldv + off;
    double wcr = 0.0, wci = 0.0;
    const double *pr = cr, *pi = ci;
    if (jj > 0) {
        wcr = Wr[(size_t)(jj - 1) * ldv + off - 1];
        wci = Wi[(size_t)(jj - 1) * ldv + off - 1];
        pr = Vr + (size_t)(jj - 1) * ldv + off;
        pi = Vi + (size_t)(jj - 1) * ldv + off;
    }
    if (tid == 0) {
        // V(c, jj-1) = 1: the missing term of the diagonal is conj(w_c), real part Re w_c
        d[c] = (jj > 0) ? cr[-1] - wcr : Hr[(size_t)c * lda + c];
    }
    double sq = 0.0;
    for (int i = tid; i < m; i += CT) {
        double xr, xi;
        if (jj > 0) {
            const double ar = pr[i], ai = pi[i];
            xr = cr[i] - (ar * wcr + ai * wci);      // p - V(i, jj-1) conj(w_c)
            xi = ci[i] - (ai * wcr - ar * wci);
        } else {
            xr = Hr[(size_t)c * lda + r + i];
            xi = Hi[(size_t)c * lda + r + i];
        }
        cr[i] = xr;
        ci[i] = xi;
        if (i > 0) sq += xr * xr + xi * xi;
    }
    sq = wave_sum(sq);
    if ((tid & 63) == 0) red[tid >> 6] = sq;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int q = 0; q < CT / 64; ++q) s += red[q];
        const double ar = cr[0], ai = ci[0];
        double tr = 0.0, ti = 0.0, beta = ar, sr = 0.0, si = 0.0;
        if (s != 0.0 || ai != 0.0) {
            const double nrm = sqrt(ar * ar + ai * ai + s);
            beta = (ar >= 0.0) ? -nrm : nrm;
            tr = (beta - ar) / beta;
            ti = -ai / beta;
            const double ur = ar - beta, den = ur * ur + ai * ai;   // 1 / (alpha - beta)
            sr = ur / den;
            si = -ai / den;
        }
        bsc[0] = sr;
        bsc[1] = si;
        tau[jj] = tr;
        tau[64 + jj] = ti;
        e[c] = beta;
    }
    __syncthreads();
    // rows above the reflector's first row hold zeros in V and W (the
    // diagonal entry's slot was read above)
    for (int i = tid; i < off; i += CT) {
        Vr[(size_t)jj * ldv + i] = 0.0;
        Vi[(size_t)jj * ldv + i] = 0.0;
        Wr[(size_t)jj * ldv + i] = 0.0;
        Wi[(size_t)jj * ldv + i] = 0.0;
    }
    const double sr = bsc[0], si = bsc[1];
    for (int i = tid; i < m; i += CT) {
        if (i == 0) {
            cr[0] = 1.0;
            ci[0] = 0.0;
        } else {
            const double xr = cr[i], xi = ci[i];
            cr[i] = xr * sr - xi * si;
            ci[i] = xr * si + xi * sr;
        }
    }
}

// Prow: per tile (I, J) 128 doubles (real parts, then imaginary parts);
// Pcol: per strip (J, s) 128 doubles; Ps: per workgroup (strip) one double,
// the sum of its tiles' scalars; Pd: per row block 256 doubles (Re, Im of
// V^H v, then Re, Im of W^H v, 64 each).
__global__ __launch_bounds__(256) void k_h_hemv(const double *__restrict__ Hr, const double *__restrict__ Hi,
                                                int lda, int r, int m, const double *__restrict__ vr,
                                                const double *__restrict__ vi, const double *__restrict__ Vr,
                                                const double *__restrict__ Vi, const double *__restrict__ Wr,
                                                const double *__restrict__ Wi, int ldv, int off, int jj,
                                                double *__restrict__ Prow, double *__restrict__ Pcol,
                                                double *__restrict__ Ps, double *__restrict__ Pd)
{
    __shared__ double vIr[OT], vIi[OT], vJr[OT], vJi[OT], pr[4][OT], pim[4][OT];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int nt = (m + OT - 1) / OT, ss = strip_len(nt);
    int s, J;
    strip_of(blockIdx.x, nt, ss, s, J);
    const int Ib = max(J, nt - (s + 1) * ss), Ie = nt - s * ss;
    const int j0 = J * OT;
    if (tid < OT) vJr[tid] = (j0 + tid < m) ? vr[j0 + tid] : 0.0;
    else if (tid < 2 * OT) vJi[tid - OT] = (j0 + tid - OT < m) ? vi[j0 + tid - OT] : 0.0;
    const double *Ar = Hr + (size_t)r * lda + r, *Ai = Hi + (size_t)r * lda + r;
    double csr[16], csi[16], scs = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) csr[q] = csi[q] = 0.0;
    for (int I = Ib; I < Ie; ++I) {
        const int i0 = I * OT, i = i0 + tx;
        if (tid < OT) vIr[tid] = (i0 + tid < m) ? vr[i0 + tid] : 0.0;
        else if (tid < 2 * OT) vIi[tid - OT] = (i0 + tid - OT < m) ? vi[i0 + tid - OT] : 0.0;
        __syncthreads();
        const double ur = vIr[tx], ui = vIi[tx];
        double rr = 0.0, ri = 0.0;
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
            const int jl = ty + 4 * q, j = j0 + jl;
            const bool in = i < m && j < m && (I != J || tx > jl);
            const double xr = in ? Ar[(size_t)j * lda + i] : 0.0;
            const double xi = in ? Ai[(size_t)j * lda + i] : 0.0;
            const double br = vJr[jl], bi = vJi[jl];
            rr = fma(xr, br, fma(-xi, bi, rr));           // L v_J
            ri = fma(xr, bi, fma(xi, br, ri));
            csr[q] = fma(xr, ur, fma(xi, ui, csr[q]));    // conj(L) v_I, summed over rows
            csi[q] = fma(xr, ui, fma(-xi, ur, csi[q]));
        }
        pr[ty][tx] = rr;
        pim[ty][tx] = ri;
        __syncthreads();
        const size_t t = (size_t)I * (I + 1) / 2 + J;
        if (ty == 0) {
            double yr = pr[0][tx] + pr[1][tx] + pr[2][tx] + pr[3][tx];
            double yi = pim[0][tx] + pim[1][tx] + pim[2][tx] + pim[3][tx];
            const double dg = (I == J && i < m) ? Hr[(size_t)(r + i) * lda + r + i] : 0.0;
            const double sc = wave_sum(2.0 * (ur * yr + ui * yi) + dg * (ur * ur + ui * ui));
            yr = fma(dg, ur, yr);
            yi = fma(dg, ui, yi);
            Prow[t * 128 + tx] = yr;
            Prow[t * 128 + 64 + tx] = yi;
            scs += sc;
        }
        if (I == J) {
            // partial dots over the block's 64 rows: wave w takes k = w, w + 4,
            // ..., all loads first
            double pv[16][2], pw[16][2];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int k = ty + 4 * u;
                const bool ok = k < jj && i < m;
                const size_t o = (size_t)k * ldv + off + i;
                pv[u][0] = ok ? Vr[o] : 0.0;
                pv[u][1] = ok ? Vi[o] : 0.0;
                pw[u][0] = ok ? Wr[o] : 0.0;
                pw[u][1] = ok ? Wi[o] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int k = ty + 4 * u;
                if (k >= jj) break;
                const double ar = wave_sum(pv[u][0] * ur + pv[u][1] * ui);
                const double ai = wave_sum(pv[u][0] * ui - pv[u][1] * ur);
                const double br = wave_sum(pw[u][0] * ur + pw[u][1] * ui);
                const double bi = wave_sum(pw[u][0] * ui - pw[u][1] * ur);
                if (tx == 0) {
                    Pd[(size_t)I * 256 + k] = ar;
                    Pd[(size_t)I * 256 + 64 + k] = ai;
                    Pd[(size_t)I * 256 + 128 + k] = br;
                    Pd[(size_t)I * 256 + 192 + k] = bi;
                }
            }
        }
        __syncthreads();
    }
    double *pc = Pcol + ((size_t)J * nstrips(nt) + s) * 128;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const double a = wave_sum(csr[q]), b = wave_sum(csi[q]);
        if (tx == 0) {
            pc[ty + 4 * q] = a;
            pc[64 + ty + 4 * q] = b;
        }
    }
    if (tid == 0) Ps[blockIdx.x] = scs;
}

// D: [0, 64) Re D1, [64, 128) Im D1, [128, 192) Re D2, [192, 256) Im D2,
// D[256] = alpha.  T: real and imaginary planes, column-major, ldt = 64.
__global__ __launch_bounds__(256) void k_h_dots(const double *__restrict__ Pd, int nt, const double *__restrict__ Ps,
                                                int nps, int jj, const double *__restrict__ tau,
                                                double *__restrict__ D, double *__restrict__ Tr,
                                                double *__restrict__ Ti)
{
    __shared__ double Tsr[64 * 64], Tsi[64 * 64];
    __shared__ double dv[256], red[256];
    const int tid = threadIdx.x, k = tid & 63;
    for (int x = tid; x < jj * 64; x += 256) {
        Tsr[x] = Tr[x];
        Tsi[x] = Ti[x];
    }
    double a0 = 0.0, a1 = 0.0;
    if (k < jj) {
        int I = 0;
        for (; I + 1 < nt; I += 2) {
            a0 += Pd[(size_t)I * 256 + tid];
            a1 += Pd[(size_t)(I + 1) * 256 + tid];
        }
        if (I < nt) a0 += Pd[(size_t)I * 256 + tid];
    }
    dv[tid] = a0 + a1;
    D[tid] = a0 + a1;
    double sc0 = 0.0, sc1 = 0.0;
    int t = tid;
    for (; t + 256 < nps; t += 512) {
        sc0 += Ps[t];
        sc1 += Ps[t + 256];
    }
    if (t < nps) sc0 += Ps[t];
    red[tid] = sc0 + sc1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    const double tr = tau[jj], ti = tau[64 + jj];
    if (tid == 0) {
        double g = 0.0;   // Re(D1^H D2)
        for (int q = 0; q < jj; ++q) g += dv[q] * dv[128 + q] + dv[64 + q] * dv[192 + q];
        D[256] = -0.5 * (tr * tr + ti * ti) * (red[0] - 2.0 * g);
    }
    if (tid < 64) {
        if (k < jj) {
            double gr = 0.0, gi = 0.0;    // (T(:jj, :jj) D1)_k, T upper
            for (int u = k; u < jj; ++u) {
                const double xr = Tsr[u * 64 + k], xi = Tsi[u * 64 + k], br = dv[u], bi = dv[64 + u];
                gr += xr * br - xi * bi;
                gi += xr * bi + xi * br;
            }
            Tr[(size_t)jj * 64 + k] = -(tr * gr - ti * gi);
            Ti[(size_t)jj * 64 + k] = -(tr * gi + ti * gr);
        } else {
            Tr[(size_t)jj * 64 + k] = (k == jj) ? tr : 0.0;
            Ti[(size_t)jj * 64 + k] = (k == jj) ? ti : 0.0;
        }
    }
}

// w for rows i0 .. i0 + 63; with next set, the partial next column (rows
// from r, the diagonal entry first) into column jj + 1 of V.  Wave q takes
// the tiles, strips and columns k = q mod 4; the wave sums are added in order.
__global__ __launch_bounds__(256) void k_h_w(const double *__restrict__ Hr, const double *__restrict__ Hi, int lda,
                                             int r, int m, int nt, const double *__restrict__ Prow,
                                             const double *__restrict__ Pcol, const double *__restrict__ D,
                                             double *__restrict__ Vr, double *__restrict__ Vi,
                                             double *__restrict__ Wr, double *__restrict__ Wi, int ldv, int off,
                                             int jj, const double *__restrict__ tau, int next)
{
    __shared__ double p[4][4][OT];
    const int I = blockIdx.x, tx = threadIdx.x & 63, q = threadIdx.x >> 6, i = I * OT + tx;
    const bool in = i < m, nx = next && in;
    double yr = 0.0, yi = 0.0, ar = 0.0, ai = 0.0;
    const double *prw = Prow + (size_t)(I * (I + 1) / 2) * 128 + tx;
    for (int J = q; J <= I; J += 4) {
        yr += prw[(size_t)J * 128];
        yi += prw[(size_t)J * 128 + 64];
    }
    const double *pc = Pcol + (size_t)I * nstrips(nt) * 128 + tx;
    const int ss = strip_len(nt);
    for (int s = q; s * ss < nt - I; s += 4) {
        yr += pc[(size_t)s * 128];
        yi += pc[(size_t)s * 128 + 64];
    }
    if (in)
        for (int k = q; k < jj; k += 4) {
            const size_t o = (size_t)k * ldv + off;
            const double vr_ = Vr[o + i], vi_ = Vi[o + i], wr_ = Wr[o + i], wi_ = Wi[o + i];
            const double d1r = D[k], d1i = D[64 + k], d2r = D[128 + k], d2i = D[192 + k];
            yr -= (vr_ * d2r - vi_ * d2i) + (wr_ * d1r - wi_ * d1i);     // - V D2 - W D1
            yi -= (vr_ * d2i + vi_ * d2r) + (wr_ * d1i + wi_ * d1r);
            if (nx) {
                // - V(i, k) conj(W(r, k)) - W(i, k) conj(V(r, k))
                const double qwr = Wr[o], qwi = Wi[o], qvr = Vr[o], qvi = Vi[o];
                ar -= (vr_ * qwr + vi_ * qwi) + (wr_ * qvr + wi_ * qvi);
                ai -= (vi_ * qwr - vr_ * qwi) + (wi_ * qvr - wr_ * qvi);
            }
        }
    p[0][q][tx] = yr;
    p[1][q][tx] = yi;
    p[2][q][tx] = ar;
    p[3][q][tx] = ai;
    __syncthreads();
    if (q != 0 || !in) return;
    const double ur = ((p[0][0][tx] + p[0][1][tx]) + p[0][2][tx]) + p[0][3][tx];
    const double ui = ((p[1][0][tx] + p[1][1][tx]) + p[1][2][tx]) + p[1][3][tx];
    const double tr = tau[jj], ti = tau[64 + jj], alpha = D[256];
    const size_t o = (size_t)jj * ldv + off + i;
    const double wr = (tr * ur - ti * ui) + alpha * Vr[o];
    const double wi = (tr * ui + ti * ur) + alpha * Vi[o];
    Wr[o] = wr;
    Wi[o] = wi;
    if (nx) {
        const double nr = ((p[2][0][tx] + p[2][1][tx]) + p[2][2][tx]) + p[2][3][tx];
        const double ni = ((p[3][0][tx] + p[3][1][tx]) + p[3][2][tx]) + p[3][3][tx];
        // H(r + i, r): the diagonal entry (real) for i = 0
        const double hr = Hr[(size_t)r * lda + r + i], hi = (i > 0) ? Hi[(size_t)r * lda + r + i] : 0.0;
        Vr[(size_t)(jj + 1) * ldv + off + i] = hr + nr - wr;   // V(r, jj) = 1: - w(i) conj(1)
        Vi[(size_t)(jj + 1) * ldv + off + i] = hi + ni - wi;
    }
}

// Lower tiles of the trailing block (r0, r0), m x m: IM = 0 updates the real
// plane (diagonal included) by -[Vr Vi Wr Wi][Wr Wi Vr Vi]^T, IM = 1 the
// imaginary plane (strict lower part) by -[Vi -Vr Wi -Wr][Wr Wi Vr Vi]^T,
// over the panel's B columns (rank 4B).
template <int IM>
__global__ __launch_bounds__(256) GEMM_OCC2 void k_her2k(double *__restrict__ P, int lda, int r0, int m,
                                                         const double *__restrict__ Vr, const double *__restrict__ Vi,
                                                         const double *__restrict__ Wr, const double *__restrict__ Wi,
                                                         int ldv, int B)
{
    constexpr int TT = 64;
    extern __shared__ char smraw[];
    double *smem = (double *)smraw;
    int I, J;
    tri_index(blockIdx.x, I, J);
    const int m0 = I * TT, n0 = J * TT;
    // k runs to a multiple of the k-step: entries past rank 4B are zero
    auto fa = [=](int i, int k) -> double {
        if (k >= 4 * B) return 0.0;
        const int g = k / B, kk = k - g * B;
        const double *src;
        double sg = 1.0;
        if (IM == 0) {
            src = (g == 0) ? Vr : (g == 1) ? Vi : (g == 2) ? Wr : Wi;
        } else {
            src = (g == 0) ? Vi : (g == 1) ? Vr : (g == 2) ? Wi : Wr;
            sg = (g & 1) ? -1.0 : 1.0;
        }
        const double x = src[(size_t)kk * ldv + min(i, m - 1)];
        return x * (i < m ? sg : 0.0);
    };
    auto fb = [=](int j, int k) -> double {
        if (k >= 4 * B) return 0.0;
        const int g = k / B, kk = k - g * B;
        const double *src = (g == 0) ? Wr : (g == 1) ? Wi : (g == 2) ? Vr : Vi;
        const double x = src[(size_t)kk * ldv + min(j, m - 1)];
        return x * (j < m ? 1.0 : 0.0);
    };
    gemm::Acc<double, TT, TT> acc;
    acc.zero();
    gemm::kloop<double, TT, TT, false, false>(fa, fb, m0, n0, 0, 4 * B, smem, acc);
    double *A0 = P + (size_t)r0 * lda + r0;
    const bool diag = (I == J);
    auto inside = [=](int i, int j) {
        return m0 + i < m && n0 + j < m && (!diag || (IM ? i > j : i >= j));
    };
    gemm::epilogue_rmw<double, TT, TT>(
        acc, smem,
        [=](int i, int j) -> double { return A0[(size_t)min(n0 + j, m - 1) * lda + min(m0 + i, m - 1)]; },
        [=](int i, int j, double old, double v) {
            if (inside(i, j)) A0[(size_t)(n0 + j) * lda + m0 + i] = old - v;
        });
}

// W = V^H Z of a panel from the GEMM partials P1 = Vr^T [Zr Zi] (S1 parts)
// and P2 = Vi^T [Zr Zi] (S2 parts), each 64 x 2 nev (ld 64):
// Re W = P1[:, :nev] + P2[:, nev:], Im W = P1[:, nev:] - P2[:, :nev]; then
// W2 = T W and B1 = [Re W2, Im W2], B2 = [-Im W2, Re W2] (64 x 2 nev, ld 64),
// so that Z -= Vr B1 + Vi B2 is Z -= V W2 on [Re Z, Im Z].  32 columns per
// workgroup.
__global__ __launch_bounds__(256) void k_h_bt_t(const double *__restrict__ P1, int S1, const double *__restrict__ P2,
                                                int S2, const double *__restrict__ Tr, const double *__restrict__ Ti,
                                                int nev, double *__restrict__ B1, double *__restrict__ B2)
{
    __shared__ double wr[32][65], wi[32][65];
    const int tid = threadIdx.x, j0 = blockIdx.x * 32;
    const size_t N = 2 * (size_t)nev, pst = 64 * N;
    for (int x = tid; x < 64 * 32; x += 256) {
        const int u = x & 63, jl = x >> 6, j = j0 + jl;
        double a = 0.0, b = 0.0;
        if (j < nev) {
            for (int s = 0; s < S1; ++s) {
                a += P1[s * pst + (size_t)j * 64 + u];
                b += P1[s * pst + (size_t)(nev + j) * 64 + u];
            }
            for (int s = 0; s < S2; ++s) {
                a += P2[s * pst + (size_t)(nev + j) * 64 + u];
                b -= P2[s * pst + (size_t)j * 64 + u];
            }
        }
        wr[jl][u] = a;
        wi[jl][u] = b;
    }
    __syncthreads();
    const int k = tid & 63, jg = tid >> 6;
    double accr[8], acci[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) accr[c] = acci[c] = 0.0;
    for (int u = k; u < 64; ++u) {
        const double xr = Tr[(size_t)u * 64 + k], xi = Ti[(size_t)u * 64 + k];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double br = wr[jg + 4 * c][u], bi = wi[jg + 4 * c][u];
            accr[c] += xr * br - xi * bi;
            acci[c] += xr * bi + xi * br;
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int j = j0 + jg + 4 * c;
        if (j >= nev) continue;
        B1[(size_t)j * 64 + k] = accr[c];
        B1[(size_t)(nev + j) * 64 + k] = acci[c];
        B2[(size_t)j * 64 + k] = -acci[c];
        B2[(size_t)(nev + j) * 64 + k] = accr[c];
    }
}

__global__ void k_negate(double *__restrict__ X, size_t count)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) X[i] = -X[i];
}

}  // namespace

namespace skew {

size_t herm_scratch_doubles(int n)
{
    const size_t nt = (size_t)(n + OT - 1) / OT, ntiles = nt * (nt + 1) / 2;
    return ntiles * 128 + nt * nt * 128 + ntiles + nt * 256 + 264;   // Pcol: up to nt strips per block
}

// Panel of columns c0 .. c0 + nb - 1 (nb <= 64) of the Hermitian matrix whose
// lower triangle is in (Hr, Hi) (lda), then the trailing update.  Vr, Vi, Wr,
// Wi: (n - c0 - 1) x 64 (ldv = n - c0 - 1); tau: 128; Tr, Ti: 64 x 64; d, e:
// the tridiagonal matrix; scratch: herm_scratch_doubles(n).
void launch_herm_panel(double *Hr, double *Hi, int lda, int n, int c0, int nb, double *Vr, double *Vi, double *Wr,
                       double *Wi, int ldv, double *tau, double *Tr, double *Ti, double *d, double *e,
                       double *scratch, hipStream_t st)
{
    const size_t ntm = (size_t)(n + OT - 1) / OT, ntt = ntm * (ntm + 1) / 2;
    double *Prow = scratch, *Pcol = Prow + ntt * 128;
    double *Ps = Pcol + ntm * ntm * 128;
    double *Pd = Ps + ntt, *D = Pd + ntm * 256;
    for (int jj = 0; jj < nb; ++jj) {
        const int c = c0 + jj, r = c + 1, m = n - r, off = jj;
        hipLaunchKernelGGL(k_h_col, dim3(1), dim3(CT), 0, st, (const double *)Hr, (const double *)Hi, lda, n, c0, jj,
                           Vr, Vi, Wr, Wi, ldv, tau, d, e);
        const int nt = (int)cdiv(m, OT);
        const int ss = strip_len(nt);
        int nwg = 0;
        for (int s = 0; s * ss < nt; ++s) nwg += nt - s * ss;
        const size_t o = (size_t)jj * ldv + off;
        hipLaunchKernelGGL(k_h_hemv, dim3(nwg), dim3(256), 0, st, (const double *)Hr, (const double *)Hi, lda, r, m,
                           (const double *)(Vr + o), (const double *)(Vi + o), (const double *)Vr,
                           (const double *)Vi, (const double *)Wr, (const double *)Wi, ldv, off, jj, Prow, Pcol, Ps,
                           Pd);
        hipLaunchKernelGGL(k_h_dots, dim3(1), dim3(256), 0, st, (const double *)Pd, nt, (const double *)Ps, nwg, jj,
                           (const double *)tau, D, Tr, Ti);
        hipLaunchKernelGGL(k_h_w, dim3(nt), dim3(256), 0, st, (const double *)Hr, (const double *)Hi, lda, r, m, nt,
                           (const double *)Prow, (const double *)Pcol, (const double *)D, Vr, Vi, Wr, Wi, ldv, off,
                           jj, (const double *)tau, (int)(jj + 1 < nb));
    }
    // trailing update from row and column c0 + nb (the diagonal included)
    const int r0 = c0 + nb, m0 = n - r0;
    if (m0 >= 1) {
        const size_t ro = (size_t)(r0 - (c0 + 1));
        const unsigned nt = cdiv(m0, 64), ntiles = nt * (nt + 1) / 2;
        const size_t shm = gemm::smem_bytes<double, 64, 64>();
        hipLaunchKernelGGL((k_her2k<0>), dim3(ntiles), dim3(256), shm, st, Hr, lda, r0, m0, (const double *)(Vr + ro),
                           (const double *)(Vi + ro), (const double *)(Wr + ro), (const double *)(Wi + ro), ldv, nb);
        hipLaunchKernelGGL((k_her2k<1>), dim3(ntiles), dim3(256), shm, st, Hi, lda, r0, m0, (const double *)(Vr + ro),
                           (const double *)(Vi + ro), (const double *)(Wr + ro), (const double *)(Wi + ro), ldv, nb);
    }
}

// One panel of the back-transformation, rows r0 .. r0 + m - 1 of Z = [Re Z, Im Z]
// (n x 2 nev, ldz): Z <- (I - V T V^H) Z.  P1, P2: tn_parts_max() x 64 x
// 2 nev doubles each; B: 2 x 64 x 2 nev doubles.
void launch_herm_bt(double *Z, int ldz, int r0, int m, int nev, const double *Vr, const double *Vi, const double *Tr,
                    const double *Ti, double *P1, double *P2, double *B, hipStream_t st)
{
    if (m <= 0 || nev <= 0) return;
    const int S1 = launch_gemm_tn_part<double>(Vr, m, Z + r0, ldz, 64, 2 * nev, m, P1, st);
    const int S2 = launch_gemm_tn_part<double>(Vi, m, Z + r0, ldz, 64, 2 * nev, m, P2, st);
    double *B1 = B, *B2 = B + (size_t)64 * 2 * nev;
    hipLaunchKernelGGL(k_h_bt_t, dim3(cdiv(nev, 32)), dim3(256), 0, st, (const double *)P1, S1, (const double *)P2,
                       S2, Tr, Ti, nev, B1, B2);
    launch_gemm_nn<double>(Vr, m, B1, 1, m, 2 * nev, 64, Z + r0, ldz, -1.0, 1, st);
    launch_gemm_nn<double>(Vi, m, B2, 1, m, 2 * nev, 64, Z + r0, ldz, -1.0, 1, st);
}

void launch_negate(double *X, size_t count, hipStream_t st)
{
    if (count == 0) return;
    const size_t g = cdiv(count, 256);
    hipLaunchKernelGGL(k_negate, dim3(g > 2048 ? 2048 : (unsigned)g), dim3(256), 0, st, X, count);
}

}  // namespace skew
