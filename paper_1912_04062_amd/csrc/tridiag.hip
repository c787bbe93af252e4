// Symmetric tridiagonal eigensolver for T = tridiag(alpha, 0, alpha)
// (Algorithm 1, step 2; Lemma 1 turns the skew tridiagonal into this matrix,
// whose off-diagonal is the super-diagonal alpha of the skew one).  With a
// diagonal given, the same kernels solve tridiag(alpha, diag, alpha) (the
// complex Hermitian route's real tridiagonal matrix): the Sturm counts and
// the factorizations take d_i - x, and each vector is normalised as a whole.
//
//   k_bisect   eigenvalues by Sturm-sequence multisection: 16 lanes evaluate
//              the inertia count at 16 interior points of the current
//              interval, which shrinks 17-fold per round (4 bits).  The
//              counts use d_i = -x - alpha_{i-1}^2 / d_{i-1} with tiny pivots
//              replaced by -pivmin.  alpha^2 is staged through LDS in chunks.
//   k_invit    eigenvectors by inverse iteration, one thread per vector, on
//              T - lambda I factored by Gaussian elimination with partial
//              pivoting (U gets a second super-diagonal); factors and
//              iterates live in [i][k] layout so that consecutive vectors are
//              consecutive in memory.  For lambda > 0 the even- and odd-
//              indexed halves of an exact eigenvector have equal norms, so
//              each half is scaled to 1/sqrt(2).
//   k_nullvec  for odd n the exact zero eigenvalue's vector from the two-term
//              recurrence of T q = 0 (odd entries zero), when it applies.
// Orthogonality across close eigenvalues is restored afterwards by a block
// Gram-Schmidt pass in eigenvalue order (host code, using the GEMM kernels).
#include "common.h"
#include "gemm.h"
#include "kernels.h"
#include "small64.h"

namespace {

constexpr int BIS_NS = 16;       // shifts per eigenvalue
constexpr int BIS_CH = 2048;     // alpha^2 chunk staged in LDS

// The kernels below serve one problem (probs null: the problem is `one`,
// blockIdx.x its block index) or a batch: probs[p] for p = 0..cnt-1, where
// block g belongs to the problem p with pre[p] <= g < pre[p + 1] (a prefix
// table of the problems' block counts) as its block g - pre[p].  The same
// code runs either way, so batched results equal single ones bitwise.
__device__ __forceinline__ int find_prob(const int *pre, int cnt, int g)
{
    int lo = 0, hi = cnt;   // pre[lo] <= g < pre[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// A descriptor's pointers as global-address-space pointers (pointers read
// from memory would otherwise compile to flat accesses, which also wait on
// the LDS counter).
template <typename T> using gp = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ gp<T> gptr(T *p) { return (gp<T>)p; }
template <typename T> __device__ __forceinline__ gp<const T> gptr(const T *p) { return (gp<const T>)p; }

// Every field of a descriptor is the same in all lanes of a block: stated to
// the compiler, so that sizes and pointers live in scalar registers (loop
// bounds stay scalar, loads take a scalar base).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T> __device__ __forceinline__ T *uni(T *p)
{
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (T *)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double uni(double d)
{
    const unsigned long long v = __double_as_longlong(d);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// the problem of this block and the block's index within it
__device__ __forceinline__ skew::TriProb tri_prob(const skew::TriProb &one, const skew::TriProb *probs,
                                                  const int *pre, int cnt, int &bx)
{
    bx = blockIdx.x;
    skew::TriProb t = one;
    if (probs) {
        const int p = uni(pre ? find_prob(pre, cnt, bx) : bx);
        bx = pre ? bx - uni(pre[p]) : 0;
        t = probs[p];
    }
    skew::TriProb u;
    u.ab = uni(t.ab);
    u.alpha = uni(t.alpha);
    u.a2 = uni(t.a2);
    u.stats = uni(t.stats);
    u.w = uni(t.w);
    u.U0 = uni(t.U0);
    u.U1 = uni(t.U1);
    u.U2 = uni(t.U2);
    u.Lm = uni(t.Lm);
    u.Y = uni(t.Y);
    u.fac = uni(t.fac);
    u.Q = uni(t.Q);
    u.Sw = uni(t.Sw);
    u.err = uni(t.err);
    u.gcnt = uni(t.gcnt);
    u.diag = uni(t.diag);
    u.shifts = uni(t.shifts);
    u.ctol = uni(t.ctol);
    u.ldab = uni(t.ldab);
    u.n = uni(t.n);
    u.first = uni(t.first);
    u.nev = uni(t.nev);
    u.ldq = uni(t.ldq);
    u.iters = uni(t.iters);
    return u;
}

// One block per problem.  With the band given (Q.ab), alpha is first taken
// from it (alpha_j = -A[j+1, j]; a 1 x 1 problem gets alpha_0 = 0).  Then
// a2[i] = alpha[i]^2 (i < n-1), stats[0] = ||T||_inf, stats[1] = max alpha^2.
__global__ void k_alpha2(skew::TriProb one, const skew::TriProb *__restrict__ probs)
{
    __shared__ double mx[256], mg[256];
    int bx;
    const skew::TriProb Q = tri_prob(one, probs, nullptr, 0, bx);
    const int n = Q.n;
    const gp<double> __restrict__ alpha = gptr(Q.alpha);
    const gp<const double> __restrict__ diag = gptr(Q.diag);
    if (Q.ab) {
        const gp<const double> ab = gptr(Q.ab);
        for (int j = threadIdx.x; j < n - 1; j += 256) alpha[j] = -ab[(size_t)j * Q.ldab + 1];
        if (n == 1 && threadIdx.x == 0) alpha[0] = 0.0;
        __syncthreads();
    }
    const gp<double> __restrict__ a2 = gptr(Q.a2);
    double lm = 0.0, lg = 0.0;
    for (int i = threadIdx.x; i < n - 1; i += 256) {
        double a = alpha[i];
        a2[i] = a * a;
        lm = fmax(lm, a * a);
        if (!diag) {
            double r = fabs(a) + ((i + 1 < n - 1) ? fabs(alpha[i + 1]) : 0.0);
            lg = fmax(lg, r);
            if (i == 0) lg = fmax(lg, fabs(a));
        }
    }
    if (diag)       // row i: |d_i| + |alpha_{i-1}| + |alpha_i|
        for (int i = threadIdx.x; i < n; i += 256)
            lg = fmax(lg, fabs(diag[i]) + ((i > 0) ? fabs(alpha[i - 1]) : 0.0) + ((i < n - 1) ? fabs(alpha[i]) : 0.0));
    mx[threadIdx.x] = lm;
    mg[threadIdx.x] = lg;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + o]);
            mg[threadIdx.x] = fmax(mg[threadIdx.x], mg[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const gp<double> stats = gptr(Q.stats);
        stats[0] = mg[0];
        stats[1] = mx[0];
    }
}

// Inertia count of T - x I (the eigenvalues below x), by all threads of the
// block together: alpha^2 (and the diagonal) staged through LDS in chunks.
__device__ __forceinline__ int sturm_count(double xq, gp<const double> a2, gp<const double> diag, int n,
                                           double pivmin, double *sa, double *sd)
{
    double d = diag ? diag[0] - xq : -xq;
    if (fabs(d) < pivmin) d = -pivmin;
    int cnt = (d < 0.0) ? 1 : 0;
    for (int c0 = 0; c0 < n - 1; c0 += BIS_CH) {
        const int len = min(BIS_CH, n - 1 - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < len; i += 256) {
            sa[i] = a2[c0 + i];
            if (diag) sd[i] = diag[c0 + i + 1];
        }
        __syncthreads();
        if (diag) {
            for (int i = 0; i < len; ++i) {
                d = (sd[i] - xq) - sa[i] * recip(d);
                if (fabs(d) < pivmin) d = -pivmin;
                cnt += (d < 0.0) ? 1 : 0;
            }
        } else {
            for (int i = 0; i < len; ++i) {
                d = -xq - sa[i] * recip(d);
                if (fabs(d) < pivmin) d = -pivmin;
                cnt += (d < 0.0) ? 1 : 0;
            }
        }
    }
    return cnt;
}

// The Gershgorin interval that starts the bisection, and pivmin.
__device__ __forceinline__ void bis_bounds(gp<const double> stats, double &lo, double &hi, double &pivmin)
{
    const double g = stats[0];
    pivmin = 2.2250738585072014e-308 * fmax(1.0, stats[1]);
    const double eps = 2.220446049250313e-16;
    lo = -g * (1.0 + 2.0 * eps) - 2.0 * pivmin;
    hi = g * (1.0 + 2.0 * eps) + 2.0 * pivmin;
}

// Points of the grid pre-pass: one per thread of the bisection launch.
__device__ __forceinline__ int grid_points(int nev) { return 256 * ((nev + (256 / BIS_NS) - 1) / (256 / BIS_NS)); }

// Grid pre-pass of the bisection: the inertia counts at the NP points
// x_t = lo + (t + 1) h, h = (hi - lo) / (NP + 1), of the Gershgorin
// interval, one per thread (the bisection's grid).  Each eigenvalue's
// starting bracket is then the grid interval that holds it, which saves
// the rounds that would narrow the whole interval down to one grid step.
__global__ __launch_bounds__(256) void k_gridcount(skew::TriProb one, const skew::TriProb *__restrict__ probs,
                                                   const int *__restrict__ pre, int cnt)
{
    __shared__ double sa[BIS_CH], sd[BIS_CH];
    int bx;
    const skew::TriProb Q = tri_prob(one, probs, pre, cnt, bx);
    if (!Q.gcnt) return;
    const gp<const double> __restrict__ a2 = gptr(Q.a2);
    const gp<const double> __restrict__ stats = gptr(Q.stats);
    const gp<const double> __restrict__ diag =
        __builtin_amdgcn_readfirstlane((int)(Q.diag != nullptr)) ? gptr(Q.diag) : nullptr;
    const int NP = grid_points(Q.nev);
    double lo, hi, pivmin;
    bis_bounds(stats, lo, hi, pivmin);
    const double h = (hi - lo) / (NP + 1);
    const int t = bx * 256 + threadIdx.x;
    const int c = sturm_count(lo + (t + 1) * h, a2, diag, Q.n, pivmin, sa, sd);
    gptr(Q.gcnt)[t] = c;
}

// 256 threads = 16 eigenvalues x 16 shifts.  Eigenvalue index first + e.
// rounds: for the whole Gershgorin interval; after the grid pre-pass the
// bracket starts (NP + 1) times narrower and takes only the rounds that
// bring it below the same width.
__global__ __launch_bounds__(256) void k_bisect(skew::TriProb one, const skew::TriProb *__restrict__ probs,
                                                const int *__restrict__ pre, int cnt, int rounds)
{
    __shared__ double sa[BIS_CH], sd[BIS_CH];
    int bx;
    const skew::TriProb Q = tri_prob(one, probs, pre, cnt, bx);
    const gp<const double> __restrict__ a2 = gptr(Q.a2);
    const gp<const double> __restrict__ stats = gptr(Q.stats);
    // the diagonal's presence is uniform: a scalar branch
    const gp<const double> __restrict__ diag =
        __builtin_amdgcn_readfirstlane((int)(Q.diag != nullptr)) ? gptr(Q.diag) : nullptr;
    const gp<double> __restrict__ w = gptr(Q.w);
    const int n = Q.n, first = Q.first, count = Q.nev;
    const int q = threadIdx.x & (BIS_NS - 1);
    const int e = bx * (256 / BIS_NS) + threadIdx.x / BIS_NS;
    const bool active = e < count;
    const int idx = first + (active ? e : 0);
    double lo, hi, pivmin;
    bis_bounds(stats, lo, hi, pivmin);
    int nr = rounds;
    if (Q.gcnt) {
        // the grid interval that holds lambda_idx: the first point whose
        // count exceeds idx (the counts grow with x)
        const gp<const int> gc = gptr(Q.gcnt);
        const int NP = grid_points(count);
        int a = 0, b = NP;
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (gc[mid] > idx) b = mid;
            else a = mid + 1;
        }
        const double h = (hi - lo) / (NP + 1);
        const double nlo = (a > 0) ? lo + a * h : lo;          // x_{a-1}
        const double nhi = (a < NP) ? lo + (a + 1) * h : hi;   // x_a
        lo = nlo;
        hi = nhi;
        // rounds until (NP + 1) 17^r reaches 17^rounds
        double f = NP + 1.0, full = 1.0;
        for (int r = 0; r < rounds; ++r) full *= (BIS_NS + 1);
        nr = 0;
        while (nr < rounds && f < full) {
            f *= (BIS_NS + 1);
            ++nr;
        }
    }
    for (int r = 0; r < nr; ++r) {
        const double h = (hi - lo) / (BIS_NS + 1);
        const double xq = lo + (q + 1) * h;
        const int cnt = sturm_count(xq, a2, diag, n, pivmin, sa, sd);
        // lanes with count <= idx have lambda_idx >= x_q
        unsigned long long m = __ballot(cnt <= idx);
        const int sh = (threadIdx.x & 63) & ~(BIS_NS - 1);
        const int qs = __popcll((m >> sh) & ((1ull << BIS_NS) - 1));
        const double nlo = (qs > 0) ? lo + qs * h : lo;
        const double nhi = (qs < BIS_NS) ? lo + (qs + 1) * h : hi;
        lo = nlo;
        hi = nhi;
    }
    if (active && q == 0) {
        // zero diagonal: the requested indices are the upper half of a
        // spectrum symmetric about 0, so lambda >= 0: a final bracket that
        // still holds 0 (the zero matrix, or a split block of odd order)
        // gives exactly 0, which is as close as its midpoint
        double lam = 0.5 * (lo + hi);
        if (!diag) {
            if (lo <= 0.0) lam = 0.0;
            if ((n & 1) && idx == n / 2) lam = 0.0;
        }
        w[e] = lam;
    }
}

__device__ __forceinline__ double hash_uniform(unsigned long long seed, unsigned long long a, unsigned long long b)
{
    unsigned long long z = seed ^ (a * 0x9e3779b97f4a7c15ull) ^ (b * 0xc2b2ae3d27d4eb4full);
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

// Inverse iteration, one thread per vector (one wavefront per workgroup so
// that the vectors spread over as many CUs as possible).  Workspace (each
// n x nev, [i][k] layout, so a wavefront's accesses are contiguous):
// U0, U1, U2 (rows of U; U0 holds the reciprocals of the pivots, which are
// clamped away from 0), Lm (multipliers),
// Sw (row swaps), Y (iterate).  Every pass runs in chunks of IV_CH steps
// whose loads are all issued before the chunk's sequential arithmetic.
// The iterate is normalised on the fly (its norm is accumulated by the
// previous backward pass), the start vector is generated, and the final
// scaling (even and odd halves each to 1/sqrt(2) for lambda > 0) is left to
// the transposition: fac[k] (even rows) and fac[nev + k] (odd rows).
// With shifts given, vector k uses shifts[k] and starts from its current
// values in Y (the polishing step of degenerate clusters, see
// launch_tridiag_polish); otherwise from w[k] and a generated start.
// Convergence: the last iteration's input has unit norm, so its solution's
// norm |y| gives the residual |(T - shift I) y/|y|| = 1/|y| of the returned
// vector; a vector whose residual exceeds ctol ||T|| sets code 8 in *err
// (ctol = 0 makes every vector fail: a test hook of the error path).
constexpr int IV_CH = 32;
constexpr unsigned ERR_INVIT = 8u;

__global__ __launch_bounds__(64) void k_invit(skew::TriProb one, const skew::TriProb *__restrict__ probs,
                                              const int *__restrict__ pre, int cnt)
{
    int bx;
    const skew::TriProb Q = tri_prob(one, probs, pre, cnt, bx);
    const gp<const double> __restrict__ alpha = gptr(Q.alpha);
    const gp<const double> __restrict__ w = gptr(Q.w);
    const gp<const double> __restrict__ stats = gptr(Q.stats);
    const gp<double> __restrict__ U0 = gptr(Q.U0);
    const gp<double> __restrict__ U1 = gptr(Q.U1);
    const gp<double> __restrict__ U2 = gptr(Q.U2);
    const gp<double> __restrict__ Lm = gptr(Q.Lm);
    const gp<unsigned char> __restrict__ Sw = gptr(Q.Sw);
    const gp<double> __restrict__ Y = gptr(Q.Y);
    const gp<double> __restrict__ fac = gptr(Q.fac);
    // presence of shifts and diagonal is uniform: scalar branches
    const gp<const double> __restrict__ shifts =
        __builtin_amdgcn_readfirstlane((int)(Q.shifts != nullptr)) ? gptr(Q.shifts) : nullptr;
    const gp<const double> __restrict__ diag =
        __builtin_amdgcn_readfirstlane((int)(Q.diag != nullptr)) ? gptr(Q.diag) : nullptr;
    unsigned *err = Q.err;
    const double ctol = Q.ctol;
    const int n = Q.n, nev = Q.nev, iters = Q.iters;
    const int k = bx * 64 + threadIdx.x;
    if (k >= nev) return;
    const size_t st = nev;
    const double g = stats[0];
    const double eps = 2.220446049250313e-16;
    const double tiny = eps * (g > 0.0 ? g : 1.0);
    const double lam = w[k];
    // perturb coincident shifts apart (consecutive equal eigenvalues)
    double shift = lam;
    if (shifts) {
        shift = shifts[k];
    } else if (k > 0) {
        int r = 0;
        while (k - r - 1 >= 0 && w[k - r - 1] == lam && r < 64) ++r;
        shift = lam + r * 10.0 * eps * fmax(fabs(lam), tiny);
    }
    auto clampu = [=](double u) { return (fabs(u) < tiny) ? ((u < 0.0) ? -tiny : tiny) : u; };
    // factor T - shift I with partial pivoting (rows i, i+1 at step i)
    {
        double a = diag ? diag[0] - shift : -shift, bb = (n > 1) ? alpha[0] : 0.0, cc = 0.0;
        for (int i0 = 0; i0 + 1 < n; i0 += IV_CH) {
            double al[IV_CH + 1], dl[IV_CH];
#pragma unroll
            for (int j = 0; j <= IV_CH; ++j) {
                const double x = alpha[min(i0 + j, n - 2)];
                al[j] = (i0 + j < n - 1) ? x : 0.0;
            }
#pragma unroll
            for (int j = 0; j < IV_CH; ++j) dl[j] = diag ? diag[min(i0 + j + 1, n - 1)] : 0.0;
#pragma unroll
            for (int j = 0; j < IV_CH; ++j) {
                const int i = i0 + j;
                if (i + 1 >= n) continue;           // predicated (no break: keeps the loop unrolled)
                const double sub = al[j], dn = diag ? dl[j] - shift : -shift, en = al[j + 1];
                // the pivot is clamped away from 0 (the factorization is
                // that of T - shift I perturbed by at most tiny) and stored
                // as its reciprocal
                if (fabs(a) >= fabs(sub)) {
                    const double r = recip(clampu(a));
                    const double l = sub * r;
                    Sw[i * st + k] = 0;
                    Lm[i * st + k] = l;
                    U0[i * st + k] = r; U1[i * st + k] = bb; U2[i * st + k] = cc;
                    a = dn - l * bb; bb = en - l * cc; cc = 0.0;
                } else {
                    const double r = recip(clampu(sub));
                    const double l = a * r;
                    Sw[i * st + k] = 1;
                    Lm[i * st + k] = l;
                    U0[i * st + k] = r; U1[i * st + k] = dn; U2[i * st + k] = en;
                    a = bb - l * dn; bb = cc - l * en; cc = 0.0;
                }
            }
        }
        U0[(size_t)(n - 1) * st + k] = recip(clampu(a));
    }
    // norm of the start vector (generated, or the given one in Y)
    double inv;
    {
        double s = 0.0;
        for (int i = 0; i < n; ++i) {
            const double y = shifts ? Y[(size_t)i * st + k]
                                    : hash_uniform(0x51ab5eedull, (unsigned long long)k, (unsigned long long)i);
            s += y * y;
        }
        inv = 1.0 / sqrt(s);
    }
    double se = 0.0, so = 0.0;
    for (int it = 0; it < iters; ++it) {
        // forward: P, L (row i+1 of the right-hand side enters at step i)
        auto yin = [&](int i, double stored) -> double {
            return (it == 0 && !shifts)
                       ? hash_uniform(0x51ab5eedull, (unsigned long long)k, (unsigned long long)i) * inv
                       : stored * inv;
        };
        double yprev = yin(0, Y[k]);
        for (int i0 = 0; i0 + 1 < n; i0 += IV_CH) {
            double yv[IV_CH], lv[IV_CH];
            unsigned char sv[IV_CH];
#pragma unroll
            for (int j = 0; j < IV_CH; ++j) {
                // unconditional loads at a clamped row: all of the chunk's
                // loads are in flight together (guards become selects)
                const int ic = min(i0 + j, n - 2);
                yv[j] = Y[(size_t)(ic + 1) * st + k];
                lv[j] = Lm[(size_t)ic * st + k];
                sv[j] = Sw[(size_t)ic * st + k];
            }
            __builtin_amdgcn_sched_barrier(0);     // keep the chunk's loads ahead of its arithmetic
#pragma unroll
            for (int j = 0; j < IV_CH; ++j) {
                const int i = i0 + j;
                if (i + 1 >= n) continue;
                double ynext = yin(i + 1, yv[j]);
                double yi = yprev;
                if (sv[j]) { const double tt = yi; yi = ynext; ynext = tt; }
                ynext -= lv[j] * yi;
                Y[i * st + k] = yi;
                yprev = ynext;
            }
        }
        Y[(size_t)(n - 1) * st + k] = yprev;
        // backward: U, accumulating the squared norms of the even and odd rows
        double x1 = 0.0, x2 = 0.0;
        se = 0.0;
        so = 0.0;
        for (int i1 = n - 1; i1 >= 0; i1 -= IV_CH) {
            double rv[IV_CH], u0[IV_CH], u1[IV_CH], u2[IV_CH];
#pragma unroll
            for (int j = 0; j < IV_CH; ++j) {
                const size_t ic = (size_t)max(i1 - j, 0);
                rv[j] = Y[ic * st + k];
                u0[j] = U0[ic * st + k];
                u1[j] = U1[ic * st + k];
                u2[j] = U2[ic * st + k];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < IV_CH; ++j) {
                const int i = i1 - j;
                if (i < 0) continue;
                // U1, U2 of the last rows are never written: they multiply x1 = x2 = 0
                const double xi = (rv[j] - ((i + 1 < n) ? u1[j] : 0.0) * x1 - ((i + 2 < n) ? u2[j] : 0.0) * x2) * u0[j];
                Y[i * st + k] = xi;
                if (i & 1) so += xi * xi;
                else se += xi * xi;
                x2 = x1;
                x1 = xi;
            }
        }
        inv = 1.0 / sqrt(se + so);
    }
    if (err && g > 0.0 && !(sqrt(se + so) * ctol * g >= 1.0)) atomicOr(err, ERR_INVIT);
    // final scaling factors
    double fe, fo;
    if (!diag && lam > 0.0 && se > 0.0 && so > 0.0) {
        fe = sqrt(0.5 / se);
        fo = sqrt(0.5 / so);
    } else {
        fe = fo = 1.0 / sqrt(se + so);
    }
    fac[k] = fe;
    fac[nev + k] = fo;
}

// Odd n, lambda_0 = 0: q_0 = 1, q_{2m+2} = -alpha_{2m} q_{2m} / alpha_{2m+1},
// odd entries 0; used only when every alpha_{2m+1} != 0 (else the inverse
// iteration result stays).  Single thread; writes column 0 of Y ([i][k]).
__global__ void k_nullvec(skew::TriProb one, const skew::TriProb *__restrict__ probs)
{
    int bx;
    const skew::TriProb P = tri_prob(one, probs, nullptr, 0, bx);
    const gp<const double> __restrict__ alpha = gptr(P.alpha);
    const gp<double> __restrict__ Y = gptr(P.Y);
    const gp<double> __restrict__ fac = gptr(P.fac);
    const int n = P.n, nev = P.nev;
    if (threadIdx.x != 0 || bx != 0 || !(n & 1) || P.diag || nev <= 0) return;
    for (int i = 1; i < n - 1; i += 2)
        if (alpha[i] == 0.0) return;
    const size_t st = nev;
    double q = 1.0, s = 1.0;
    Y[0] = 1.0;
    for (int m2 = 0; m2 + 2 < n; m2 += 2) {
        q = -alpha[m2] * q / alpha[m2 + 1];
        if (fabs(q) > 1e150) {
            for (int i = 0; i <= m2; i += 2) Y[i * st] *= 1e-150;
            q *= 1e-150;
            s *= 1e-300;
        }
        Y[(size_t)(m2 + 2) * st] = q;
        s += q * q;
    }
    double ss = 0.0;
    for (int i = 0; i < n; i += 2) ss += Y[i * st] * Y[i * st];
    const double inv = 1.0 / sqrt(ss);
    for (int i = 0; i < n; ++i) Y[i * st] = (i & 1) ? 0.0 : Y[i * st] * inv;
    fac[0] = 1.0;
    fac[nev] = 1.0;
}

// Y ([i][k], n x nev) -> Q (column-major, ldq), row i of column k scaled by
// fac[k] (even i) or fac[nev + k] (odd i)
__global__ void k_transpose(skew::TriProb one, const skew::TriProb *__restrict__ probs, const int *__restrict__ pre,
                            int cnt)
{
    __shared__ double tile[32][33];
    int bx;
    const skew::TriProb P = tri_prob(one, probs, pre, cnt, bx);
    const gp<const double> __restrict__ Y = gptr(P.Y);
    const gp<const double> __restrict__ fac = gptr(P.fac);
    const gp<double> __restrict__ Q = gptr(P.Q);
    const int n = P.n, nev = P.nev, ldq = P.ldq;
    const int nbx = (nev + 31) / 32;   // blocks: nbx columns of tiles by row tiles
    const int k0 = (bx % nbx) * 32, i0 = (bx / nbx) * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        int i = i0 + r, k = k0 + tx;
        tile[r][tx] = (i < n && k < nev) ? Y[(size_t)i * nev + k] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        int k = k0 + r, i = i0 + tx;
        if (i < n && k < nev) Q[(size_t)k * ldq + i] = tile[tx][r] * fac[(i & 1) ? nev + k : k];
    }
}

// *flag |= 2 when two consecutive values of w (ascending) are closer than
// tol * stats[0]: a degenerate cluster (the batched form then solves the
// problem again on its own, where such clusters are polished)
__global__ void k_degenerate(const double *__restrict__ w, int m, const double *__restrict__ stats, double tol,
                             unsigned *flag)
{
    const double lim = tol * stats[0];
    bool d = false;
    for (int k = blockIdx.x * 256 + threadIdx.x; k + 1 < m; k += gridDim.x * 256)
        if (w[k + 1] - w[k] <= lim) d = true;
    if (__any(d) && (threadIdx.x & 63) == 0) atomicOr(flag, 2u);
}

// Q (column-major, ldq, n x m) -> Y ([i][k] layout, n x m)
__global__ void k_transpose_in(const double *__restrict__ Q, int ldq, int n, int m, double *__restrict__ Y)
{
    __shared__ double tile[32][33];
    const int k0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        int k = k0 + r, i = i0 + tx;
        tile[r][tx] = (i < n && k < m) ? Q[(size_t)k * ldq + i] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        int i = i0 + r, k = k0 + tx;
        if (i < n && k < m) Y[(size_t)i * m + k] = tile[tx][r];
    }
}

// Cholesky of G = sum of partials (NB x NB, NB <= 64) and R^{-1} (upper);
// a non-positive pivot is replaced by 1e-300.  When G = I + E with
// max |E_ij| <= 1e-8 (a block already orthonormal to that level) R^{-1} is
// taken to first order, I - diag(E)/2 - strict upper(E); the neglected terms
// are O(|E|^2) <= 1e-16.
__global__ __launch_bounds__(256) void k_chol_inv(const double *__restrict__ Gp, int nparts, int NB,
                                                  double *__restrict__ Rinv)
{
    __shared__ double G[64 * 65], X[64 * 65], part[4][64];
    __shared__ __attribute__((aligned(16))) double buf[320];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    double emax = 0.0;
    {
        double acc[16];
        sum_partials_2d(Gp, nparts, (size_t)NB * NB,
                        [=](int i, int j) -> int { return (i < NB && j < NB) ? j * NB + i : -1; }, acc);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = ty + 4 * q;
            G[tx * 65 + j] = acc[q];   // G[i][j]
            if (tx < NB && j < NB) emax = fmax(emax, fabs(acc[q] - ((tx == j) ? 1.0 : 0.0)));
        }
    }
    part[ty][tx] = wave_max(emax);
    __syncthreads();
    if (fmax(fmax(part[0][0], part[1][0]), fmax(part[2][0], part[3][0])) <= 1e-8) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = ty + 4 * q;
            if (tx < NB && j < NB) {
                const double e = G[tx * 65 + j] - ((tx == j) ? 1.0 : 0.0);
                Rinv[(size_t)j * NB + tx] = (tx == j) ? 1.0 - 0.5 * e : ((tx < j) ? -e : 0.0);
            }
        }
        return;
    }
    __syncthreads();
    chol_inv64(G, X, NB, true, 0.0, 0.0, buf);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int j = ty + 4 * q;
        if (tx < NB && j < NB) Rinv[(size_t)j * NB + tx] = (tx <= j) ? X[tx * 65 + j] : 0.0;   // column-major
    }
}

}  // namespace

namespace skew {

int tri_bisect_groups(int nev) { return nev > 0 ? (int)cdiv(nev, 256 / BIS_NS) : 0; }
int tri_invit_groups(int nev) { return nev > 0 ? (int)cdiv(nev, 64) : 0; }
int tri_transpose_groups(int n, int nev) { return (nev > 0 && n > 0) ? (int)(cdiv(nev, 32) * cdiv(n, 32)) : 0; }

constexpr int BIS_ROUNDS = 14;   // 17^14 > 2^57

static TriProb tri_one(const double *alpha, int n, int nev, const double *w, const double *stats)
{
    TriProb t{};
    t.alpha = const_cast<double *>(alpha);
    t.n = n;
    t.first = n / 2;
    t.nev = nev;
    t.w = const_cast<double *>(w);
    t.stats = const_cast<double *>(stats);
    return t;
}

int tri_grid_points(int nev) { return 256 * tri_bisect_groups(nev); }

void launch_tridiag_eigvals(const double *alpha, int n, int first, int count, double *a2, double *stats,
                            double *w, hipStream_t st, const double *diag, int *gcnt)
{
    if (count <= 0) return;
    TriProb t = tri_one(alpha, n, count, w, stats);
    t.first = first;
    t.a2 = a2;
    t.diag = diag;
    t.gcnt = gcnt;
    hipLaunchKernelGGL(k_alpha2, dim3(1), dim3(256), 0, st, t, (const TriProb *)nullptr);
    if (gcnt)
        hipLaunchKernelGGL(k_gridcount, dim3(tri_bisect_groups(count)), dim3(256), 0, st, t,
                           (const TriProb *)nullptr, (const int *)nullptr, 0);
    hipLaunchKernelGGL(k_bisect, dim3(tri_bisect_groups(count)), dim3(256), 0, st, t, (const TriProb *)nullptr,
                       (const int *)nullptr, 0, BIS_ROUNDS);
}

void launch_tridiag_eigvecs(const double *alpha, int n, int nev, const double *w, const double *stats,
                            double *U0, double *U1, double *U2, double *Lm, unsigned char *Sw, double *Y,
                            double *fac, double *Q, int ldq, double ctol, unsigned *err, hipStream_t st,
                            const double *diag)
{
    if (nev <= 0) return;
    TriProb t = tri_one(alpha, n, nev, w, stats);
    t.U0 = U0;
    t.U1 = U1;
    t.U2 = U2;
    t.Lm = Lm;
    t.Sw = Sw;
    t.Y = Y;
    t.fac = fac;
    t.Q = Q;
    t.ldq = ldq;
    t.ctol = ctol;
    t.err = err;
    t.diag = diag;
    t.iters = 2;
    hipLaunchKernelGGL(k_invit, dim3(tri_invit_groups(nev)), dim3(64), 0, st, t, (const TriProb *)nullptr,
                       (const int *)nullptr, 0);
    if ((n & 1) && !diag) hipLaunchKernelGGL(k_nullvec, dim3(1), dim3(64), 0, st, t, (const TriProb *)nullptr);
    hipLaunchKernelGGL(k_transpose, dim3(tri_transpose_groups(n, nev)), dim3(32, 8), 0, st, t,
                       (const TriProb *)nullptr, (const int *)nullptr, 0);
}

// One more inverse-iteration step for the columns Q[:, 0..m) (eigenvalues
// w[0..m), shifts[0..m)) from their current values: factor T - shifts[k] I,
// solve, scale the halves, write back.  The workspace is that of
// launch_tridiag_eigvecs, used with m in place of nev.
void launch_tridiag_polish(const double *alpha, int n, int m, const double *w, const double *shifts,
                           const double *stats, double *U0, double *U1, double *U2, double *Lm, unsigned char *Sw,
                           double *Y, double *fac, double *Q, int ldq, hipStream_t st, const double *diag)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_transpose_in, dim3(cdiv(m, 32), cdiv(n, 32)), dim3(32, 8), 0, st, (const double *)Q, ldq, n,
                       m, Y);
    TriProb t = tri_one(alpha, n, m, w, stats);
    t.U0 = U0;
    t.U1 = U1;
    t.U2 = U2;
    t.Lm = Lm;
    t.Sw = Sw;
    t.Y = Y;
    t.fac = fac;
    t.Q = Q;
    t.ldq = ldq;
    t.ctol = 1e300;
    t.err = nullptr;
    t.shifts = shifts;
    t.diag = diag;
    t.iters = 1;
    hipLaunchKernelGGL(k_invit, dim3(tri_invit_groups(m)), dim3(64), 0, st, t, (const TriProb *)nullptr,
                       (const int *)nullptr, 0);
    hipLaunchKernelGGL(k_transpose, dim3(tri_transpose_groups(n, m)), dim3(32, 8), 0, st, t,
                       (const TriProb *)nullptr, (const int *)nullptr, 0);
}

void launch_tridiag_batched(const TriProb *probs, const int *pre, int cnt, const int tot[3], hipStream_t st)
{
    if (cnt <= 0) return;
    const TriProb none{};
    hipLaunchKernelGGL(k_alpha2, dim3(cnt), dim3(256), 0, st, none, probs);
    if (tot[0] > 0) {
        hipLaunchKernelGGL(k_gridcount, dim3(tot[0]), dim3(256), 0, st, none, probs, pre, cnt);
        hipLaunchKernelGGL(k_bisect, dim3(tot[0]), dim3(256), 0, st, none, probs, pre, cnt, BIS_ROUNDS);
    }
    if (tot[1] > 0)
        hipLaunchKernelGGL(k_invit, dim3(tot[1]), dim3(64), 0, st, none, probs, pre + (cnt + 1), cnt);
    hipLaunchKernelGGL(k_nullvec, dim3(cnt), dim3(64), 0, st, none, probs);
    if (tot[2] > 0)
        hipLaunchKernelGGL(k_transpose, dim3(tot[2]), dim3(32, 8), 0, st, none, probs, pre + 2 * (cnt + 1), cnt);
}

void launch_degenerate_check(const double *w, int m, const double *stats, double tol, unsigned *flag,
                             hipStream_t st)
{
    if (m < 2) return;
    hipLaunchKernelGGL(k_degenerate, dim3(cdiv(m, 256) > 64 ? 64 : cdiv(m, 256)), dim3(256), 0, st, w, m, stats, tol,
                       flag);
}

void launch_chol_inv(const double *Gp, int nparts, int NB, double *Rinv, hipStream_t st)
{
    hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(256), 0, st, Gp, nparts, NB, Rinv);
}

}  // namespace skew
