// Band-to-tridiagonal reduction of a skew-symmetric band matrix by bulge
// chasing (Section 2.3.2, last part: pipelined bulge chasing; the diagonal
// blocks get the skew rank-2 update A <- A - v u^T + u v^T after a skew
// matrix-vector product).
//
// Storage: lower band, ab[d + j*ldab] = A[j+d, j] for d = 0..2b (fill-in
// reaches d = 2b-1; d = 0 is the zero diagonal).
//
// Sweep s (s = 0..n-3) removes column s below the sub-diagonal.  Step k of
// sweep s uses the reflector H = I - tau v v^T on rows/columns
// R_k = [lo, hi] (lo = s+1+k*b, hi = min(lo+b-1, n-1)) built from column
// c (c = s for k = 0, c = lo-b otherwise), and applies it
//   from the left   to column c (which becomes beta e1) and, for k > 0, to the
//                   block A[R_k, c+1..lo-1];
//   on both sides   to the skew diagonal block A[R_k, R_k]:
//                   y = A v, w = tau y, A <- A + v w^T - w v^T;
//   from the right  to A[hi+1..hi+b, R_k] (this creates the next bulge).
// The reflector of step k+1 comes from column lo of that bulge.
//
// Pipelining: sweep s+1 may run step k once sweep s has completed step k+2
// (or all its steps); this orders every pair of steps that touch a common
// entry.  Sweeps are dealt round-robin to the workgroups of a cooperative
// launch; per-sweep progress counters carry the dependency (agent-scope
// release/acquire), and every wait is bounded.
//
// Each reflector is written, for the back-transformation, into the group of
// nb2 consecutive sweeps at the same step k: V2[g][col][0..b) with
// g = goff[s / nb2] + k, col = s % nb2, and tau2[g][col].
#include "common.h"
#include "kernels.h"

namespace {

constexpr int CH_LD = 65;

__device__ __forceinline__ int nsteps_of(int n, int b, int s) { return 1 + (n - 2 - s) / b; }

// The below block of step k, A[R_{k+1}, R_k], is exactly the next step's
// pivot column (its column 0) and left block (columns 1..b-1), and no other
// sweep writes it between the two steps (sweep s-1 is then at steps >= k+3,
// which start at row s + (k+3) b).  It therefore stays in LDS (two buffers,
// alternating), the next reflector is computed from it before waiting on the
// previous sweep, and only the diagonal block and the new below block are
// loaded after the wait.
__global__ __launch_bounds__(256) void k_bulge_chase(double *__restrict__ ab, int ldab, int n, int b,
                                                     int nb2, double *__restrict__ V2,
                                                     double *__restrict__ tau2,
                                                     const int *__restrict__ goff,
                                                     unsigned *progress, unsigned *err)
{
    __shared__ double v[64], wv[64], dots[64], y2[64];
    __shared__ double dia[64 * CH_LD];
    __shared__ double bw[2][64 * CH_LD];
    __shared__ double scal[2];
    __shared__ int abort_flag;
    const int tid = threadIdx.x;
    if (tid == 0) abort_flag = 0;
    __syncthreads();

    // Householder reflector of x (L entries, lane i holds x_i) by wavefront 0;
    // writes v, scal and the reduced column back to the band.
    auto reflect = [&](double xi, int L, int c, int lo) {
        double sq = (tid >= 1 && tid < L) ? xi * xi : 0.0;
        sq = wave_sum(sq);
        const double x0 = __shfl(xi, 0, 64);
        double t = 0.0, beta = x0, scale = 0.0;
        if (sq != 0.0) {
            const double nrm = sqrt(x0 * x0 + sq);
            beta = (x0 >= 0.0) ? -nrm : nrm;
            t = (beta - x0) / beta;
            scale = 1.0 / (x0 - beta);
        }
        v[tid] = (tid == 0) ? 1.0 : ((tid < L) ? xi * scale : 0.0);
        if (tid == 0) { scal[0] = t; scal[1] = beta; }
        if (tid < L) st_coh(&ab[(size_t)c * ldab + (lo + tid - c)], (tid == 0) ? beta : 0.0);
    };

    for (int s = blockIdx.x; s < n - 2; s += gridDim.x) {
        const int nst = nsteps_of(n, b, s);
        const int nprev = (s > 0) ? nsteps_of(n, b, s - 1) : 0;
        const int sig = s / nb2, col = s % nb2;
        int cur = 0;                              // buffer holding the previous below block
        for (int k = 0; k < nst; ++k) {
            const int lo = s + 1 + k * b;
            const int c = (k == 0) ? s : lo - b;
            const int hi = min(lo + b - 1, n - 1);
            const int L = hi - lo + 1;
            const int bhi = min(hi + b, n - 1);
            const int L2 = bhi - hi;
            const int nlc = lo - c - 1;           // 0 for k = 0, b - 1 otherwise
            const double *lb = bw[cur];           // previous below block: rows R_k, cols R_{k-1}
            double *nb = bw[cur ^ 1];
            // reflector from the carried pivot column (before the wait)
            if (k > 0 && tid < 64) reflect((tid < L) ? lb[tid * CH_LD] : 0.0, L, c, lo);
            if (s > 0) {
                if (tid == 0) {
                    const unsigned need = (unsigned)min(k + 3, nprev);
                    unsigned spins = 0;
                    while (ld_relaxed(&progress[s - 1]) < need) {
                        __builtin_amdgcn_s_sleep(1);
                        if (++spins > SKEW_SPIN_LIMIT) {
                            atomicOr(err, 2u);
                            abort_flag = 1;
                            break;
                        }
                    }
                }
                __syncthreads();
                if (abort_flag) return;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
            // diagonal and new below block (all loads issued before use)
            {
                const int nd = L * L, nbn = L2 * L;
                double vd[16], vb[16];
                double x0v = 0.0;
                if (k == 0 && tid < 64 && tid < L) x0v = ld_coh(&ab[(size_t)c * ldab + (lo + tid - c)]);
#pragma unroll
                for (int p = 0; p < 16; ++p) {
                    const int e = tid + 256 * p;
                    vd[p] = 0.0;
                    vb[p] = 0.0;
                    if (e < nd) {
                        const int il = e % L, jl = e / L;
                        if (il > jl) vd[p] = ld_coh(&ab[(size_t)(lo + jl) * ldab + (il - jl)]);
                    }
                    if (e < nbn) {
                        const int il = e % L2, jl = e / L2;
                        const int i = hi + 1 + il, j = lo + jl;
                        vb[p] = ld_coh(&ab[(size_t)j * ldab + (i - j)]);
                    }
                }
                if (k == 0 && tid < 64) reflect(x0v, L, c, lo);
#pragma unroll
                for (int p = 0; p < 16; ++p) {
                    const int e = tid + 256 * p;
                    if (e < nd) {
                        const int il = e % L, jl = e / L;
                        if (il > jl) {
                            dia[il * CH_LD + jl] = vd[p];
                            dia[jl * CH_LD + il] = -vd[p];
                        } else if (il == jl) {
                            dia[il * CH_LD + il] = 0.0;
                        }
                    }
                    if (e < nbn) nb[(e % L2) * CH_LD + e / L2] = vb[p];
                }
            }
            __syncthreads();
            const double t = scal[0];
            // ---- products with v
            if (tid < 64) {
                if (tid < nlc) {                  // left block = columns 1.. of the carried block
                    double s2 = 0.0;
                    for (int il = 0; il < L; ++il) s2 += v[il] * lb[il * CH_LD + 1 + tid];
                    dots[tid] = t * s2;
                }
            } else if (tid < 128) {
                const int il = tid - 64;
                if (il < L) {
                    double s2 = 0.0;
                    for (int jl = 0; jl < L; ++jl) s2 += dia[il * CH_LD + jl] * v[jl];
                    wv[il] = t * s2;
                }
            } else if (tid < 192) {
                const int il = tid - 128;
                if (il < L2) {
                    double s2 = 0.0;
                    for (int jl = 0; jl < L; ++jl) s2 += nb[il * CH_LD + jl] * v[jl];
                    y2[il] = t * s2;
                }
            }
            __syncthreads();
            // ---- updates, written back (the new below block also stays in LDS)
            for (int e = tid; e < L * nlc; e += 256) {
                const int il = e % L, jl = e / L;
                const int j = c + 1 + jl;
                st_coh(&ab[(size_t)j * ldab + (lo + il - j)], lb[il * CH_LD + 1 + jl] - v[il] * dots[jl]);
            }
            for (int e = tid; e < L * L; e += 256) {
                const int il = e % L, jl = e / L;
                if (il > jl)
                    st_coh(&ab[(size_t)(lo + jl) * ldab + (il - jl)],
                           dia[il * CH_LD + jl] + v[il] * wv[jl] - wv[il] * v[jl]);
            }
            for (int e = tid; e < L2 * L; e += 256) {
                const int il = e % L2, jl = e / L2;
                const int i = hi + 1 + il, j = lo + jl;
                const double val = nb[il * CH_LD + jl] - y2[il] * v[jl];
                nb[il * CH_LD + jl] = val;
                st_coh(&ab[(size_t)j * ldab + (i - j)], val);
            }
            // ---- reflector for the back-transformation
            {
                const size_t g = (size_t)goff[sig] + k;
                if (tid < b) V2[(g * nb2 + col) * b + tid] = (tid < L) ? v[tid] : 0.0;
                if (tid == 0) tau2[g * nb2 + col] = t;
            }
            wg_publish();
            if (tid == 0) st_relaxed(&progress[s], (unsigned)(k + 1));
            cur ^= 1;
        }
    }
}

__global__ void k_alpha(const double *__restrict__ ab, int ldab, int n, double *__restrict__ alpha)
{
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n - 1) alpha[j] = -ab[(size_t)j * ldab + 1];
}

}  // namespace

namespace skew {

int chase_ngroups(int n, int b, int nb2, int *goff_host)
{
    int nsw = n - 2;
    if (nsw <= 0) return 0;
    int nsig = (nsw + nb2 - 1) / nb2;
    int tot = 0;
    for (int sg = 0; sg < nsig; ++sg) {
        if (goff_host) goff_host[sg] = tot;
        tot += 1 + (n - 2 - sg * nb2) / b;
    }
    if (goff_host) goff_host[nsig] = tot;
    return tot;
}

// Workgroups of the cooperative bulge-chase launch: enough for the sweeps
// that can be in flight at once (a sweep of n/b steps starts every third
// step of its predecessor), never more than the device holds.
int chase_workgroups(int n, int b)
{
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    int occ = 1;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_bulge_chase, 256, 0);
    if (occ < 1) occ = 1;
    int G = ncu * occ;
    const int inflight = (n / (b > 0 ? b : 1)) / 3 + 16;
    if (G > inflight) G = inflight;
    if (G > n - 2) G = n - 2;
    if (G < 1) G = 1;
    return G;
}

hipError_t launch_chase(double *ab, int ldab, int n, int b, int nb2, double *V2, double *tau2,
                        const int *goff, unsigned *progress, unsigned *err, double *alpha, hipStream_t st)
{
    if (n >= 3) {
        int G = chase_workgroups(n, b);
        void *args[] = {&ab, &ldab, &n, &b, &nb2, &V2, &tau2, &goff, &progress, &err};
        hipError_t e = hipLaunchCooperativeKernel((const void *)k_bulge_chase, dim3(G), dim3(256), args, 0, st);
        if (e != hipSuccess) return e;
    }
    if (n >= 2) hipLaunchKernelGGL(k_alpha, dim3(cdiv(n, 256)), dim3(256), 0, st, (const double *)ab, ldab, n, alpha);
    return hipGetLastError();
}

}  // namespace skew
